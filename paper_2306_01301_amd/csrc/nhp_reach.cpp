// nhp_reach.cpp -- the reachability entry points of include/nhp.h (App. C):
// a reachability state on a plan's tables and stream, its workspace layout
// and the launch sequence (render bits, R_0, n cycles, extract).
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "nhp_internal.h"

struct nhp_reach {
  nhp_plan* plan = nullptr;
  uint32_t max_cycles = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool own_ws = false;
  nhp::ReachDev r{};
  bool has_hard = false;
  uint32_t n_levels = 0;  // level volumes holding results (0: no sweep yet)
  // the cycles of a multi-cycle sweep, captured as one graph once the same
  // cycle count is asked for twice in a row (a count used once is launched
  // directly: capture and instantiation cost more than the launches)
  hipGraphExec_t cycles = nullptr;
  uint32_t cycles_n = 0;
  uint32_t last_n = 0;  // cycle count of the previous multi-cycle sweep
  bool graph_failed = false;
};

namespace {

#define HIP_TRY(call, what)                                                               \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return nhp::set_error(NHP_EHIP, "%s: %s", what, hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct ReachLayout {
  size_t hard, levels, img, extract, total;
};

ReachLayout reach_layout(const nhp_params& p, uint32_t max_cycles) {
  ReachLayout l{};
  const size_t vol = (size_t)p.nx * p.nx * p.ntheta / 8;  // bytes of one bit volume
  size_t o = 0;
  l.hard = o;
  o = align256(o + vol);
  l.levels = o;
  o = align256(o + vol * (max_cycles + 1));
  l.img = o;
  o = align256(o + (size_t)p.nx * p.nx / 8);
  l.extract = o;
  o = align256(o + (nhp::kExHeader + (size_t)nhp::kReachMaxSteps * nhp::kExStepWords) * 4);
  l.total = o;
  return l;
}

int check_reach_params(const nhp_params* p, uint32_t max_cycles) {
  if (!p) return nhp::set_error(NHP_EINVAL, "params is NULL");
  if (p->nx % 32 != 0 || p->nx < 32 || p->nx > (uint32_t)nhp::kReachMaxN)
    return nhp::set_error(NHP_EINVAL, "reachability needs nx a multiple of 32 in [32, %d] (got %u)", nhp::kReachMaxN,
                          p->nx);
  if (p->ntheta > (uint32_t)nhp::kReachMaxL)
    return nhp::set_error(NHP_EINVAL, "reachability needs ntheta <= %d (got %u)", nhp::kReachMaxL, p->ntheta);
  if (max_cycles < 1 || max_cycles > nhp::kReachMaxCycles)
    return nhp::set_error(NHP_EINVAL, "max_cycles must be 1..%u", nhp::kReachMaxCycles);
  return NHP_OK;
}

int check_reach(const nhp_reach* r) {
  if (!r) return nhp::set_error(NHP_EINVAL, "reach is NULL");
  return NHP_OK;
}

}  // namespace

extern "C" {

size_t reach_workspace_bytes(const nhp_params* params, uint32_t max_cycles) {
  if (check_reach_params(params, max_cycles)) return 0;
  return reach_layout(*params, max_cycles).total;
}

int reach_create(nhp_plan* plan, uint32_t max_cycles, void* d_workspace, size_t workspace_bytes, nhp_reach** out) {
  if (!plan || !out) return nhp::set_error(NHP_EINVAL, "plan or out is NULL");
  *out = nullptr;
  int rc = check_reach_params(&plan->p, max_cycles);
  if (rc) return rc;
  const ReachLayout l = reach_layout(plan->p, max_cycles);
  HIP_TRY(nhp::prepare_reach_kernels(), "reach kernel set-up");
  nhp_reach* r = new (std::nothrow) nhp_reach;
  if (!r) return nhp::set_error(NHP_ENOMEM, "host allocation");
  r->plan = plan;
  r->max_cycles = max_cycles;
  if (d_workspace) {
    if (workspace_bytes < l.total) {
      delete r;
      return nhp::set_error(NHP_EINVAL, "workspace of %zu bytes, %zu needed", workspace_bytes, l.total);
    }
    if (reinterpret_cast<uintptr_t>(d_workspace) % 256) {
      delete r;
      return nhp::set_error(NHP_EINVAL, "workspace must be 256-byte aligned");
    }
    r->ws = d_workspace;
  } else {
    const hipError_t e = hipMalloc(&r->ws, l.total);
    if (e != hipSuccess) {
      delete r;
      return nhp::set_error(NHP_ENOMEM, "hipMalloc of %zu bytes: %s", l.total, hipGetErrorString(e));
    }
    r->own_ws = true;
  }
  r->ws_bytes = l.total;
  char* base = static_cast<char*>(r->ws);
  nhp::ReachDev& d = r->r;
  d.N = (int)plan->p.nx;
  d.L = (int)plan->p.ntheta;
  d.W = d.N / 32;
  d.turn_off = plan->d.turn_off;
  d.skew = plan->d.skew;
  d.family = plan->d.family;
  d.fwd = plan->d.fwd;
  d.taps = plan->d.taps;
  d.hard = reinterpret_cast<uint32_t*>(base + l.hard);
  d.levels = reinterpret_cast<uint32_t*>(base + l.levels);
  d.img = reinterpret_cast<uint32_t*>(base + l.img);
  d.extract = reinterpret_cast<uint32_t*>(base + l.extract);
  d.vol_words = (size_t)d.N * d.N * d.L / 32;
  *out = r;
  return nhp::clear_error();
}

int reach_destroy(nhp_reach* r) {
  if (!r) return nhp::clear_error();
  (void)hipStreamSynchronize(r->plan->stream);
  if (r->cycles) (void)hipGraphExecDestroy(r->cycles);
  if (r->own_ws && r->ws) (void)hipFree(r->ws);
  delete r;
  return nhp::clear_error();
}

int reach_render(nhp_reach* r, const uint8_t* d_image, int32_t front, int32_t rear, int32_t half_width) {
  int rc = check_reach(r);
  if (rc) return rc;
  if (!d_image) return nhp::set_error(NHP_EINVAL, "image is NULL");
  rc = nhp::upload_taps(r->plan, front, rear, half_width);
  if (rc) return rc;
  HIP_TRY(nhp::launch_reach_render(r->r, d_image, 2 * half_width + 1, front + rear + 1, r->plan->stream),
          "reach_render launch");
  r->has_hard = true;
  r->n_levels = 0;
  return nhp::clear_error();
}

int reach_set_cspace(nhp_reach* r, const uint8_t* d_codes) {
  int rc = check_reach(r);
  if (rc) return rc;
  if (!d_codes) return nhp::set_error(NHP_EINVAL, "codes is NULL");
  HIP_TRY(nhp::launch_reach_pack(r->r, d_codes, r->plan->stream), "reach_set_cspace launch");
  r->has_hard = true;
  r->n_levels = 0;
  return nhp::clear_error();
}

// The launches of n cycles captured once (they depend only on the state's
// buffers); on any capture failure the eager launches are used from then on.
static hipGraphExec_t capture_cycles(nhp_reach* r, uint32_t n) {
  const nhp_params& p = r->plan->p;
  hipStream_t cs = nullptr;
  hipGraph_t g = nullptr;
  hipGraphExec_t exec = nullptr;
  bool ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess &&
            hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    for (uint32_t m = 0; m < n; m++)
      ok = ok && nhp::launch_reach_cycle(r->r, p.schedule, (int)p.n_schedule, m, cs) == hipSuccess;
    ok = (hipStreamEndCapture(cs, &g) == hipSuccess) && ok && g != nullptr;
  }
  if (ok) ok = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess;
  if (g) (void)hipGraphDestroy(g);
  if (cs) (void)hipStreamDestroy(cs);
  if (!ok) {
    exec = nullptr;
    r->graph_failed = true;
    (void)hipGetLastError();  // clear a sticky capture error
  }
  return exec;
}

int reach_sweep(nhp_reach* r, uint32_t si, uint32_t sj, uint32_t st, uint32_t n_cycles) {
  int rc = check_reach(r);
  if (rc) return rc;
  if (!r->has_hard) return nhp::set_error(NHP_ESTATE, "reach_sweep before reach_render/reach_set_cspace");
  const nhp_params& p = r->plan->p;
  if (si >= p.nx || sj >= p.nx || st >= p.ntheta) return nhp::set_error(NHP_EINVAL, "start outside the grid");
  if (n_cycles > r->max_cycles)
    return nhp::set_error(NHP_EINVAL, "%u cycles, the state keeps %u", n_cycles, r->max_cycles);
  const size_t idx = ((size_t)st * p.nx + sj) * p.nx + si;
  uint32_t word = 0;
  hipStream_t s = r->plan->stream;
  HIP_TRY(hipMemcpyAsync(&word, r->r.hard + idx / 32, 4, hipMemcpyDeviceToHost, s), "start check");
  HIP_TRY(hipStreamSynchronize(s), "start check");
  if ((word >> (idx % 32)) & 1u) return nhp::set_error(NHP_ESTART, "start pose (%u, %u, %u) is in collision", si, sj, st);
  HIP_TRY(nhp::launch_reach_start(r->r, (uint32_t)idx, s), "reach start launch");
  const bool repeated = n_cycles > 1 && n_cycles == r->last_n;
  if (n_cycles > 1) r->last_n = n_cycles;
  if (repeated && !r->graph_failed && (!r->cycles || r->cycles_n != n_cycles)) {
    if (r->cycles) (void)hipGraphExecDestroy(r->cycles);
    r->cycles = capture_cycles(r, n_cycles);
    r->cycles_n = r->cycles ? n_cycles : 0;
  }
  if (n_cycles > 1 && r->cycles && r->cycles_n == n_cycles) {
    HIP_TRY(hipGraphLaunch(r->cycles, s), "reach cycles graph launch");
  } else {
    for (uint32_t m = 0; m < n_cycles; m++)
      HIP_TRY(nhp::launch_reach_cycle(r->r, p.schedule, (int)p.n_schedule, m, s), "reach cycle launch");
  }
  r->n_levels = n_cycles + 1;
  return nhp::clear_error();
}

int reach_extract(nhp_reach* r, uint32_t gi, uint32_t gj, uint32_t gt, uint32_t radius, nhp_step* h_steps,
                  uint32_t cap, uint32_t* n_steps, uint32_t* best_ijt, uint32_t* level) {
  int rc = check_reach(r);
  if (rc) return rc;
  if (!r->n_levels) return nhp::set_error(NHP_ESTATE, "reach_extract before reach_sweep");
  const nhp_params& p = r->plan->p;
  if (gi >= p.nx || gj >= p.nx || gt >= p.ntheta) return nhp::set_error(NHP_EINVAL, "goal outside the grid");
  if (radius > (uint32_t)nhp::kMaxRadius) return nhp::set_error(NHP_EINVAL, "radius must be <= %d", nhp::kMaxRadius);
  if (!n_steps || (cap > 0 && !h_steps)) return nhp::set_error(NHP_EINVAL, "output pointers are NULL");
  nhp::ReachExArgs x{};
  x.d = r->plan->d;
  x.hard = r->r.hard;
  x.levels = r->r.levels;
  x.vol_words = r->r.vol_words;
  x.W = r->r.W;
  x.n_levels = (int)r->n_levels;
  x.gi = gi;
  x.gj = gj;
  x.gt = gt;
  x.radius = (int)radius;
  x.out = r->r.extract;
  hipStream_t s = r->plan->stream;
  HIP_TRY(nhp::launch_reach_extract(x, s), "reach extract launch");
  uint32_t head[nhp::kExHeader];
  HIP_TRY(hipMemcpyAsync(head, x.out, sizeof(head), hipMemcpyDeviceToHost, s), "extract copy");
  HIP_TRY(hipStreamSynchronize(s), "extract copy");
  const int status = -(int)head[0];
  *n_steps = head[1];
  if (status == NHP_EUNREACH) return nhp::set_error(NHP_EUNREACH, "no pose of the goal window is reachable");
  if (best_ijt) {
    best_ijt[0] = head[2];
    best_ijt[1] = head[3];
    best_ijt[2] = head[4];
  }
  if (level) *level = head[5];
  const uint32_t n = head[1];
  if (n > cap) return nhp::set_error(NHP_ECAP, "%u steps, room for %u", n, cap);
  std::vector<uint32_t> raw((size_t)n * nhp::kExStepWords);
  if (n) {
    HIP_TRY(hipMemcpyAsync(raw.data(), x.out + nhp::kExHeader, raw.size() * 4, hipMemcpyDeviceToHost, s),
            "extract copy");
    HIP_TRY(hipStreamSynchronize(s), "extract copy");
  }
  for (uint32_t k = 0; k < n; k++) {  // goal-first on the device, start-first out
    const uint32_t* w = &raw[(size_t)(n - 1 - k) * nhp::kExStepWords];
    nhp_step& o = h_steps[k];
    memset(&o, 0, sizeof(o));
    o.maneuver = (uint8_t)w[0];
    o.steps = w[1];
    o.from_ijt[0] = w[2];
    o.from_ijt[1] = w[3];
    o.from_ijt[2] = w[4];
    o.to_ijt[0] = w[5];
    o.to_ijt[1] = w[6];
    o.to_ijt[2] = w[7];
    o.cost_q10 = w[8];
  }
  return nhp::clear_error();
}

int reach_device_ptrs(const nhp_reach* r, uint32_t** d_hard, uint32_t** d_levels) {
  int rc = check_reach(r);
  if (rc) return rc;
  if (d_hard) *d_hard = r->r.hard;
  if (d_levels) *d_levels = r->r.levels;
  return nhp::clear_error();
}

}  // extern "C"
