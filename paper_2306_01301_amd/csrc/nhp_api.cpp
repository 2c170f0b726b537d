// nhp_api.cpp -- the C ABI of include/nhp.h: plan lifetime, argument checks,
// call order, workspace layout and the launch sequence of Sec. XI.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "nhp_internal.h"

using nhp::DevPlan;
using nhp::HostTables;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int ok() {
  g_err[0] = 0;
  return NHP_OK;
}

}  // namespace

int nhp::set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int nhp::clear_error() { return ok(); }

namespace {

int hip_fail(hipError_t e, const char* what) {
  return fail(NHP_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_CHECK(call, what)                 \
  do {                                        \
    hipError_t e_ = (call);                   \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t V, B, turn_off, skew, edge_len, fwd, family, planes, taps, extract, starts, seeds, goals, total;
};

static_assert(NHP_MAX_GOALS * 16 >= NHP_MAX_SOFT_TABLE, "the soft-cost table lives in the goal-set buffer");

int seed_slots_of(const nhp_params& p) { return (int)(p.nx > p.ntheta ? p.nx : p.ntheta); }

int check_params(const nhp_params* p) {
  if (!p) return fail(NHP_EINVAL, "params is NULL");
  if (p->nx < 16 || p->nx > 1024 || p->nx % 8 != 0)
    return fail(NHP_EINVAL, "nx must be a multiple of 8 in [16, 1024] (got %u)", p->nx);
  if (p->ntheta < 8 || p->ntheta > 1024 || p->ntheta % 8 != 0)
    return fail(NHP_EINVAL, "ntheta must be a multiple of 8 in [8, 1024] (got %u)", p->ntheta);
  if (!(p->turn_radius > 0.0) || p->turn_radius > 1e6) return fail(NHP_EINVAL, "turn_radius must be > 0");
  if (p->n_schedule < 1 || p->n_schedule > 6) return fail(NHP_EINVAL, "n_schedule must be 1..6");
  for (int k = 0; k < p->n_schedule; k++)
    if (p->schedule[k] > 5) return fail(NHP_EINVAL, "schedule[%d] is not a maneuver", k);
  if (p->half_cell > 1) return fail(NHP_EINVAL, "half_cell must be 0 or 1");
  for (int mu = 0; mu < 6; mu++)
    if (p->gear_q8[mu] == 0 || p->gear_q8[mu] > 4096) return fail(NHP_EINVAL, "gear_q8 must be 1..4096");
  return NHP_OK;
}

Layout layout_of(const nhp_params& p) {
  Layout l{};
  const size_t NR = (size_t)p.nx * p.nx * p.ntheta;
  size_t o = 0;
  l.V = o;
  o = align256(o + NR * 4);
  l.B = o;
  o = align256(o + NR);
  l.turn_off = o;
  o = align256(o + 4 * (size_t)p.ntheta * 4);
  l.skew = o;
  o = align256(o + (size_t)p.ntheta * p.nx * 2);
  l.edge_len = o;
  o = align256(o + 6 * (size_t)p.ntheta * 4);
  l.fwd = o;
  o = align256(o + (size_t)p.ntheta * 4);
  l.family = o;
  o = align256(o + (size_t)p.ntheta * 4);
  l.planes = o;
  o = align256(o + (size_t)p.ntheta * 4);
  l.taps = o;
  o = align256(o + (size_t)p.ntheta * 2 * nhp::kMaxTaps * 4);
  l.extract = o;
  o = align256(o + (nhp::kExHeader + (size_t)NHP_MAX_STEPS_DEVICE * nhp::kExStepWords + nhp::kExSyncWords) * 4);
  l.starts = o;
  o = align256(o + NHP_MAX_STARTS * sizeof(nhp_start));
  l.seeds = o;
  o = align256(o + (size_t)NHP_MAX_STARTS * seed_slots_of(p) * nhp::kSeedWords * 4);
  l.goals = o;
  o = align256(o + (size_t)NHP_MAX_GOALS * 4 * 4);
  l.total = o;
  return l;
}

int check_plan(const nhp_plan* plan) {
  if (!plan) return fail(NHP_EINVAL, "plan is NULL");
  return NHP_OK;
}

// The order in which an x-major launch takes its planes (every plane is
// swept independently, so only speed depends on it).  A steeper plane has
// taller bands (64 lines plus the change of B over a chunk), so its tiles
// take longer.  The planes are dealt, steepest first, round-robin to eight
// consecutive ranges, one per XCD of the XCD-aware tile order: every XCD
// gets the same mix and works through its steep planes first, so the flat
// ones fill the launch's last round.
std::vector<int32_t> balanced_xmajor_order(const std::vector<int32_t>& planes_x, const std::vector<int16_t>& skew,
                                           int N) {
  std::vector<int32_t> by_steepness(planes_x);
  auto rise = [&](int32_t T) {
    const int d = skew[(size_t)T * N + N - 1] - skew[(size_t)T * N];
    return d < 0 ? -d : d;
  };
  std::stable_sort(by_steepness.begin(), by_steepness.end(),
                   [&](int32_t a, int32_t b) { return rise(a) > rise(b); });
  std::vector<int32_t> out;
  out.reserve(by_steepness.size());
  for (size_t x = 0; x < 8; x++)
    for (size_t i = x; i < by_steepness.size(); i += 8) out.push_back(by_steepness[i]);
  return out;
}

}  // namespace

static int finish_extract(nhp_plan* plan, nhp_step* h_steps, uint32_t cap, uint32_t* n_steps, uint32_t* best_ijt,
                          uint32_t* best_index, uint32_t* goal_value_q10, uint32_t* score_q10);

extern "C" {

const char* plan_last_error(void) { return g_err; }

int nhp_set_section_steps(uint32_t curve_len, uint32_t steps) {
  if (nhp::set_section_steps((int)curve_len, (int)steps) != NHP_OK)
    return fail(NHP_EINVAL, "steps %u is not valid for curves of length %u", steps, curve_len);
  return ok();
}

int nhp_set_knob(uint32_t knob, int32_t value) {
  if (nhp::set_knob((int)knob, (int)value) != NHP_OK)
    return fail(NHP_EINVAL, "knob %u does not take the value %d", knob, value);
  return ok();
}

int32_t nhp_get_knob(uint32_t knob) { return nhp::get_knob((int)knob); }

size_t plan_workspace_bytes(const nhp_params* params) {
  if (check_params(params) != NHP_OK) return 0;
  return layout_of(*params).total;
}

int plan_create(const nhp_params* params, void* d_workspace, size_t workspace_bytes, void* stream,
                nhp_plan** out) {
  if (!out) return fail(NHP_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = check_params(params);
  if (rc) return rc;
  if (d_workspace && ((uintptr_t)d_workspace & 255)) return fail(NHP_EINVAL, "workspace must be 256-byte aligned");
  const Layout l = layout_of(*params);
  if (d_workspace && workspace_bytes < l.total)
    return fail(NHP_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", workspace_bytes, l.total);

  nhp_plan* plan = new (std::nothrow) nhp_plan();
  if (!plan) return fail(NHP_ENOMEM, "out of host memory");
  plan->p = *params;
  plan->stream = reinterpret_cast<hipStream_t>(stream);
  rc = nhp::build_tables(plan->p, plan->t);
  if (rc) {
    delete plan;
    return fail(rc, "edge lengths out of range: every edge must be 1/1024..2048 cells (turn radius or gear)");
  }
  hipError_t e = hipGetDevice(&plan->device);
  if (e != hipSuccess) {
    delete plan;
    return hip_fail(e, "hipGetDevice");
  }
  if (d_workspace) {
    plan->ws = d_workspace;
    plan->ws_bytes = workspace_bytes;
  } else {
    e = hipMalloc(&plan->ws, l.total);
    if (e != hipSuccess) {
      delete plan;
      return fail(NHP_ENOMEM, "hipMalloc of %zu bytes failed: %s", l.total, hipGetErrorString(e));
    }
    plan->ws_bytes = l.total;
    plan->own_ws = true;
  }
  char* base = reinterpret_cast<char*>(plan->ws);
  DevPlan& d = plan->d;
  d.nx = (int)params->nx;
  d.nt = (int)params->ntheta;
  d.V = reinterpret_cast<uint32_t*>(base + l.V);
  d.B = reinterpret_cast<uint8_t*>(base + l.B);
  d.turn_off = reinterpret_cast<int32_t*>(base + l.turn_off);
  d.skew = reinterpret_cast<int16_t*>(base + l.skew);
  d.edge_len = reinterpret_cast<uint32_t*>(base + l.edge_len);
  d.fwd = reinterpret_cast<int32_t*>(base + l.fwd);
  d.family = reinterpret_cast<int32_t*>(base + l.family);
  d.planes = reinterpret_cast<int32_t*>(base + l.planes);
  d.taps = reinterpret_cast<int32_t*>(base + l.taps);
  d.extract = reinterpret_cast<uint32_t*>(base + l.extract);
  d.starts = reinterpret_cast<nhp_start*>(base + l.starts);
  d.seeds = reinterpret_cast<uint32_t*>(base + l.seeds);
  d.goals = reinterpret_cast<uint32_t*>(base + l.goals);
  d.seed_slots = seed_slots_of(*params);
  d.n_planes_x = (int)plan->t.planes_x.size();
  d.n_planes_y = (int)plan->t.planes_y.size();
  for (int mu = 0; mu < 6; mu++) {
    d.ct[mu] = params->ct_q10[mu];
    d.turn_lq[mu] = plan->t.edge_len[(size_t)mu * params->ntheta];
    d.schedule[mu] = params->schedule[mu];
  }
  d.n_schedule = params->n_schedule;

  const HostTables& t = plan->t;
  std::vector<int32_t> planes = balanced_xmajor_order(t.planes_x, *t.skew16, (int)params->nx);
  planes.insert(planes.end(), t.planes_y.begin(), t.planes_y.end());
  struct Up {
    void* dst;
    const void* src;
    size_t n;
  } ups[] = {
      {d.turn_off, t.turn_off.data(), t.turn_off.size() * 4}, {d.skew, t.skew16->data(), t.skew16->size() * 2},
      {d.edge_len, t.edge_len.data(), t.edge_len.size() * 4}, {d.fwd, t.fwd.data(), t.fwd.size() * 4},
      {d.family, t.family.data(), t.family.size() * 4},       {d.planes, planes.data(), planes.size() * 4},
  };
  for (const Up& u : ups) {
    e = hipMemcpyAsync(u.dst, u.src, u.n, hipMemcpyHostToDevice, plan->stream);
    if (e == hipSuccess) continue;
    plan_destroy(plan);
    return hip_fail(e, "table upload");
  }
  // the host vectors above are pageable and `planes` is local: wait for the copies
  e = hipStreamSynchronize(plan->stream);
  if (e != hipSuccess) {
    plan_destroy(plan);
    return hip_fail(e, "hipStreamSynchronize");
  }
  *out = plan;
  return ok();
}

int plan_destroy(nhp_plan* plan) {
  if (!plan) return ok();
  (void)hipStreamSynchronize(plan->stream);
  for (auto& row : plan->cycle)
    for (hipGraphExec_t g : row)
      if (g) (void)hipGraphExecDestroy(g);
  if (plan->own_ws && plan->ws) (void)hipFree(plan->ws);
  if (plan->readback) (void)hipHostFree(plan->readback);
  delete plan;
  return ok();
}

int plan_set_stream(nhp_plan* plan, void* stream) {
  int rc = check_plan(plan);
  if (rc) return rc;
  plan->stream = reinterpret_cast<hipStream_t>(stream);
  return ok();
}

int render_cspace(nhp_plan* plan, const uint8_t* d_image, int32_t front, int32_t rear, int32_t half_width) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (!d_image) return fail(NHP_EINVAL, "image is NULL");
  if (front < 0 || rear < 0 || half_width < 0 || front > 255 || rear > 255 || half_width > 255)
    return fail(NHP_EINVAL, "box extents must be 0..255 cells");
  const int n_side = 2 * half_width + 1, n_len = front + rear + 1;
  rc = nhp::upload_taps(plan, front, rear, half_width);
  if (rc) return rc;
  HIP_CHECK(nhp::launch_render(plan->d, d_image, n_side, n_len, plan->stream), "render_cspace launch");
  plan->has_cspace = true;
  plan->has_value = false;
  return ok();
}

}  // extern "C"

// Uploads the footprint sample offsets of every plane for a vehicle box
// (kept while the box does not change).
int nhp::check_box(int front, int rear, int half_width) {
  if (front < 0 || rear < 0 || half_width < 0 || front > 255 || rear > 255 || half_width > 255)
    return fail(NHP_EINVAL, "box extents must be 0..255 cells");
  return NHP_OK;
}

size_t nhp::taps_words(const nhp_plan* plan, int front, int rear, int half_width) {
  return (size_t)plan->p.ntheta * (size_t)((2 * half_width + 1) + (front + rear + 1));
}

// [T][n_side + n_len]: the sideways samples of plane T, then its lengthwise ones
void nhp::build_taps(const nhp_plan* plan, int front, int rear, int half_width, int32_t* out) {
  const int L = (int)plan->p.ntheta, n = (2 * half_width + 1) + (front + rear + 1);
  for (int T = 0; T < L; T++)
    nhp::render_taps_host(plan->p, plan->t, T, front, rear, half_width, out + (size_t)T * n,
                          out + (size_t)T * n + 2 * half_width + 1);
}

int nhp::upload_taps(nhp_plan* plan, int front, int rear, int half_width) {
  const int rc = nhp::check_box(front, rear, half_width);
  if (rc) return rc;
  if (front == plan->front && rear == plan->rear && half_width == plan->half_width) return NHP_OK;
  std::vector<int32_t> taps(nhp::taps_words(plan, front, rear, half_width));
  nhp::build_taps(plan, front, rear, half_width, taps.data());
  HIP_CHECK(hipMemcpyAsync(plan->d.taps, taps.data(), taps.size() * 4, hipMemcpyHostToDevice, plan->stream),
            "sample offset upload");
  HIP_CHECK(hipStreamSynchronize(plan->stream), "sample offset upload");
  plan->front = front;
  plan->rear = rear;
  plan->half_width = half_width;
  return NHP_OK;
}

extern "C" {

int soft_cost_image(nhp_plan* plan, const uint8_t* d_image, uint8_t* d_out, const uint8_t* h_table,
                    uint32_t table_len) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (!d_image || !d_out || !h_table) return fail(NHP_EINVAL, "image, out or table is NULL");
  if (table_len < 1 || table_len > NHP_MAX_SOFT_TABLE) return fail(NHP_EINVAL, "table length must be 1..%u", NHP_MAX_SOFT_TABLE);
  // scratch: the column distances in the value volume's memory, the table in
  // the goal-set buffer (both are rewritten before their next use)
  uint8_t* tab = reinterpret_cast<uint8_t*>(plan->d.goals);
  HIP_CHECK(hipMemcpyAsync(tab, h_table, table_len, hipMemcpyHostToDevice, plan->stream), "table upload");
  HIP_CHECK(nhp::launch_soft_costs(d_image, plan->d.V, tab, table_len, d_out, (int)plan->p.nx, plan->stream),
            "soft cost launch");
  HIP_CHECK(hipStreamSynchronize(plan->stream), "soft costs");  // the table copy is pageable
  plan->has_value = false;
  return ok();
}

int plan_set_cspace(nhp_plan* plan, const uint8_t* d_cspace) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (!d_cspace) return fail(NHP_EINVAL, "cspace is NULL");
  const size_t NR = (size_t)plan->p.nx * plan->p.nx * plan->p.ntheta;
  HIP_CHECK(hipMemcpyAsync(plan->d.B, d_cspace, NR, hipMemcpyDeviceToDevice, plan->stream), "cspace copy");
  HIP_CHECK(nhp::launch_force_walls(plan->d, plan->stream), "wall launch");
  plan->has_cspace = true;
  plan->has_value = false;
  return ok();
}

// The passes of one cycle of the schedule.  skip_first: the previous
// cycle's last pass already applied schedule[0].  pair_next: the cycle's last
// sweep may share a pass with the next cycle's first.  Returns whether it did.
static bool cycle_passes(const nhp_params& p, bool skip_first, bool pair_next, bool pairs,
                         std::vector<nhp::Pass>& out) {
  const uint64_t m = (uint64_t)p.n_schedule, first = skip_first ? 1 : 0;
  nhp::schedule_passes(p.schedule, (int)m, first, m - first + (pair_next ? 1 : 0), pairs, out);
  if (!pair_next || !pairs) return false;
  // the extra step is the next cycle's first sweep: keep it only inside a pair
  if (out.back().mu2 >= 0) return true;
  out.pop_back();
  return false;
}

// Captures the launches of one cycle into a graph on a private stream; the
// graph depends only on the plan's fixed device state, so it is replayed on
// whatever stream the plan uses.
static hipGraphExec_t capture_passes(nhp_plan* plan, const std::vector<nhp::Pass>& passes) {
  hipStream_t cs = nullptr;
  hipGraph_t g = nullptr;
  hipGraphExec_t exec = nullptr;
  bool ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess &&
            hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    for (const nhp::Pass& q : passes) ok = ok && nhp::launch_sweep(plan->d, q, cs) == hipSuccess;
    ok = (hipStreamEndCapture(cs, &g) == hipSuccess) && ok && g != nullptr;
  }
  if (ok) ok = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess;
  if (g) (void)hipGraphDestroy(g);
  if (cs) (void)hipStreamDestroy(cs);
  if (!ok) {
    exec = nullptr;
    plan->graph_failed = true;
    (void)hipGetLastError();  // clear a sticky capture error
  }
  return exec;
}

// n_cycles cycles of the schedule as passes (consecutive turns on shared
// curves fused, also across cycle boundaries).  A cycle's launches come from
// a captured graph once a plan runs more than one cycle for the second time:
// capturing and instantiating costs more than the launches it saves on a
// plan that is swept only once.
static int run_cycles(nhp_plan* plan, uint32_t n_cycles) {
  const bool pairs = nhp::can_fuse(plan->d);
  const bool graphs = n_cycles > 1 && plan->multi_cycle_runs++ > 0;
  bool skip = false;
  std::vector<nhp::Pass> passes;
  for (uint32_t n = 0; n < n_cycles; n++) {
    const bool pair_next = n + 1 < n_cycles;
    passes.clear();
    const bool consumed = cycle_passes(plan->p, skip, pair_next, pairs, passes);
    hipGraphExec_t& g = plan->cycle[skip][pair_next];
    if (graphs && !g && !plan->graph_failed) g = capture_passes(plan, passes);
    if (graphs && g) {
      HIP_CHECK(hipGraphLaunch(g, plan->stream), "cycle graph launch");
    } else {
      for (const nhp::Pass& q : passes) HIP_CHECK(nhp::launch_sweep(plan->d, q, plan->stream), "sweep launch");
    }
    skip = consumed;
  }
  return NHP_OK;
}

int sweep_n_turns(nhp_plan* plan, uint32_t si, uint32_t sj, uint32_t st, uint32_t n_cycles) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (!plan->has_cspace) return fail(NHP_ESTATE, "sweep_n_turns before render_cspace/plan_set_cspace");
  if (si >= plan->p.nx || sj >= plan->p.nx || st >= plan->p.ntheta) return fail(NHP_EINVAL, "start outside the grid");
  const size_t s = ((size_t)st * plan->p.nx + sj) * plan->p.nx + si;
  uint8_t code = 0;
  HIP_CHECK(hipMemcpyAsync(&code, plan->d.B + s, 1, hipMemcpyDeviceToHost, plan->stream), "start check");
  HIP_CHECK(hipStreamSynchronize(plan->stream), "start check");
  if (code == NHP_HARD) return fail(NHP_ESTART, "start pose (%u, %u, %u) is in collision", si, sj, st);
  HIP_CHECK(nhp::launch_init(plan->d, (uint32_t)s, plan->stream), "init launch");
  plan->n_starts = 0;
  plan->start[0] = si;
  plan->start[1] = sj;
  plan->start[2] = st;
  plan->has_value = true;
  return (rc = run_cycles(plan, n_cycles)) ? rc : ok();
}

int sweep_from_set(nhp_plan* plan, const nhp_start* h_starts, uint32_t n_starts, uint32_t n_cycles) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (!plan->has_cspace) return fail(NHP_ESTATE, "sweep_from_set before render_cspace/plan_set_cspace");
  if (!h_starts || n_starts < 1 || n_starts > NHP_MAX_STARTS)
    return fail(NHP_EINVAL, "1..%u starts needed (got %u)", NHP_MAX_STARTS, n_starts);
  std::vector<uint8_t> codes(n_starts);
  for (uint32_t k = 0; k < n_starts; k++) {
    const nhp_start& st = h_starts[k];
    if (st.i >= plan->p.nx || st.j >= plan->p.nx || st.T >= plan->p.ntheta)
      return fail(NHP_EINVAL, "start %u outside the grid", k);
    if (st.maneuver < -1 || st.maneuver > 5) return fail(NHP_EINVAL, "start %u: maneuver must be -1..5", k);
    const size_t idx = ((size_t)st.T * plan->p.nx + st.j) * plan->p.nx + st.i;
    HIP_CHECK(hipMemcpyAsync(&codes[k], plan->d.B + idx, 1, hipMemcpyDeviceToHost, plan->stream), "start check");
  }
  HIP_CHECK(hipMemcpyAsync(plan->d.starts, h_starts, n_starts * sizeof(nhp_start), hipMemcpyHostToDevice,
                           plan->stream),
            "start upload");
  HIP_CHECK(hipStreamSynchronize(plan->stream), "start check");
  for (uint32_t k = 0; k < n_starts; k++)
    if (codes[k] == NHP_HARD) return fail(NHP_ESTART, "start %u is in collision", k);
  // init with the start pose outside the volume: V = INF everywhere
  HIP_CHECK(nhp::launch_init(plan->d, 0xFFFFFFFFu, plan->stream), "init launch");
  HIP_CHECK(nhp::launch_seed(plan->d, (int)n_starts, plan->stream), "seed launch");
  plan->n_starts = (int)n_starts;
  plan->start[0] = h_starts[0].i;
  plan->start[1] = h_starts[0].j;
  plan->start[2] = h_starts[0].T;
  plan->has_value = true;
  return (rc = run_cycles(plan, n_cycles)) ? rc : ok();
}

int sweep_resume(nhp_plan* plan, uint32_t n_more_cycles) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (!plan->has_value) return fail(NHP_ESTATE, "sweep_resume before sweep_n_turns");
  return (rc = run_cycles(plan, n_more_cycles)) ? rc : ok();
}

int sweep_pass(nhp_plan* plan, int32_t first, int32_t second) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (!plan->has_cspace) return fail(NHP_ESTATE, "sweep_pass before render_cspace/plan_set_cspace");
  if (first < 0 || first > 5 || second < -1 || second > 5) return fail(NHP_EINVAL, "maneuvers must be 0..5 (second: -1 for none)");
  HIP_CHECK(nhp::launch_sweep(plan->d, nhp::Pass{(int8_t)first, (int8_t)second}, plan->stream), "sweep launch");
  return ok();
}

int sweep_straight_family(nhp_plan* plan, uint32_t maneuver, uint32_t family) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (!plan->has_cspace) return fail(NHP_ESTATE, "sweep_straight_family before render_cspace/plan_set_cspace");
  if (maneuver != NHP_SF && maneuver != NHP_SB) return fail(NHP_EINVAL, "maneuver must be NHP_SF or NHP_SB");
  if (family > 1) return fail(NHP_EINVAL, "family must be 0 or 1");
  HIP_CHECK(nhp::launch_sweep_part(plan->d, nhp::Pass{(int8_t)maneuver, (int8_t)-1}, family ? 1 : 2, plan->stream),
            "sweep launch");
  return ok();
}

int schedule_passes(const uint8_t* schedule, uint32_t n_schedule, uint64_t first_step, uint64_t n_steps,
                    int32_t pairs, int8_t* first, int8_t* second, uint32_t cap, uint32_t* n_passes) {
  if (!schedule || n_schedule < 1 || n_schedule > 6 || !n_passes) return fail(NHP_EINVAL, "bad schedule or NULL count");
  for (uint32_t k = 0; k < n_schedule; k++)
    if (schedule[k] > 5) return fail(NHP_EINVAL, "schedule entries must be 0..5");
  std::vector<nhp::Pass> v;
  nhp::schedule_passes(schedule, (int)n_schedule, first_step, n_steps, pairs != 0, v);
  *n_passes = (uint32_t)v.size();
  if (v.size() > cap) return fail(NHP_ECAP, "%zu passes, room for %u", v.size(), cap);
  if (!v.empty() && (!first || !second)) return fail(NHP_EINVAL, "output arrays are NULL");
  for (size_t k = 0; k < v.size(); k++) {
    first[k] = v[k].mu;
    second[k] = v[k].mu2;
  }
  return ok();
}

int sweep_one(nhp_plan* plan, uint32_t maneuver) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (!plan->has_cspace) return fail(NHP_ESTATE, "sweep_one before render_cspace/plan_set_cspace");
  if (maneuver > 5) return fail(NHP_EINVAL, "maneuver must be 0..5");
  HIP_CHECK(nhp::launch_sweep(plan->d, nhp::Pass{(int8_t)maneuver, (int8_t)-1}, plan->stream), "sweep launch");
  return ok();
}

int extract_path(nhp_plan* plan, uint32_t gi, uint32_t gj, uint32_t gt, uint32_t radius, uint32_t w_xy_q10,
                 uint32_t w_t_q10, nhp_step* h_steps, uint32_t cap, uint32_t* n_steps, uint32_t* best_ijt,
                 uint32_t* goal_value_q10, uint32_t* score_q10) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (!plan->has_value) return fail(NHP_ESTATE, "extract_path before sweep_n_turns");
  if (gi >= plan->p.nx || gj >= plan->p.nx || gt >= plan->p.ntheta) return fail(NHP_EINVAL, "goal outside the grid");
  if (radius > (uint32_t)nhp::kMaxRadius) return fail(NHP_EINVAL, "goal radius must be 0..%d", nhp::kMaxRadius);
  if (cap > 0 && !h_steps) return fail(NHP_EINVAL, "h_steps is NULL");
  nhp::ExArgs x{};
  x.d = plan->d;
  x.si = plan->start[0];
  x.sj = plan->start[1];
  x.st = plan->start[2];
  x.gi = gi;
  x.gj = gj;
  x.gt = gt;
  x.radius = (int)radius;
  x.w_xy = w_xy_q10;
  x.w_t = w_t_q10;
  x.n_starts = plan->n_starts;
  HIP_CHECK(nhp::launch_extract(x, plan->stream), "extract launch");
  return finish_extract(plan, h_steps, cap, n_steps, best_ijt, nullptr, goal_value_q10, score_q10);
}

// extract_path with its extract area in the library's file-scope device
// array: no allocation of any kind on this path (the header comes back into a
// local array, the steps straight into the caller's step buffer, which is
// then put into start -> goal order in place).
static_assert(sizeof(nhp_step) == nhp::kExStepWords * 4, "a device step record and an nhp_step have one size");

int extract_path_noalloc(nhp_plan* plan, uint32_t gi, uint32_t gj, uint32_t gt, uint32_t radius, uint32_t w_xy_q10,
                         uint32_t w_t_q10, nhp_step* h_steps, uint32_t cap, uint32_t* n_steps, uint32_t* best_ijt,
                         uint32_t* goal_value_q10, uint32_t* score_q10) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (!plan->has_value) return fail(NHP_ESTATE, "extract_path_noalloc before sweep_n_turns");
  if (gi >= plan->p.nx || gj >= plan->p.nx || gt >= plan->p.ntheta) return fail(NHP_EINVAL, "goal outside the grid");
  if (radius > (uint32_t)nhp::kMaxRadius) return fail(NHP_EINVAL, "goal radius must be 0..%d", nhp::kMaxRadius);
  if (cap > 0 && !h_steps) return fail(NHP_EINVAL, "h_steps is NULL");
  uint32_t* area = nullptr;
  HIP_CHECK(nhp::noalloc_extract_area(plan->device, &area), "extract area lookup");
  nhp::ExArgs x{};
  x.d = plan->d;
  x.d.extract = area;  // the kernels take the looked-up address, never the array's name
  x.si = plan->start[0];
  x.sj = plan->start[1];
  x.st = plan->start[2];
  x.gi = gi;
  x.gj = gj;
  x.gt = gt;
  x.radius = (int)radius;
  x.w_xy = w_xy_q10;
  x.w_t = w_t_q10;
  x.n_starts = plan->n_starts;
  HIP_CHECK(nhp::launch_extract(x, plan->stream), "extract launch");
  uint32_t head[nhp::kExHeader];
  HIP_CHECK(hipMemcpyAsync(head, area, sizeof(head), hipMemcpyDeviceToHost, plan->stream), "extract copy");
  HIP_CHECK(hipStreamSynchronize(plan->stream), "extract copy");
  const uint32_t status = head[0], n = head[1];
  if (n_steps) *n_steps = n;
  if (status != 0 && status != (uint32_t)(-NHP_EUNREACH))
    return fail(NHP_EHIP, "extract kernel returned status %u", status);
  if (status == (uint32_t)(-NHP_EUNREACH))
    return fail(NHP_EUNREACH, "no reached pose in the goal window (or back-tracking lost the path)");
  if (best_ijt) memcpy(best_ijt, head + 2, 3 * sizeof(uint32_t));
  if (goal_value_q10) *goal_value_q10 = head[5];
  if (score_q10) *score_q10 = head[6];
  if (n > NHP_MAX_STEPS_DEVICE || n > cap) return fail(NHP_ECAP, "plan has %u steps, buffer holds %u", n, cap);
  if (n == 0) return ok();
  HIP_CHECK(hipMemcpyAsync(h_steps, area + nhp::kExHeader, (size_t)n * sizeof(nhp_step), hipMemcpyDeviceToHost,
                           plan->stream),
            "extract copy");
  HIP_CHECK(hipStreamSynchronize(plan->stream), "extract copy");
  // device records are goal -> start: reverse them and convert each
  auto convert = [](const uint32_t* s, nhp_step& o) {
    memset(&o, 0, sizeof(o));
    o.maneuver = (uint8_t)s[0];
    o.steps = s[1];
    memcpy(o.from_ijt, s + 2, 3 * sizeof(uint32_t));
    memcpy(o.to_ijt, s + 5, 3 * sizeof(uint32_t));
    o.cost_q10 = s[8];
  };
  for (uint32_t a = 0, b = n - 1; a <= b; a++, b--) {
    uint32_t ra[nhp::kExStepWords], rb[nhp::kExStepWords];
    memcpy(ra, &h_steps[a], sizeof(ra));
    memcpy(rb, &h_steps[b], sizeof(rb));
    convert(rb, h_steps[a]);
    if (a != b) convert(ra, h_steps[b]);
    if (b == 0) break;
  }
  return ok();
}

// Reads back the result of an extract launch: header, then the steps in
// start -> goal order.
static int finish_extract(nhp_plan* plan, nhp_step* h_steps, uint32_t cap, uint32_t* n_steps, uint32_t* best_ijt,
                          uint32_t* best_index, uint32_t* goal_value_q10, uint32_t* score_q10) {
  // the header and the first steps in one copy to pinned memory; longer
  // plans fetch the rest with a second copy
  const size_t first_words = nhp::kExHeader + (size_t)nhp::kReadbackSteps * nhp::kExStepWords;
  if (!plan->readback)
    HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&plan->readback), first_words * 4, hipHostMallocDefault),
              "hipHostMalloc");
  HIP_CHECK(hipMemcpyAsync(plan->readback, plan->d.extract, first_words * 4, hipMemcpyDeviceToHost, plan->stream),
            "extract copy");
  HIP_CHECK(hipStreamSynchronize(plan->stream), "extract copy");
  const uint32_t* head = plan->readback;
  const uint32_t status = head[0], n = head[1];
  if (n_steps) *n_steps = n;
  if (status != 0 && status != (uint32_t)(-NHP_EUNREACH))
    return fail(NHP_EHIP, "extract kernel returned status %u", status);
  if (status == (uint32_t)(-NHP_EUNREACH))
    return fail(NHP_EUNREACH, "no reached pose in the goal window (or back-tracking lost the path)");
  if (best_ijt) memcpy(best_ijt, head + 2, 3 * sizeof(uint32_t));
  if (best_index) *best_index = head[7];
  if (goal_value_q10) *goal_value_q10 = head[5];
  if (score_q10) *score_q10 = head[6];
  if (n > NHP_MAX_STEPS_DEVICE || n > cap) return fail(NHP_ECAP, "plan has %u steps, buffer holds %u", n, cap);
  std::vector<uint32_t> rest;
  const uint32_t* raw = head + nhp::kExHeader;
  if (n > (uint32_t)nhp::kReadbackSteps) {
    rest.resize((size_t)n * nhp::kExStepWords);
    HIP_CHECK(hipMemcpyAsync(rest.data(), plan->d.extract + nhp::kExHeader, rest.size() * 4, hipMemcpyDeviceToHost,
                             plan->stream),
              "extract copy");
    HIP_CHECK(hipStreamSynchronize(plan->stream), "extract copy");
    raw = rest.data();
  }
  for (uint32_t k = 0; k < n; k++) {  // device order is goal -> start
    const uint32_t* s = &raw[(size_t)(n - 1 - k) * nhp::kExStepWords];
    nhp_step& o = h_steps[k];
    memset(&o, 0, sizeof(o));
    o.maneuver = (uint8_t)s[0];
    o.steps = s[1];
    o.from_ijt[0] = s[2];
    o.from_ijt[1] = s[3];
    o.from_ijt[2] = s[4];
    o.to_ijt[0] = s[5];
    o.to_ijt[1] = s[6];
    o.to_ijt[2] = s[7];
    o.cost_q10 = s[8];
  }
  return ok();
}

int extract_path_set(nhp_plan* plan, const uint32_t* goals_ijt, const uint32_t* penalty_q10, uint32_t n_goals,
                     nhp_step* h_steps, uint32_t cap, uint32_t* n_steps, uint32_t* best_index,
                     uint32_t* goal_value_q10, uint32_t* score_q10) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (!plan->has_value) return fail(NHP_ESTATE, "extract_path_set before a sweep");
  if (!goals_ijt || !penalty_q10 || n_goals < 1 || n_goals > NHP_MAX_GOALS)
    return fail(NHP_EINVAL, "1..%u goals needed (got %u)", NHP_MAX_GOALS, n_goals);
  if (cap > 0 && !h_steps) return fail(NHP_EINVAL, "h_steps is NULL");
  std::vector<uint32_t> g((size_t)n_goals * 4);
  for (uint32_t k = 0; k < n_goals; k++) {
    if (goals_ijt[3 * k] >= plan->p.nx || goals_ijt[3 * k + 1] >= plan->p.nx || goals_ijt[3 * k + 2] >= plan->p.ntheta)
      return fail(NHP_EINVAL, "goal %u outside the grid", k);
    g[4 * k] = goals_ijt[3 * k];
    g[4 * k + 1] = goals_ijt[3 * k + 1];
    g[4 * k + 2] = goals_ijt[3 * k + 2];
    g[4 * k + 3] = penalty_q10[k];
  }
  HIP_CHECK(hipMemcpyAsync(plan->d.goals, g.data(), g.size() * 4, hipMemcpyHostToDevice, plan->stream), "goal upload");
  nhp::ExArgs x{};
  x.d = plan->d;
  x.si = plan->start[0];
  x.sj = plan->start[1];
  x.st = plan->start[2];
  x.n_goals = (int)n_goals;
  x.n_starts = plan->n_starts;
  HIP_CHECK(nhp::launch_extract(x, plan->stream), "extract launch");
  // finish_extract synchronises, so the pageable goal copy has completed
  return finish_extract(plan, h_steps, cap, n_steps, nullptr, best_index, goal_value_q10, score_q10);
}

int plan_device_ptrs(const nhp_plan* plan, uint32_t** d_value, uint8_t** d_cspace) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (d_value) *d_value = plan->d.V;
  if (d_cspace) *d_cspace = plan->d.B;
  return ok();
}

int plan_get_tables(const nhp_plan* plan, int32_t* beta, int32_t* psi, int32_t* family, int32_t* fwd_sign,
                    int32_t* skew, uint32_t* edge_len) {
  int rc = check_plan(plan);
  if (rc) return rc;
  const HostTables& t = plan->t;
  if (beta) memcpy(beta, t.beta.data(), t.beta.size() * 4);
  if (psi) memcpy(psi, t.psi.data(), t.psi.size() * 4);
  if (family) memcpy(family, t.family.data(), t.family.size() * 4);
  if (fwd_sign) memcpy(fwd_sign, t.fwd.data(), t.fwd.size() * 4);
  if (skew)
    for (size_t k = 0; k < t.skew16->size(); k++) skew[k] = (*t.skew16)[k];
  if (edge_len) memcpy(edge_len, t.edge_len.data(), t.edge_len.size() * 4);
  return ok();
}

}  // extern "C"
