// nhp_batch.cpp -- batched launches over many plans: one launch per pass
// covers the current maneuver of every plan in the batch (tiles of all plans
// in one grid), so small plans fill the GPU together and a plan that joins
// later runs alongside plans that are further along (continuous batching).
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "nhp_internal.h"

namespace {

constexpr int kSlots = 4;  // job tables in flight (ring), each reused only after its launches finished
constexpr int kMaxGraphs = 16;  // captured launch sequences kept per batch
constexpr int kSeen = 64;       // launch sequences remembered (by hash) to capture on their second run

// A launch sequence captured into a graph: its key (the knob values, the job
// table and the launch list, byte for byte), the device job table its kernels
// read, and an event recorded after its latest replay.
struct CachedGraph {
  std::vector<unsigned char> key;
  uint64_t hash = 0;
  hipGraphExec_t exec = nullptr;
  void* table = nullptr;
  hipEvent_t last = nullptr;
  uint64_t used = 0;
};

uint64_t fnv1a(const unsigned char* p, size_t n) {
  uint64_t h = 1469598103934665603ull;
  for (size_t k = 0; k < n; k++) h = (h ^ p[k]) * 1099511628211ull;
  return h;
}

struct Slot {
  void* host = nullptr;  // pinned staging buffer
  void* dev = nullptr;   // device copy read by the kernels
  size_t bytes = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
};

#define HIP_TRY(call, what)                                                               \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return nhp::set_error(NHP_EHIP, "%s: %s", what, hipGetErrorString(e_)); \
  } while (0)

}  // namespace

struct nhp_batch {
  hipStream_t stream = nullptr;
  uint32_t capacity = 0;
  Slot slot[kSlots];
  int next = 0;
  std::vector<CachedGraph> graphs;
  uint64_t seen[kSeen] = {};
  int seen_next = 0;
  uint64_t clock = 0;
  bool graph_failed = false;  // capture unavailable: launch directly
};

namespace {

// A slot whose previous launches have finished, with room for `bytes`.
int take_slot(nhp_batch* b, size_t bytes, Slot** out) {
  Slot& s = b->slot[b->next];
  b->next = (b->next + 1) % kSlots;
  if (s.pending) {
    HIP_TRY(hipEventSynchronize(s.done), "hipEventSynchronize");
    s.pending = false;
  }
  if (s.bytes < bytes) {
    size_t nb = std::max(bytes, (size_t)65536);
    if (s.host) (void)hipHostFree(s.host);
    if (s.dev) (void)hipFree(s.dev);
    s.host = s.dev = nullptr;
    s.bytes = 0;
    HIP_TRY(hipHostMalloc(&s.host, nb, hipHostMallocDefault), "hipHostMalloc");
    HIP_TRY(hipMalloc(&s.dev, nb), "hipMalloc");
    s.bytes = nb;
  }
  *out = &s;
  return NHP_OK;
}

int finish_slot(nhp_batch* b, Slot* s) {
  HIP_TRY(hipEventRecord(s->done, b->stream), "hipEventRecord");
  s->pending = true;
  return NHP_OK;
}

int check_plans(nhp_batch* b, nhp_plan* const* plans, uint32_t n) {
  if (!b) return nhp::set_error(NHP_EINVAL, "batch is NULL");
  if (n > b->capacity) return nhp::set_error(NHP_EINVAL, "%u plans exceed the batch capacity %u", n, b->capacity);
  if (n && !plans) return nhp::set_error(NHP_EINVAL, "plans is NULL");
  for (uint32_t k = 0; k < n; k++) {
    if (!plans[k]) return nhp::set_error(NHP_EINVAL, "plans[%u] is NULL", k);
    for (uint32_t m = 0; m < k; m++)
      if (plans[m] == plans[k]) return nhp::set_error(NHP_EINVAL, "plan listed twice (%u and %u)", m, k);
  }
  return NHP_OK;
}

}  // namespace

extern "C" {

int batch_create(uint32_t capacity, void* stream, nhp_batch** out) {
  if (!out) return nhp::set_error(NHP_EINVAL, "out is NULL");
  *out = nullptr;
  if (capacity == 0 || capacity > 65536) return nhp::set_error(NHP_EINVAL, "capacity must be 1..65536");
  nhp_batch* b = new (std::nothrow) nhp_batch();
  if (!b) return nhp::set_error(NHP_ENOMEM, "out of host memory");
  b->stream = reinterpret_cast<hipStream_t>(stream);
  b->capacity = capacity;
  for (Slot& s : b->slot) {
    if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) {
      batch_destroy(b);
      return nhp::set_error(NHP_EHIP, "hipEventCreate failed");
    }
  }
  *out = b;
  return nhp::clear_error();
}

int batch_destroy(nhp_batch* b) {
  if (!b) return nhp::clear_error();
  (void)hipStreamSynchronize(b->stream);
  for (CachedGraph& g : b->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.table) (void)hipFree(g.table);
    if (g.last) (void)hipEventDestroy(g.last);
  }
  for (Slot& s : b->slot) {
    if (s.host) (void)hipHostFree(s.host);
    if (s.dev) (void)hipFree(s.dev);
    if (s.done) (void)hipEventDestroy(s.done);
  }
  delete b;
  return nhp::clear_error();
}

int batch_render(nhp_batch* b, nhp_plan* const* plans, const uint8_t* const* d_images, const int32_t* boxes_frs,
                 uint32_t n) {
  int rc = check_plans(b, plans, n);
  if (rc) return rc;
  if (n == 0) return nhp::clear_error();
  if (!d_images || !boxes_frs) return nhp::set_error(NHP_EINVAL, "images or boxes is NULL");
  std::vector<nhp::RenderJob> jobs(n);
  // plans whose box changed get new sample offsets, built straight into the
  // pinned staging slot after the job table and copied on the batch stream
  std::vector<size_t> tap_at(n, 0), tap_len(n, 0);
  size_t tap_words = 0;
  int total = 0, pad_rows = 0;
  for (uint32_t k = 0; k < n; k++) {
    nhp_plan* p = plans[k];
    if (!d_images[k]) return nhp::set_error(NHP_EINVAL, "images[%u] is NULL", k);
    const int f = boxes_frs[3 * k], r = boxes_frs[3 * k + 1], hw = boxes_frs[3 * k + 2];
    rc = nhp::check_box(f, r, hw);
    if (rc) return rc;
    if (f != p->front || r != p->rear || hw != p->half_width) {
      tap_at[k] = tap_words;
      tap_len[k] = nhp::taps_words(p, f, r, hw);
      tap_words += tap_len[k];
    }
    nhp::RenderJob& job = jobs[k];
    job.image = d_images[k];
    job.side = reinterpret_cast<uint8_t*>(p->d.V);
    job.B = p->d.B;
    job.taps = p->d.taps;
    job.N = p->d.nx;
    job.nt = p->d.nt;
    job.n_side = 2 * hw + 1;
    job.n_len = f + r + 1;
    job.blocks = nhp::render_blocks(job.N, job.nt);
    job.first_block = total;
    total += job.blocks;
    job.pad_first = pad_rows;
    pad_rows += job.N;
  }
  const size_t job_bytes = (jobs.size() * sizeof(nhp::RenderJob) + 255) & ~(size_t)255;
  Slot* s;
  rc = take_slot(b, job_bytes + tap_words * 4, &s);
  if (rc) return rc;
  memcpy(s->host, jobs.data(), jobs.size() * sizeof(nhp::RenderJob));
  int32_t* taps = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(s->host) + job_bytes);
  for (uint32_t k = 0; k < n; k++) {
    if (!tap_len[k]) continue;
    nhp_plan* p = plans[k];
    const int f = boxes_frs[3 * k], r = boxes_frs[3 * k + 1], hw = boxes_frs[3 * k + 2];
    // work of the plan's own stream may still read its old offsets
    if (p->stream != b->stream) HIP_TRY(hipStreamSynchronize(p->stream), "plan stream");
    nhp::build_taps(p, f, r, hw, taps + tap_at[k]);
    HIP_TRY(hipMemcpyAsync(p->d.taps, taps + tap_at[k], tap_len[k] * 4, hipMemcpyHostToDevice, b->stream),
            "sample offset upload");
    p->front = f;
    p->rear = r;
    p->half_width = hw;
  }
  HIP_TRY(hipMemcpyAsync(s->dev, s->host, jobs.size() * sizeof(nhp::RenderJob), hipMemcpyHostToDevice, b->stream),
          "job upload");
  HIP_TRY(nhp::launch_render_batch(reinterpret_cast<const nhp::RenderJob*>(s->dev), (int)n, total, pad_rows,
                                   b->stream),
          "render launch");
  for (uint32_t k = 0; k < n; k++) {
    plans[k]->has_cspace = true;
    plans[k]->has_value = false;
  }
  rc = finish_slot(b, s);
  return rc ? rc : nhp::clear_error();
}

int batch_init(nhp_batch* b, nhp_plan* const* plans, const uint32_t* starts_ijt, uint32_t n) {
  int rc = check_plans(b, plans, n);
  if (rc) return rc;
  if (n == 0) return nhp::clear_error();
  if (!starts_ijt) return nhp::set_error(NHP_EINVAL, "starts is NULL");
  std::vector<nhp::InitJob> jobs(n);
  size_t max_n4 = 0;
  std::vector<uint8_t> codes(n, 0);
  for (uint32_t k = 0; k < n; k++) {
    nhp_plan* p = plans[k];
    if (!p->has_cspace) return nhp::set_error(NHP_ESTATE, "plans[%u] has no obstacle volume", k);
    const uint32_t si = starts_ijt[3 * k], sj = starts_ijt[3 * k + 1], st = starts_ijt[3 * k + 2];
    if (si >= p->p.nx || sj >= p->p.nx || st >= p->p.ntheta)
      return nhp::set_error(NHP_EINVAL, "start of plans[%u] outside its grid", k);
    const size_t idx = ((size_t)st * p->p.nx + sj) * p->p.nx + si;
    HIP_TRY(hipMemcpyAsync(&codes[k], p->d.B + idx, 1, hipMemcpyDeviceToHost, b->stream), "start check");
    jobs[k].V = p->d.V;
    jobs[k].n4 = (size_t)p->p.nx * p->p.nx * p->p.ntheta / 4;
    jobs[k].start = (uint32_t)idx;
    max_n4 = std::max(max_n4, jobs[k].n4);
  }
  HIP_TRY(hipStreamSynchronize(b->stream), "start check");
  for (uint32_t k = 0; k < n; k++)
    if (codes[k] == NHP_HARD) return nhp::set_error(NHP_ESTART, "start of plans[%u] is in collision", k);
  Slot* s;
  rc = take_slot(b, jobs.size() * sizeof(nhp::InitJob), &s);
  if (rc) return rc;
  memcpy(s->host, jobs.data(), jobs.size() * sizeof(nhp::InitJob));
  HIP_TRY(hipMemcpyAsync(s->dev, s->host, jobs.size() * sizeof(nhp::InitJob), hipMemcpyHostToDevice, b->stream),
          "job upload");
  HIP_TRY(nhp::launch_init_batch(reinterpret_cast<const nhp::InitJob*>(s->dev), (int)n, max_n4, b->stream),
          "init launch");
  for (uint32_t k = 0; k < n; k++) {
    plans[k]->has_value = true;
    plans[k]->n_starts = 0;
    plans[k]->start[0] = starts_ijt[3 * k];
    plans[k]->start[1] = starts_ijt[3 * k + 1];
    plans[k]->start[2] = starts_ijt[3 * k + 2];
  }
  rc = finish_slot(b, s);
  return rc ? rc : nhp::clear_error();
}

// One launch of a batched pass: a group of jobs with the same kernel shape.
struct Launch {
  size_t first;  // index of the group's first job in the uploaded table
  int n_jobs, blocks;
  int P, fused, guard, pow2, waves;  // waves = 0: x-major jobs
};

// Appends one pass for each listed plan: row jobs grouped by section size,
// fused or single, guard, power-of-two grid side and wave count (workgroups
// of exactly the job's waves), x-major jobs in one more group; one launch
// per group.
static int add_pass(nhp_plan* const* plans, const nhp::Pass* passes, uint32_t n, std::vector<nhp::SweepJob>& table,
                    std::vector<Launch>& launches) {
  struct Group {
    int P, fused, guard, pow2, waves;
    std::vector<nhp::SweepJob> jobs;
  };
  std::vector<Group> groups;
  auto group_of = [&](int P, int fused, int guard, int pow2, int waves) -> Group& {
    for (Group& g : groups)
      if (g.P == P && g.fused == fused && g.guard == guard && g.pow2 == pow2 && g.waves == waves) return g;
    groups.push_back(Group{P, fused, guard, pow2, waves, {}});
    return groups.back();
  };
  for (uint32_t k = 0; k < n; k++) {
    nhp::SweepJob row{}, xm{};
    if (nhp::make_sweep_jobs(plans[k]->d, passes[k], &row, &xm) < 0)
      return nhp::set_error(NHP_EINVAL, "section sizes changed while a batch was being formed");
    if (row.blocks) {
      if (row.P != 8 && row.P != 16 && row.P != 32 && row.P != 64)
        return nhp::set_error(NHP_EINVAL, "a plan has no section size for its curve length");
      group_of(row.P, row.fused, row.L % row.P != 0, (row.N & (row.N - 1)) == 0, (row.L + row.P - 1) / row.P)
          .jobs.push_back(row);
    }
    if (xm.blocks) group_of(0, 0, 0, nhp::xmajor_wide(xm.N) ? 1 : 0, 0).jobs.push_back(xm);
  }
  for (Group& g : groups) {
    Launch l{table.size(), (int)g.jobs.size(), 0, g.P, g.fused, g.guard, g.pow2, g.waves};
    for (nhp::SweepJob& j : g.jobs) {
      j.first_block = l.blocks;
      l.blocks += j.blocks;
      table.push_back(j);
    }
    launches.push_back(l);
  }
  return NHP_OK;
}

static hipError_t enqueue_launches(const nhp::SweepJob* d, const std::vector<Launch>& launches, hipStream_t st) {
  for (const Launch& l : launches) {
    const hipError_t e = nhp::launch_sweep_batch(d + l.first, l.n_jobs, l.blocks, l.P, l.fused != 0, l.guard != 0,
                                                 l.pow2 != 0, l.waves == 0, l.waves, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The launches of a job table captured into a graph over a device copy of the
// table that the graph owns; nullptr when capture is unavailable.
static hipGraphExec_t capture_launches(const std::vector<nhp::SweepJob>& table, const std::vector<Launch>& launches,
                                       void** d_table) {
  *d_table = nullptr;
  const size_t bytes = table.size() * sizeof(nhp::SweepJob);
  if (hipMalloc(d_table, bytes) != hipSuccess) return nullptr;
  hipStream_t cs = nullptr;
  hipGraph_t g = nullptr;
  hipGraphExec_t exec = nullptr;
  bool ok = hipMemcpy(*d_table, table.data(), bytes, hipMemcpyHostToDevice) == hipSuccess &&
            hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess &&
            hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    ok = enqueue_launches(reinterpret_cast<const nhp::SweepJob*>(*d_table), launches, cs) == hipSuccess;
    ok = (hipStreamEndCapture(cs, &g) == hipSuccess) && ok && g != nullptr;
  }
  if (ok) ok = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess;
  if (g) (void)hipGraphDestroy(g);
  if (cs) (void)hipStreamDestroy(cs);
  if (!ok) {
    (void)hipGetLastError();  // clear a sticky capture error
    if (*d_table) (void)hipFree(*d_table);
    *d_table = nullptr;
    return nullptr;
  }
  return exec;
}

// Runs the launches of a job table.  A table (with the same knob values and
// launch list) seen before in this batch is captured into a graph the second
// time and replayed from then on (the cycles of a batch_sweep, or a batch of
// the same plans planned again); otherwise the table is uploaded from a ring
// slot and the launches go out directly.
static int run_launches(nhp_batch* b, const std::vector<nhp::SweepJob>& table, const std::vector<Launch>& launches) {
  if (table.empty()) return NHP_OK;
  std::vector<unsigned char> key(nhp::kKnobs * sizeof(int32_t) + table.size() * sizeof(nhp::SweepJob) +
                                 launches.size() * sizeof(Launch));
  unsigned char* kp = key.data();
  for (int k = 0; k < nhp::kKnobs; k++) {
    const int32_t v = nhp::get_knob(k);
    memcpy(kp, &v, sizeof(v));
    kp += sizeof(v);
  }
  memcpy(kp, table.data(), table.size() * sizeof(nhp::SweepJob));
  kp += table.size() * sizeof(nhp::SweepJob);
  memcpy(kp, launches.data(), launches.size() * sizeof(Launch));
  const uint64_t h = fnv1a(key.data(), key.size());
  for (CachedGraph& g : b->graphs) {
    if (g.hash != h || g.key != key) continue;
    HIP_TRY(hipGraphLaunch(g.exec, b->stream), "graph launch");
    HIP_TRY(hipEventRecord(g.last, b->stream), "hipEventRecord");
    g.used = ++b->clock;
    return NHP_OK;
  }
  bool again = false;
  for (uint64_t x : b->seen) again = again || x == h;
  if (again && !b->graph_failed) {
    CachedGraph g;
    g.exec = capture_launches(table, launches, &g.table);
    if (!g.exec) {
      b->graph_failed = true;
    } else {
      HIP_TRY(hipEventCreateWithFlags(&g.last, hipEventDisableTiming), "hipEventCreate");
      if ((int)b->graphs.size() >= kMaxGraphs) {
        // the least recently used graph goes, once its latest replay is done
        auto victim = std::min_element(b->graphs.begin(), b->graphs.end(),
                                       [](const CachedGraph& x, const CachedGraph& y) { return x.used < y.used; });
        HIP_TRY(hipEventSynchronize(victim->last), "hipEventSynchronize");
        (void)hipGraphExecDestroy(victim->exec);
        (void)hipFree(victim->table);
        (void)hipEventDestroy(victim->last);
        b->graphs.erase(victim);
      }
      g.key = std::move(key);
      g.hash = h;
      g.used = ++b->clock;
      b->graphs.push_back(g);
      CachedGraph& c = b->graphs.back();
      HIP_TRY(hipGraphLaunch(c.exec, b->stream), "graph launch");
      HIP_TRY(hipEventRecord(c.last, b->stream), "hipEventRecord");
      return NHP_OK;
    }
  }
  b->seen[b->seen_next] = h;
  b->seen_next = (b->seen_next + 1) % kSeen;
  Slot* s;
  int rc = take_slot(b, table.size() * sizeof(nhp::SweepJob), &s);
  if (rc) return rc;
  memcpy(s->host, table.data(), table.size() * sizeof(nhp::SweepJob));
  HIP_TRY(hipMemcpyAsync(s->dev, s->host, table.size() * sizeof(nhp::SweepJob), hipMemcpyHostToDevice, b->stream),
          "job upload");
  HIP_TRY(enqueue_launches(reinterpret_cast<const nhp::SweepJob*>(s->dev), launches, b->stream), "sweep launch");
  return finish_slot(b, s);
}

int batch_advance(nhp_batch* b, nhp_plan* const* plans, const uint32_t* steps, const uint32_t* counts, uint32_t n) {
  int rc = check_plans(b, plans, n);
  if (rc) return rc;
  if (n == 0) return nhp::clear_error();
  if (!steps || !counts) return nhp::set_error(NHP_EINVAL, "steps or counts is NULL");
  std::vector<std::vector<nhp::Pass>> passes(n);
  size_t most = 0;
  for (uint32_t k = 0; k < n; k++) {
    nhp_plan* p = plans[k];
    if (!p->has_value) return nhp::set_error(NHP_ESTATE, "plans[%u] has no value volume (batch_init first)", k);
    nhp::schedule_passes(p->p.schedule, p->p.n_schedule, steps[k], counts[k], nhp::can_fuse(p->d), passes[k]);
    most = std::max(most, passes[k].size());
  }
  std::vector<nhp_plan*> live;
  std::vector<nhp::Pass> now;
  std::vector<nhp::SweepJob> table;
  std::vector<Launch> launches;
  for (size_t t = 0; t < most; t++) {
    live.clear();
    now.clear();
    for (uint32_t k = 0; k < n; k++)
      if (t < passes[k].size()) {
        live.push_back(plans[k]);
        now.push_back(passes[k][t]);
      }
    rc = add_pass(live.data(), now.data(), (uint32_t)live.size(), table, launches);
    if (rc) return rc;
  }
  rc = run_launches(b, table, launches);
  return rc ? rc : nhp::clear_error();
}

int batch_step(nhp_batch* b, nhp_plan* const* plans, const uint32_t* steps, uint32_t n) {
  int rc = check_plans(b, plans, n);
  if (rc) return rc;
  if (n == 0) return nhp::clear_error();
  if (!steps) return nhp::set_error(NHP_EINVAL, "steps is NULL");
  std::vector<nhp::Pass> now(n);
  for (uint32_t k = 0; k < n; k++) {
    nhp_plan* p = plans[k];
    if (!p->has_value) return nhp::set_error(NHP_ESTATE, "plans[%u] has no value volume (batch_init first)", k);
    now[k] = nhp::Pass{(int8_t)p->p.schedule[steps[k] % p->p.n_schedule], (int8_t)-1};
  }
  std::vector<nhp::SweepJob> table;
  std::vector<Launch> launches;
  rc = add_pass(plans, now.data(), n, table, launches);
  if (!rc) rc = run_launches(b, table, launches);
  return rc ? rc : nhp::clear_error();
}

int batch_sweep(nhp_batch* b, nhp_plan* const* plans, const uint32_t* starts_ijt, const uint32_t* n_cycles,
                uint32_t n) {
  int rc = check_plans(b, plans, n);
  if (rc) return rc;
  if (n == 0) return nhp::clear_error();
  if (!n_cycles) return nhp::set_error(NHP_EINVAL, "n_cycles is NULL");
  rc = batch_init(b, plans, starts_ijt, n);
  if (rc) return rc;
  // One batch_advance per cycle, with the passes sweep_n_turns would run: a
  // cycle's last sweep shares a pass with the next cycle's first when they
  // fuse and the plan goes on.  From the third cycle on, the cycles of the
  // same plans repeat the same launches, which run from a captured graph.
  uint32_t most = 0;
  for (uint32_t k = 0; k < n; k++) most = std::max(most, n_cycles[k]);
  std::vector<uint32_t> done(n, 0), skip(n, 0);
  std::vector<nhp_plan*> active;
  std::vector<uint32_t> steps, counts;
  std::vector<nhp::Pass> v;
  for (uint32_t c = 0; c < most; c++) {
    active.clear();
    steps.clear();
    counts.clear();
    for (uint32_t k = 0; k < n; k++) {
      if (c >= n_cycles[k]) continue;
      const nhp_plan* p = plans[k];
      const uint32_t m = p->p.n_schedule;
      const bool pair_next = c + 1 < n_cycles[k], pairs = nhp::can_fuse(p->d);
      v.clear();
      nhp::schedule_passes(p->p.schedule, (int)m, c * (uint64_t)m + skip[k], m - skip[k] + (pair_next ? 1 : 0), pairs,
                           v);
      const bool consumed = pair_next && pairs && !v.empty() && v.back().mu2 >= 0;
      active.push_back(plans[k]);
      steps.push_back(done[k]);
      counts.push_back(m - skip[k] + (consumed ? 1 : 0));
      done[k] += counts.back();
      skip[k] = consumed ? 1 : 0;
    }
    rc = batch_advance(b, active.data(), steps.data(), counts.data(), (uint32_t)active.size());
    if (rc) return rc;
  }
  return nhp::clear_error();
}

int batch_extract(nhp_batch* b, nhp_plan* const* plans, uint32_t n, const uint32_t* goals_ijt, const uint32_t* radius,
                  const uint32_t* w_xy_q10, const uint32_t* w_t_q10, nhp_step* h_steps, uint32_t cap_per_plan,
                  uint32_t* n_steps, int32_t* status, uint32_t* best_ijt, uint32_t* goal_value_q10,
                  uint32_t* score_q10) {
  int rc = check_plans(b, plans, n);
  if (rc) return rc;
  if (n == 0) return nhp::clear_error();
  if (!goals_ijt || !radius || !w_xy_q10 || !w_t_q10 || !n_steps || !status)
    return nhp::set_error(NHP_EINVAL, "a required array is NULL");
  if (cap_per_plan > 0 && !h_steps) return nhp::set_error(NHP_EINVAL, "h_steps is NULL");
  std::vector<nhp::ExArgs> args(n);
  for (uint32_t k = 0; k < n; k++) {
    nhp_plan* p = plans[k];
    if (!p->has_value) return nhp::set_error(NHP_ESTATE, "plans[%u]: extract before any sweep", k);
    const uint32_t gi = goals_ijt[3 * k], gj = goals_ijt[3 * k + 1], gt = goals_ijt[3 * k + 2];
    if (gi >= p->p.nx || gj >= p->p.nx || gt >= p->p.ntheta)
      return nhp::set_error(NHP_EINVAL, "goal of plans[%u] outside its grid", k);
    if (radius[k] > (uint32_t)nhp::kMaxRadius) return nhp::set_error(NHP_EINVAL, "goal radius of plans[%u] > 31", k);
    args[k] = nhp::ExArgs{p->d, p->start[0], p->start[1], p->start[2], gi, gj, gt, (int)radius[k], w_xy_q10[k],
                          w_t_q10[k], 0, p->n_starts};
  }
  // each plan's header and first kReadbackSteps steps come back in one copy
  // to the pinned slot; only longer paths need a second copy
  const size_t per_plan = nhp::kExHeader + (size_t)nhp::kReadbackSteps * nhp::kExStepWords;
  Slot* s;
  rc = take_slot(b, std::max(args.size() * sizeof(nhp::ExArgs), (size_t)n * per_plan * 4), &s);
  if (rc) return rc;
  memcpy(s->host, args.data(), args.size() * sizeof(nhp::ExArgs));
  HIP_TRY(hipMemcpyAsync(s->dev, s->host, args.size() * sizeof(nhp::ExArgs), hipMemcpyHostToDevice, b->stream),
          "job upload");
  HIP_TRY(nhp::launch_extract_batch(reinterpret_cast<const nhp::ExArgs*>(s->dev), (int)n, b->stream),
          "extract launch");
  // the pinned staging buffer now receives the results (the upload ahead of
  // them on the stream has been consumed by then)
  uint32_t* back = reinterpret_cast<uint32_t*>(s->host);
  for (uint32_t k = 0; k < n; k++)
    HIP_TRY(hipMemcpyAsync(back + (size_t)k * per_plan, plans[k]->d.extract, per_plan * 4,
                           hipMemcpyDeviceToHost, b->stream),
            "result copy");
  HIP_TRY(hipStreamSynchronize(b->stream), "result copy");
  std::vector<uint32_t> raw;
  for (uint32_t k = 0; k < n; k++) {
    const uint32_t* h = back + (size_t)k * per_plan;
    n_steps[k] = h[1];
    if (h[0] != 0) {
      status[k] = NHP_EUNREACH;
      continue;
    }
    if (best_ijt) memcpy(best_ijt + 3 * k, h + 2, 3 * sizeof(uint32_t));
    if (goal_value_q10) goal_value_q10[k] = h[5];
    if (score_q10) score_q10[k] = h[6];
    const uint32_t m = h[1];
    if (m > NHP_MAX_STEPS_DEVICE || m > cap_per_plan) {
      status[k] = NHP_ECAP;
      continue;
    }
    const uint32_t* steps = h + nhp::kExHeader;
    if (m > (uint32_t)nhp::kReadbackSteps) {
      raw.resize((size_t)m * nhp::kExStepWords);
      HIP_TRY(hipMemcpyAsync(raw.data(), plans[k]->d.extract + nhp::kExHeader, raw.size() * 4,
                             hipMemcpyDeviceToHost, b->stream),
              "result copy");
      HIP_TRY(hipStreamSynchronize(b->stream), "result copy");
      steps = raw.data();
    }
    nhp_step* out = h_steps + (size_t)k * cap_per_plan;
    for (uint32_t q = 0; q < m; q++) {  // device order is goal -> start
      const uint32_t* w = steps + (size_t)(m - 1 - q) * nhp::kExStepWords;
      nhp_step& o = out[q];
      memset(&o, 0, sizeof(o));
      o.maneuver = (uint8_t)w[0];
      o.steps = w[1];
      memcpy(o.from_ijt, w + 2, 3 * sizeof(uint32_t));
      memcpy(o.to_ijt, w + 5, 3 * sizeof(uint32_t));
      o.cost_q10 = w[8];
    }
    status[k] = NHP_OK;
  }
  rc = finish_slot(b, s);
  return rc ? rc : nhp::clear_error();
}

}  // extern "C"
