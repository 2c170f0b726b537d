// nhp_internal.h -- private declarations of the HIP planner library.
// Shared only by the library's own translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <memory>
#include <string>
#include <vector>

#include "nhp.h"

namespace nhp {

constexpr uint32_t kInf = NHP_INF;
constexpr uint32_t kHard = NHP_HARD;
constexpr int kMaxTaps = 512;        // per pass: 2*half_width+1 and front+rear+1 are <= 511
constexpr int kMaxRadius = 31;       // goal window radius
constexpr uint32_t kMaxLq = 1u << 21;  // keeps Lq * 1276 + 128 below 2^32

// Host copy of the tables of eqs. (11)-(31), built once per plan.
struct HostTables {
  std::vector<int32_t> beta, psi, family, fwd;
  std::vector<uint32_t> edge_len;  // [mu][T], Q10, gear applied
  // [T][y'] signed B(y', T) (|B| < nx <= 1024); depends on (nx, ntheta) only
  // and is shared by every plan of that shape in the process
  std::shared_ptr<const std::vector<int16_t>> skew16;
  // derived device layouts
  std::vector<int32_t> turn_off;  // [4][T]: LEFT x, LEFT y, RIGHT x, RIGHT y, reduced mod nx
  std::vector<int32_t> planes_x;  // heading planes of the x-major straight family (I = 0)
  std::vector<int32_t> planes_y;  // heading planes of the y-major straight family (I = 1)
};

int build_tables(const nhp_params& p, HostTables& t);
void render_taps_host(const nhp_params& p, const HostTables& t, int T, int front, int rear, int half_width,
                      int32_t* side_packed, int32_t* len_packed);
double grid_sin(int nt, long T);
double grid_cos(int nt, long T);

// Device-side view of a plan (plain pointers, passed to the launchers).
struct DevPlan {
  int nx, nt;
  uint32_t* V;           // value volume, N_R uint32
  uint8_t* B;            // obstacle volume, N_R codes
  int32_t* turn_off;     // [4][nt]
  int16_t* skew;         // [nt][nx]
  uint32_t* edge_len;    // [6][nt]
  int32_t* fwd;          // [nt]
  int32_t* family;       // [nt]
  int32_t* planes;       // planes_x then planes_y
  int n_planes_x, n_planes_y;
  int32_t* taps;         // [nt][n_side + n_len] packed (dx & 0xffff) | (dy << 16): side then length
  uint32_t* extract;     // result header + steps
  nhp_start* starts;     // start set (NHP_MAX_STARTS entries)
  uint32_t* seeds;       // per start, seed_slots entries of kSeedWords words
  uint32_t* goals;       // goal set: NHP_MAX_GOALS entries of (i, j, T, penalty)
  int seed_slots;        // slots per start: max(nx, nt)
  uint32_t ct[6];
  uint32_t turn_lq[6];   // host copy of the (plane-independent) turn edge lengths
  uint8_t schedule[6];
  int n_schedule;
};

// One maneuver of one plan, as the sweep kernels see it.  Row jobs cover
// turn curves (cyclic) or the y-major straight planes; x-major jobs cover
// the x-major straight planes.  Plain pointers and integers only, so job
// tables can be copied to the device for batched launches.
struct SweepJob {
  uint32_t* V;
  const uint8_t* B;
  const int32_t* offx;      // turns: offsets of this maneuver's curves (reduced mod N)
  const int32_t* offy;
  const int16_t* skew;      // straights: B(y', T)
  const int32_t* planes;    // straights: heading planes of this job's family
  const uint32_t* edge_len; // straights: this maneuver's edge lengths per plane
  const int32_t* fwd;       // straights: forward signs
  int N, L;                 // grid side, curve length
  uint32_t n_poses;         // poses of the volume (N N headings)
  int cyclic, dir, mu_forward;
  int tiles_x, blocks, first_block;
  int order;                // tile order: 1 = tiles sharing row segments on one XCD, 2 = launch order
  int P;                    // steps per wave (row jobs)
  uint32_t ct, lq;          // transition cost; turn edge length
  // Turns only: a second maneuver on the same circles in the opposite
  // direction, applied right after the first while the curves are in
  // registers (fused = 1); its transition cost and edge length.
  int fused;
  uint32_t ct2, lq2;
};

// A pass over the value volume: one maneuver, or two consecutive turn
// maneuvers that share their curves (mu2 >= 0).
struct Pass {
  int8_t mu, mu2;
};

// Whether `b` right after `a` can share one pass: both turns on the same
// circles (left: LF, LB; right: RF, RB) in opposite directions.
inline bool fusable(int a, int b) {
  const bool la = a == NHP_LF || a == NHP_LB, lb = b == NHP_LF || b == NHP_LB;
  const bool ra = a == NHP_RF || a == NHP_RB, rb = b == NHP_RF || b == NHP_RB;
  return a != b && ((la && lb) || (ra && rb));
}

// The passes of `count` consecutive sweeps of a schedule starting at step
// `first` (step k applies schedule[k mod n]); with `pairs`, consecutive
// fusable sweeps are paired greedily from the first.  Appends to `out`.
void schedule_passes(const uint8_t* schedule, int n, uint64_t first, uint64_t count, bool pairs,
                     std::vector<Pass>& out);

// Whether a plan's turn curves have a section size (then consecutive turns
// on shared circles run as one pass).
bool can_fuse(const DevPlan& d);

struct InitJob {
  uint32_t* V;
  size_t n4;       // poses / 4
  uint32_t start;  // start pose index
  uint32_t pad;
};

int pick_section(int len);
int set_section_steps(int len, int P);
// Launch-shape knobs (enum nhp_knob of nhp.h): set_knob checks the range,
// get_knob returns the value (0 = built-in) or -1.
constexpr int kKnobs = 4;
int set_knob(int knob, int value);
int get_knob(int knob);
int make_sweep_jobs(const DevPlan& d, Pass pass, SweepJob* row, SweepJob* xmaj);
// Whether x-major jobs of grid side N take the 4-column-load kernel (batched
// x-major launches group their jobs by it and pass it as `pow2`).
bool xmajor_wide(int N);
int xmajor_lines(int N);  // lines per x-major tile
// Row jobs of one launch share P, fused, guard (= L % P != 0) and their
// wave count (the workgroup size is 64 waves threads); x-major jobs of one
// launch share xmajor_wide(N), passed as pow2.
hipError_t launch_sweep_batch(const SweepJob* d_jobs, int n_jobs, int total_blocks, int P, bool fused, bool guard,
                              bool pow2, bool xmajor, int waves, hipStream_t s);
hipError_t launch_init_batch(const InitJob* d_jobs, int n_jobs, size_t max_n4, hipStream_t s);

// extract buffer layout (uint32 words)
constexpr int kExHeader = 16;  // status, n_steps, best i, j, T, V(best), score, best goal index, ...
constexpr int kExStepWords = 9;
constexpr int kReadbackSteps = 256;  // steps read back with the header in one copy
// after the steps: a barrier counter and, per step parity and schedule
// position, the best candidate key (2 words), its pose's value and the cost
constexpr int kExSyncWords = 1 + 2 * 6 * 4;
// seed entry: pose index (kNoSeed when unused), value, start index, edges along its maneuver
constexpr int kSeedWords = 4;
constexpr uint32_t kNoSeed = 0xFFFFFFFFu;

// Writes the seeds of n starts (init must have set V to INF before).
hipError_t launch_seed(const DevPlan& d, int n_starts, hipStream_t s);

hipError_t launch_init(const DevPlan& d, uint32_t start_index, hipStream_t s);
hipError_t launch_force_walls(const DevPlan& d, hipStream_t s);
hipError_t launch_sweep(const DevPlan& d, Pass pass, hipStream_t s);
// Part of a pass: parts bit 0 = the row kernel (turn curves, or the y-major
// straight planes), bit 1 = the x-major straight planes.
hipError_t launch_sweep_part(const DevPlan& d, Pass pass, int parts, hipStream_t s);
hipError_t launch_render(const DevPlan& d, const uint8_t* image, int n_side, int n_len, hipStream_t s);
hipError_t launch_extract(const struct ExArgs& x, hipStream_t s);

// Goal search and back-tracking arguments of one plan.
struct ExArgs {
  DevPlan d;
  uint32_t si, sj, st, gi, gj, gt;
  int radius;
  uint32_t w_xy, w_t;
  int n_goals;   // > 0: goal set in d.goals instead of the window
  int n_starts;  // > 0: the plan ends at a seed of the start set in d.seeds
};
hipError_t launch_extract_batch(const ExArgs* d_args, int n, hipStream_t s);
// Words of one extract area (header, steps, barrier counter, exchange area).
constexpr size_t kNoAllocExtractWords = kExHeader + (size_t)NHP_MAX_STEPS_DEVICE * kExStepWords + kExSyncWords;
static_assert(kNoAllocExtractWords * 4 == NHP_NOALLOC_EXTRACT_BYTES, "the header states the area's size");
// Device address of the file-scope extract area on `device` (looked up on
// the first call per device; no allocation).
hipError_t noalloc_extract_area(int device, uint32_t** out);

// Rendering of one plan: sideways pass from the image into `side`, then the
// lengthwise pass into B.  Batched launches list several plans.
struct RenderJob {
  const uint8_t* image;
  uint8_t* side;  // scratch: 2 N^2 nt + 2 N^2 bytes (the value volume's memory)
  uint8_t* B;
  const int32_t* taps;
  int N, nt, n_side, n_len;
  int blocks, first_block;
  int pad_first;  // batched: first padded-image row block of this job
};
hipError_t launch_render_batch(const RenderJob* d_jobs, int n_jobs, int total_blocks, int total_pad_rows,
                               hipStream_t s);
int render_blocks(int N, int nt);  // workgroups of one plan's render passes
// Soft costs of an n x n image; g_scratch: n^2 words.
hipError_t launch_soft_costs(const uint8_t* image, uint32_t* g_scratch, const uint8_t* table, uint32_t len,
                             uint8_t* out, int n, hipStream_t s);

// ---- maneuver-count reachability (App. C) ----
// Bit volumes: word ((T * N + j) * W + w), W = N / 32, bit t is pose
// i = 32 w + t.  A set bit means "not reachable" in a level volume (the
// paper's inverted convention, so a sweep step is an AND then an OR) and
// "hard" in the obstacle bit volume.
constexpr int kReachMaxN = 512;
constexpr int kReachMaxL = 512;
constexpr uint32_t kReachMaxCycles = 254;
constexpr int kReachMaxSteps = 256;

struct ReachDev {
  int N, L, W;
  const int32_t* turn_off;  // the plan's [4][L]
  const int16_t* skew;      // [L][N]
  const int32_t* family;    // [L]
  const int32_t* fwd;       // [L]
  const int32_t* taps;      // [L][n_side + n_len], side then length
  uint32_t* hard;           // obstacle bits, one volume
  uint32_t* levels;         // level volumes R_0 .. R_max
  uint32_t* img;            // [N][W] image bits (rendering scratch)
  uint32_t* extract;        // header + steps
  size_t vol_words;         // N * N * L / 32
};

hipError_t launch_reach_render(const ReachDev& r, const uint8_t* image, int n_side, int n_len, hipStream_t s);
hipError_t launch_reach_pack(const ReachDev& r, const uint8_t* codes, hipStream_t s);
hipError_t launch_reach_start(const ReachDev& r, uint32_t start_index, hipStream_t s);
// One cycle: R_{m+1} from R_m with the scheduled maneuvers (at most three
// launches: left circles, right circles, straight planes).
hipError_t prepare_reach_kernels();
hipError_t launch_reach_cycle(const ReachDev& r, const uint8_t* schedule, int n_schedule, uint32_t m, hipStream_t s);

struct ReachExArgs {
  DevPlan d;  // tables for the curve geometry (predecessors)
  const uint32_t* hard;
  const uint32_t* levels;
  size_t vol_words;
  int W;
  int n_levels;  // level volumes computed (cycles + 1)
  uint32_t gi, gj, gt;
  int radius;
  uint32_t* out;
};
hipError_t launch_reach_extract(const ReachExArgs& x, hipStream_t s);

}  // namespace nhp

// The plan object behind the opaque handle of the C ABI.
struct nhp_plan {
  nhp_params p{};
  hipStream_t stream = nullptr;
  int device = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool own_ws = false;
  nhp::HostTables t;
  nhp::DevPlan d{};
  bool has_cspace = false;
  bool has_value = false;
  uint32_t start[3] = {0, 0, 0};
  int front = -1, rear = -1, half_width = -1;  // box of the last render (sample offsets cached)
  // One cycle of the schedule, captured once and replayed per cycle; indexed
  // by [first sweep already done by the previous cycle's last pass][last
  // sweep may pair with the next cycle's first].
  hipGraphExec_t cycle[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  int n_starts = 0;  // > 0: the value volume was seeded from a start set
  bool graph_failed = false;  // capture unavailable: launch the kernels directly
  uint32_t multi_cycle_runs = 0;  // sweeps of more than one cycle so far (graphs from the second on)
  uint32_t* readback = nullptr;  // pinned: extract header and the first kReadbackSteps steps
};

namespace nhp {
// Thread-local error text of the C ABI (nhp_api.cpp).
int set_error(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int clear_error();
int upload_taps(nhp_plan* plan, int front, int rear, int half_width);
// Checks a vehicle box; the sample offsets of all planes then take
// taps_words() words, written by build_taps into `out`.
int check_box(int front, int rear, int half_width);
size_t taps_words(const nhp_plan* plan, int front, int rear, int half_width);
void build_taps(const nhp_plan* plan, int front, int rear, int half_width, int32_t* out);
}  // namespace nhp
