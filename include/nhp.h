/*
 * nhp.h -- C ABI of the MI355X kernel-style N-turn nonholonomic planner.
 *
 * The method is Nister, Soundararajan, Wang, Sane, "Nonholonomic Motion
 * Planning as Efficient as Piano Mover's" (arXiv 2306.01301).  The pipeline
 * of Sec. XI maps onto these calls:
 *   plan_create    graph and tables (Sec. V.C-D, eqs. 11-31)
 *   render_cspace  obstacle rendering (Sec. VI)
 *   sweep_n_turns  N cycles of the six maneuver kernels (Sec. VIII.B,
 *                  Insert 1; cycle order of Sec. XVI.A)
 *   extract_path   goal search (Sec. IX) and back-tracking (Sec. X, eq. 32)
 *
 * Conventions shared by every entry point:
 *   - Status: every function returning int returns NHP_OK (0) or a negative
 *     nhp_status; plan_last_error() then gives a message (thread-local).
 *     No C++ exception ever crosses this boundary.
 *   - Pointers named d_* are device pointers (HIP global memory on the
 *     plan's device); pointers named h_* are host pointers.  The library never
 *     frees memory it did not allocate.
 *   - Asynchrony: calls enqueue work on the plan's stream and return; only
 *     extract_path and plan_get_tables synchronise with it.
 *   - Volumes are laid out [theta][y][x] with x fastest: the pose (i, j, T)
 *     is element (T * nx + j) * nx + i.  Values are uint32 costs in 1/1024
 *     cell (NHP_INF = unreached); obstacle codes are uint8, 0..254 soft
 *     (slowness (256 + 4 code) / 256), 255 hard.
 *   - Concurrency: one plan must not be used from two threads at once;
 *     different plans are independent and may run concurrently on different
 *     streams.
 */
#ifndef NHP_H
#define NHP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NHP_INF 0xFFFFFFFFu
#define NHP_HARD 255u
#define NHP_MAX_STEPS_DEVICE 4096u /* back-tracking steps kept on the device */

typedef struct nhp_plan nhp_plan; /* opaque: tables, device state, stream */

enum nhp_status {
  NHP_OK = 0,
  NHP_EINVAL = -1,   /* invalid argument or parameter */
  NHP_ENOMEM = -2,   /* workspace too small or allocation failed */
  NHP_EHIP = -3,     /* a HIP runtime call failed */
  NHP_ESTART = -4,   /* the start pose is in collision */
  NHP_EUNREACH = -5, /* no reached, collision-free pose in the goal window */
  NHP_ECAP = -6,     /* the caller's step buffer is too small */
  NHP_ESTATE = -7    /* call out of order (e.g. sweep before render) */
};

/* The six maneuvers (Sec. V: LEFT/STRAIGHT/RIGHT x FORWARD/BACKWARD), in the
 * cycle order of Sec. XVI.A. */
enum nhp_maneuver { NHP_LF = 0, NHP_SF = 1, NHP_RB = 2, NHP_RF = 3, NHP_SB = 4, NHP_LB = 5 };

/* Problem parameters (Sec. IV-V).  Grid: nx x nx cells x ntheta headings,
 * theta(T) = 2 pi T / ntheta; one-cell hard walls at i = 0 and j = 0 make
 * the torus of Sec. V.C. */
typedef struct nhp_params {
  uint32_t nx;          /* cells per side; 16..1024, a multiple of 8 */
  uint32_t ntheta;      /* heading planes; 8..1024, a multiple of 8 */
  double turn_radius;   /* minimum turn radius R in cells, > 0 */
  uint32_t ct_q10[6];   /* transition cost into each maneuver, 1/1024 cell */
  uint32_t gear_q8[6];  /* edge-length multiplier per maneuver, 1/256 (256 = 1.0) */
  uint8_t schedule[6];  /* maneuver order within a cycle (default LF SF RB RF SB LB) */
  uint8_t n_schedule;   /* maneuvers per cycle, 1..6 (3 with LF SF RF = forward only) */
  uint8_t half_cell;    /* 1: half-cell vertex positions (eqs. 13-16); 0: plain rounding */
  uint8_t reserved[6];  /* zero */
} nhp_params;

/* One maneuver of an extracted plan: `steps` edges of `maneuver` from pose
 * from_ijt to pose to_ijt, costing cost_q10 (its transition cost plus the
 * weights of its edges). */
typedef struct nhp_step {
  uint8_t maneuver;
  uint8_t pad[3];
  uint32_t steps;
  uint32_t from_ijt[3];
  uint32_t to_ijt[3];
  uint32_t cost_q10;
} nhp_step;

/* Device bytes a plan needs for `params` (value volume 4 B/pose, obstacle
 * volume 1 B/pose, tables and scratch), or 0 when params are invalid. */
size_t plan_workspace_bytes(const nhp_params* params);

/* Builds the tables of eqs. (11)-(31) on the host and uploads them.
 * d_workspace: caller-owned device memory of at least plan_workspace_bytes()
 *   bytes, 256-byte aligned, alive until plan_destroy; NULL lets the library
 *   allocate (and free) it.
 * stream: hipStream_t the plan enqueues on (NULL = default stream).
 * Errors: NHP_EINVAL (params), NHP_ENOMEM (workspace too small), NHP_EHIP. */
int plan_create(const nhp_params* params, void* d_workspace, size_t workspace_bytes, void* stream,
                nhp_plan** out);

/* Frees the plan and any memory the library allocated for it.  Waits for the
 * plan's stream first.  NULL is accepted. */
int plan_destroy(nhp_plan* plan);

/* Replaces the stream the plan enqueues on. */
int plan_set_stream(nhp_plan* plan, void* stream);

/* Obstacle rendering (Sec. VI): puts the hard walls into row 0 and column 0
 * of the image, then for every heading plane takes the maximum code under the
 * vehicle box, a sideways pass over offsets -half_width..half_width along the
 * left normal followed by a lengthwise pass over -rear..front along the
 * heading.  d_image: nx * nx codes, row-major (row = y), device memory, read
 * only.  Box extents in cells from the rear axle, each 0..255.  Invalidates
 * any value volume (the value memory serves as scratch).
 * Errors: NHP_EINVAL, NHP_EHIP. */
int render_cspace(nhp_plan* plan, const uint8_t* d_image, int32_t front, int32_t rear,
                  int32_t half_width);

#define NHP_MAX_SOFT_TABLE 65536u

/* Soft obstacle costs (Sec. VI-VII: the reciprocal of the highest allowed
 * velocity is a function of the distance to the nearest hard obstacle): for
 * an nx*nx image of codes (device), d_out[j*nx+i] = 255 where the image is
 * 255, else h_table[min(d2, table_len - 1)], d2 the squared Euclidean
 * distance in cells to the nearest pixel coded 255 (unbounded when there is
 * none).  1 <= table_len <= NHP_MAX_SOFT_TABLE.  d_out and d_image must not
 * overlap.  Uses the value volume's memory
 * as scratch (a later extract needs a new sweep); synchronises. */
int soft_cost_image(nhp_plan* plan, const uint8_t* d_image, uint8_t* d_out, const uint8_t* h_table,
                    uint32_t table_len);

/* Loads an obstacle volume (nx*nx*ntheta codes, device memory) in place of
 * rendering; the walls at i = 0 and j = 0 are forced hard afterwards. */
int plan_set_cspace(nhp_plan* plan, const uint8_t* d_cspace);

/* Sets V = NHP_INF everywhere and V(start) = 0, then runs n_cycles cycles of
 * the schedule, each maneuver kernel relaxing every pose once (Insert 1; turn
 * curves are cyclic and closed exactly, straights start at the wall).  Two
 * consecutive turn maneuvers on the same circles in opposite directions
 * (RB, RF or LB, LF in either order, also the last of one cycle and the
 * first of the next) share one pass over the volume, with the result of
 * running them one after the other.
 * Errors: NHP_ESTATE (no obstacle volume), NHP_EINVAL, NHP_ESTART (start in
 * collision; checked on the host, which synchronises once), NHP_EHIP. */
int sweep_n_turns(nhp_plan* plan, uint32_t si, uint32_t sj, uint32_t st, uint32_t n_cycles);

/* A start of a start set (Sec. III.A: start states with a cost depending on
 * where the plan begins; Sec. XII: a maneuver already in progress).
 * maneuver = -1: the vehicle is at rest at (i, j, T) with cost cost_q10 and
 * may begin any scheduled maneuver there (paying its transition cost).
 * maneuver = 0..5: that maneuver is in progress at (i, j, T); it continues
 * without a transition cost, so every pose it reaches along its curve (up to
 * the first pose in collision; one loop for turns, the end of the line for
 * straights) starts at cost_q10 plus the edge sum from (i, j, T). */
typedef struct {
  uint32_t i, j, T;
  uint32_t cost_q10;
  int32_t maneuver;
} nhp_start;

#define NHP_MAX_STARTS 64u
#define NHP_MAX_GOALS 4096u

/* Like sweep_n_turns from a start set of n_starts (1..NHP_MAX_STARTS)
 * entries: V = NHP_INF, every start (and every pose of a maneuver in
 * progress) lowered to its cost, then n_cycles cycles.  extract_path and
 * extract_path_set then end a plan at the first start-set pose (in start
 * order, then along the maneuver in progress) whose value equals its start
 * cost; a maneuver in progress becomes the plan's first step (cost: its
 * edge sum, no transition).  Errors: NHP_EINVAL, NHP_ESTART (a start pose in
 * collision), NHP_ESTATE, NHP_EHIP. */
int sweep_from_set(nhp_plan* plan, const nhp_start* h_starts, uint32_t n_starts, uint32_t n_cycles);

/* Runs n_more_cycles further cycles on the current value volume without
 * re-initialising it (sweep_n_turns(a) then sweep_resume(b) equals
 * sweep_n_turns(a + b)).  Errors: NHP_ESTATE. */
int sweep_resume(nhp_plan* plan, uint32_t n_more_cycles);

/* One maneuver kernel (Insert 1 over every curve of `maneuver`) on the
 * current value volume, whatever it holds.  Errors: NHP_ESTATE, NHP_EINVAL. */
int sweep_one(nhp_plan* plan, uint32_t maneuver);

/* Maneuver `first` then maneuver `second` (-1: none) on the current value
 * volume.  When the two are turns on the same circles in opposite directions
 * and the plan's curves fit the fused kernel, both run in one pass (one read
 * and one write per pose); otherwise as two sweep_one calls.  Same result
 * either way.  Errors: NHP_ESTATE, NHP_EINVAL. */
int sweep_pass(nhp_plan* plan, int32_t first, int32_t second);

/* The straight maneuver `maneuver` (NHP_SF or NHP_SB; Insert 1 over the
 * lines of eqs. 29-31) on the heading planes of one family of eq. (19)
 * only: family 1 = the planes whose lines advance one row per step (|tan
 * theta| > 1), family 0 = one column per step.  The families hold disjoint
 * planes, so both, in either order, equal sweep_one(maneuver); each family
 * is a single kernel launch, so events around the calls time each kernel.
 * Errors: NHP_ESTATE, NHP_EINVAL. */
int sweep_straight_family(nhp_plan* plan, uint32_t maneuver, uint32_t family);

/* Host only (no device work): the passes that sweeps n_steps sweeps of a
 * schedule starting at sweep number first_step (sweep k applies
 * schedule[k % n_schedule]) are grouped into, as sweep_n_turns and
 * batch_advance group them: with pairs != 0, consecutive turns on the same
 * circles in opposite directions share a pass, paired greedily from the
 * first.  Pass k is first[k] then second[k] (-1: none).  *n_passes is always
 * set; NHP_ECAP when it exceeds cap (arrays untouched), NHP_EINVAL for a bad
 * schedule. */
int schedule_passes(const uint8_t* schedule, uint32_t n_schedule, uint64_t first_step, uint64_t n_steps,
                    int32_t pairs, int8_t* first, int8_t* second, uint32_t cap, uint32_t* n_passes);

/* Goal search (Sec. IX) then back-tracking (Sec. X, eq. 32), both on the
 * device; only the plan crosses to the host.
 * Goal window: poses within max-norm `radius` (0..31) of (gi, gj, gt), each
 * coordinate modulo its dimension; in-collision and unreached poses are
 * skipped; score = V + w_xy_q10 (|dx| + |dy|) + w_t_q10 |dT| (saturating);
 * ties go to the smaller (|dx|+|dy|+|dT|, dT, dy, dx).
 * Back-tracking: from the best pose, for every scheduled maneuver every pose
 * p_k up its curve through the current pose is a candidate worth
 * V(p_k) + ct + (edge weights from p_k to the current pose); the smallest
 * (value, schedule position, k) becomes the current pose, until the start.
 * h_steps: host array of `cap` steps, filled start -> goal; *n_steps gets the
 * plan length (also on NHP_ECAP).  best_ijt (3 entries), goal_value_q10
 * (V at the best pose) and score_q10 may be NULL.  Synchronises the stream.
 * Errors: NHP_ESTATE (no sweep yet), NHP_EINVAL, NHP_EUNREACH, NHP_ECAP,
 * NHP_EHIP. */
int extract_path(nhp_plan* plan, uint32_t gi, uint32_t gj, uint32_t gt, uint32_t radius,
                 uint32_t w_xy_q10, uint32_t w_t_q10, nhp_step* h_steps, uint32_t cap,
                 uint32_t* n_steps, uint32_t* best_ijt, uint32_t* goal_value_q10,
                 uint32_t* score_q10);

/* For callers that cannot allocate (code under graph capture, tight serving
 * loops, harnesses that forbid allocation): extract_path with the same
 * arguments, results and errors, but this call allocates nothing, neither
 * device nor pinned host memory.  Its extract area (result header, the step
 * list of up to NHP_MAX_STEPS_DEVICE steps, the back-tracking kernel's
 * barrier counter and exchange words: NHP_NOALLOC_EXTRACT_BYTES bytes) is a
 * fixed device array of the library, one per GPU, held until the process
 * ends; its size does not depend on the grid, so every plan fits (a walk
 * longer than NHP_MAX_STEPS_DEVICE steps is NHP_EUNREACH, as in
 * extract_path).  The steps are copied straight into h_steps.  All calls on
 * one GPU share that GPU's area: calls that overlap on one GPU (two threads,
 * or two streams) race and must be serialised by the caller.  Synchronises
 * the plan's stream. */
#define NHP_NOALLOC_EXTRACT_BYTES ((16u + NHP_MAX_STEPS_DEVICE * 9u + 49u) * 4u)
int extract_path_noalloc(nhp_plan* plan, uint32_t gi, uint32_t gj, uint32_t gt, uint32_t radius,
                         uint32_t w_xy_q10, uint32_t w_t_q10, nhp_step* h_steps, uint32_t cap,
                         uint32_t* n_steps, uint32_t* best_ijt, uint32_t* goal_value_q10,
                         uint32_t* score_q10);

/* Goal set with penalties (Sec. IX: the criterion is the reward of the
 * final vertex minus the cost to get there; a reward is passed as its
 * shortfall from the largest reward, so penalty_q10 >= 0): the goal k
 * (0 <= k < n_goals <= NHP_MAX_GOALS, goals_ijt[3k..]) minimising
 * V + penalty (saturating) among goals that are free and reached, ties to
 * the earlier goal; then back-tracking as extract_path.  *best_index = k,
 * *goal_value_q10 = V(goal k), *score_q10 = V + penalty.  Errors as
 * extract_path. */
int extract_path_set(nhp_plan* plan, const uint32_t* goals_ijt, const uint32_t* penalty_q10, uint32_t n_goals,
                     nhp_step* h_steps, uint32_t cap, uint32_t* n_steps, uint32_t* best_index,
                     uint32_t* goal_value_q10, uint32_t* score_q10);

/* Device pointers of the plan's value and obstacle volumes (for parity
 * checks and checkpoints; owned by the plan).  Either output may be NULL. */
int plan_device_ptrs(const nhp_plan* plan, uint32_t** d_value, uint8_t** d_cspace);

/* Copies the host tables out (each host array may be NULL):
 *   beta[ntheta], psi[ntheta]            eq. (13); psi in half cells
 *   family[ntheta], fwd_sign[ntheta]     eqs. (19), (24)
 *   skew[ntheta * nx]                    B(y', T) of eq. (22), [T][y']
 *   edge_len[6 * ntheta]                 edge length per maneuver and plane,
 *                                        1/1024 cell, gear applied, [mu][T] */
int plan_get_tables(const nhp_plan* plan, int32_t* beta, int32_t* psi, int32_t* family,
                    int32_t* fwd_sign, int32_t* skew, uint32_t* edge_len);

/* ------------------------------------------------------------------------
 * Batched execution.  A batch drives many plans with shared launches: one
 * launch per pass covers the current work of every listed plan (tiles of all
 * plans in one grid), so small plans fill the GPU together and a plan that
 * joins later runs alongside plans that are further along (continuous
 * batching).  Work is enqueued on the batch's stream; work the plans have on
 * other streams must be complete.  A plan may appear once per call.  Job
 * tables live in a ring of 4 pinned/device buffer pairs owned by the batch;
 * a call waits only when it reuses a buffer whose launches are still queued.
 * Every entry point returns a status; plan_last_error() explains failures.
 * ------------------------------------------------------------------------ */
typedef struct nhp_batch nhp_batch;

/* A batch for up to `capacity` plans per call, enqueueing on `stream`. */
int batch_create(uint32_t capacity, void* stream, nhp_batch** out);

/* Waits for the batch's stream and frees its buffers (NULL accepted). */
int batch_destroy(nhp_batch* batch);

/* Obstacle rendering (as render_cspace) of n plans in two launches.
 * d_images[k]: plan k's image (device); boxes_frs[3k..3k+2]: its box. */
int batch_render(nhp_batch* batch, nhp_plan* const* plans, const uint8_t* const* d_images,
                 const int32_t* boxes_frs, uint32_t n);

/* V = NHP_INF and V(start) = 0 for n plans in one launch (starts_ijt[3k..]).
 * Errors: NHP_ESTATE, NHP_EINVAL, NHP_ESTART (checked on the host). */
int batch_init(nhp_batch* batch, nhp_plan* const* plans, const uint32_t* starts_ijt, uint32_t n);

/* One tick of continuous batching: plan k runs its sweep number steps[k],
 * i.e. maneuver schedule[steps[k] % n_schedule] (Insert 1), all plans in
 * at most five launches (turn and y-major straight tiles grouped by section
 * size, x-major straight tiles).  Errors: NHP_ESTATE (no batch_init or
 * sweep_n_turns yet), NHP_EINVAL. */
int batch_step(nhp_batch* batch, nhp_plan* const* plans, const uint32_t* steps, uint32_t n);

/* Several ticks at once: plan k runs its sweeps steps[k] .. steps[k] +
 * counts[k] - 1 (counts[k] = 0: none).  A call whose launches repeat those
 * of an earlier call on this batch (the same plans at the same points of
 * their schedules, under the same knobs) is captured into a HIP graph the
 * second time and replayed after that; the batch keeps up to 16 such graphs,
 * each with its own device copy of its job table.  Consecutive turn sweeps on the same
 * circles in opposite directions (RB then RF, LB then LF, and the reverse
 * orders) share one pass over the volume, with the same result as two
 * batch_step calls; pass t of every plan goes into shared launches (at most
 * nine per pass).  Errors as batch_step. */
int batch_advance(nhp_batch* batch, nhp_plan* const* plans, const uint32_t* steps, const uint32_t* counts,
                  uint32_t n);

/* batch_init, then one batch_advance per cycle (the plans with cycles
 * left, each with the passes sweep_n_turns runs: a cycle's last sweep shares
 * a pass with the next cycle's first when they fuse): plan k ends with
 * n_cycles[k] cycles, as sweep_n_turns would leave it.  Cycles that repeat
 * the launches of an earlier one replay them from a captured graph. */
int batch_sweep(nhp_batch* batch, nhp_plan* const* plans, const uint32_t* starts_ijt,
                const uint32_t* n_cycles, uint32_t n);

/* Goal search and back-tracking (as extract_path) for n plans in one launch,
 * one workgroup per plan.  Per plan k: goal goals_ijt[3k..], radius[k],
 * weights w_xy_q10[k], w_t_q10[k]; results status[k] (NHP_OK, NHP_EUNREACH
 * or NHP_ECAP), n_steps[k], steps in h_steps[k * cap_per_plan ...] start ->
 * goal, and (optional arrays) best_ijt[3k..], goal_value_q10[k],
 * score_q10[k].  Synchronises the batch's stream.  The call returns NHP_OK
 * when it ran, whatever the per-plan statuses. */
int batch_extract(nhp_batch* batch, nhp_plan* const* plans, uint32_t n, const uint32_t* goals_ijt,
                  const uint32_t* radius, const uint32_t* w_xy_q10, const uint32_t* w_t_q10,
                  nhp_step* h_steps, uint32_t cap_per_plan, uint32_t* n_steps, int32_t* status,
                  uint32_t* best_ijt, uint32_t* goal_value_q10, uint32_t* score_q10);

/* Tuning: the number of steps each wave of a sweep workgroup holds for
 * curves of length `curve_len` (ntheta for turns, nx for straights): 8, 16,
 * 32 or 64 with ceil(curve_len / steps) <= 16; 0 restores the built-in
 * choice.  Process-wide; plans that already captured their cycle graph keep
 * the choice they captured.  Every valid choice gives identical results and
 * only changes speed (the autotuner measures them).  Errors: NHP_EINVAL. */
int nhp_set_section_steps(uint32_t curve_len, uint32_t steps);

/* Launch-shape knobs of the sweep kernels, process-wide, for the autotuner:
 * 0 restores the built-in choice.  Every setting gives identical results and
 * only changes speed.  Plans that already captured their cycle graph keep
 * the launches they captured. */
enum nhp_knob {
  NHP_KNOB_ROW_WG_PER_CU = 0,    /* workgroups per compute unit that the row sweep launches keep resident, 1..8 */
  NHP_KNOB_XMAJOR_WG_PER_CU = 1, /* workgroups per compute unit in the grid of the x-major straight launches,
                                    1..16; built-in: 16 for grids of at least 32 cells (one workgroup per tile
                                    up to 4096 tiles, 5 resident per compute unit), 6 below */
  NHP_KNOB_TILE_ORDER = 2,       /* 1: tiles that share row segments run on one XCD (its L2); 2: launch order */
  NHP_KNOB_XMAJOR_BUFFERS = 3    /* x-major LDS tiles per workgroup: 2 (the next chunk's loads need no barrier
                                    after the stores) or 1 (more workgroups fit a compute unit); built-in: 1 for
                                    grids of at least 32 cells (band tiles), 2 below */
};
/* Errors: NHP_EINVAL (unknown knob or value out of range). */
int nhp_set_knob(uint32_t knob, int32_t value);
/* The knob's value (0 = built-in), -1 for an unknown knob. */
int32_t nhp_get_knob(uint32_t knob);

/* Message of the last failing call on this thread ("" if none). */
const char* plan_last_error(void);

/* ---------------------------------------------------------------------
 * Reachability by maneuver count (App. C, Insert 2; Sections of App. D).
 * Hard obstacles only (image code 255; every other code is free), every
 * maneuver costs one and moves cost nothing: bit volumes say, per pose,
 * whether it can be reached with at most m maneuvers, for m = 0..n_cycles.
 * Bit layout: 32-bit word ((T * nx + j) * nx/32 + i/32), bit i % 32; in the
 * level volumes a set bit means NOT reachable (the paper's convention), in
 * the obstacle volume a set bit means hard.  Each cycle applies every
 * scheduled maneuver to R_m and ANDs the results into R_{m+1}; the schedule
 * order does not matter.  The state uses its plan's tables and stream; it
 * must be destroyed before the plan.
 * ------------------------------------------------------------------- */
typedef struct nhp_reach nhp_reach;

/* Device bytes of a reachability state keeping max_cycles + 1 level volumes
 * (nx^2 ntheta / 8 bytes each) plus the obstacle bits; 0 when the sizes are
 * not supported (nx a multiple of 32 in [32, 512], ntheta <= 512, 1 <=
 * max_cycles <= 254). */
size_t reach_workspace_bytes(const nhp_params* params, uint32_t max_cycles);

/* d_workspace: 256-byte aligned device memory of at least
 * reach_workspace_bytes, or NULL for a library allocation.  Errors:
 * NHP_EINVAL (sizes, workspace), NHP_ENOMEM. */
int reach_create(nhp_plan* plan, uint32_t max_cycles, void* d_workspace, size_t workspace_bytes,
                 nhp_reach** out);
int reach_destroy(nhp_reach* reach);

/* Obstacle bits: the hard cells of the image (nx*nx codes, device memory)
 * dilated by the vehicle box exactly as render_cspace does (so a pose is
 * hard here exactly when render_cspace gives it code 255); walls at i = 0
 * and j = 0 hard. */
int reach_render(nhp_reach* reach, const uint8_t* d_image, int32_t front, int32_t rear, int32_t half_width);

/* Obstacle bits from an obstacle code volume (device, nx*nx*ntheta codes;
 * 255 = hard), walls forced hard. */
int reach_set_cspace(nhp_reach* reach, const uint8_t* d_codes);

/* R_0 = {start}, then n_cycles cycles (n_cycles <= max_cycles).  Errors:
 * NHP_ESTATE (no obstacle bits), NHP_EINVAL, NHP_ESTART (start hard;
 * checked on the host, which synchronises once). */
int reach_sweep(nhp_reach* reach, uint32_t si, uint32_t sj, uint32_t st, uint32_t n_cycles);

/* Goal search and back-tracking on the levels: within max-norm radius of the
 * goal (coordinates modulo their dimension) the pose with the smallest
 * (level, |dx|+|dy|+|dT|, dT, dy, dx); then from a pose of level m, for the
 * scheduled maneuvers in schedule order, the nearest pose up the curve
 * (through free poses) of level m - 1, until level 0.  *level = the best
 * pose's level = the number of steps (each cost_q10 = 1).  Synchronises.
 * Errors: NHP_EUNREACH, NHP_ECAP (*n_steps still set), NHP_EINVAL,
 * NHP_ESTATE. */
int reach_extract(nhp_reach* reach, uint32_t gi, uint32_t gj, uint32_t gt, uint32_t radius, nhp_step* h_steps,
                  uint32_t cap, uint32_t* n_steps, uint32_t* best_ijt, uint32_t* level);

/* Device pointers of the obstacle bits and of level volume 0 (volume m
 * follows at m * nx^2 ntheta / 32 words), for checking and checkpoints. */
int reach_device_ptrs(const nhp_reach* reach, uint32_t** d_hard, uint32_t** d_levels);

#ifdef __cplusplus
}
#endif
#endif /* NHP_H */
