// k_extract.hip -- goal search (Sec. IX) and back-tracking (Sec. X, eq. 32)
// in one kernel, so the value volume never leaves the device and the serial
// back-tracking loop pays no launch per step.  A single plan uses one
// workgroup per scheduled maneuver, joined by a grid-wide barrier per step;
// a batch uses one workgroup per plan.
//
// Back-tracking step ("Bellman iteration in reverse"): for every scheduled
// maneuver mu, thread t examines the pose p_k, k = t + 1, up the mu-curve
// through the current pose; a block-wide saturating prefix sum gives the
// edge sum E_k from p_k to the current pose, the candidate is
// V(p_k) + ct_mu + E_k, and a block-wide minimum of the packed key
// (candidate, schedule position, k) picks the next pose.  Curves are at most
// 1024 poses long, so one thread per candidate suffices.
#include <mutex>

#include "nhp_internal.h"

namespace nhp {
namespace {

constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / 64;

__device__ __forceinline__ uint32_t sadd(uint32_t a, uint32_t b) { return __builtin_elementwise_add_sat(a, b); }

// v mod n for any v (goal window coordinates, once per candidate)
__device__ __forceinline__ int modn(int v, int n) {
  const int r = v % n;
  return r < 0 ? r + n : r;
}

// v mod n for v in [-2n, 3n): the back-tracking callers add or subtract at
// most two values below n (table offsets are reduced, skews are below n, k < L)
__device__ __forceinline__ int wrapn(int v, int n) {
  v += (v < 0) ? n : 0;
  v += (v < 0) ? n : 0;
  v -= (v >= n) ? n : 0;
  v -= (v >= n) ? n : 0;
  return v;
}

__device__ __forceinline__ uint32_t weight(uint32_t code, uint32_t Lq) {
  if (code == kHard) return kInf;
  return (uint32_t)(((uint64_t)Lq * (256u + 4u * code) + 128u) >> 8);
}

// Inclusive saturating prefix sums over the block (NW waves) of M values per
// thread at once (one per scheduled maneuver): thread k gets, for each m, the
// sum of x[m] over threads 0..k.
template <int M, int NW = kWaves>
__device__ void block_scan_sat(uint32_t (&x)[M], uint32_t (*red)[NW]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
    for (int m = 0; m < M; m++) {
      const uint32_t y = __shfl_up(x[m], o, 64);
      if (lane >= o) x[m] = sadd(x[m], y);
    }
  }
  if (lane == 63) {
#pragma unroll
    for (int m = 0; m < M; m++) red[m][wave] = x[m];
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int m = 0; m < M; m++) {
      uint32_t t = lane < NW ? red[m][lane] : 0u;
#pragma unroll
      for (int o = 1; o < NW; o <<= 1) {
        const uint32_t y = __shfl_up(t, o, 64);
        if (lane >= o) t = sadd(t, y);
      }
      if (lane < NW) red[m][lane] = t;
    }
  }
  __syncthreads();
  if (wave > 0) {
#pragma unroll
    for (int m = 0; m < M; m++) x[m] = sadd(x[m], red[m][wave - 1]);
  }
  __syncthreads();
}

template <int NW = kWaves>
__device__ uint64_t block_min_u64(uint64_t x, uint64_t* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t y = __shfl_xor(x, o, 64);
    x = y < x ? y : x;
  }
  if (lane == 0) red[wave] = x;
  __syncthreads();
  uint64_t r = red[0];
  for (int w = 1; w < NW; w++) r = red[w] < r ? red[w] : r;
  __syncthreads();
  return r;
}


__device__ __forceinline__ size_t pose_index(int N, int i, int j, int T) {
  return ((size_t)T * N + j) * N + i;
}

// k-th pose before (i, j, T) on the curve of maneuver mu through it, in the
// maneuver's direction of travel; false if the curve has no such pose.
__device__ bool predecessor(const DevPlan& d, int mu, int i, int j, int T, int k, int* pi, int* pj, int* pT) {
  const int N = d.nx, L = d.nt;
  if (mu != NHP_SF && mu != NHP_SB) {
    if (k >= L) return false;
    const bool left = (mu == NHP_LF || mu == NHP_LB);
    const bool asc = (mu == NHP_LF || mu == NHP_RB);
    const int32_t* ox = d.turn_off + (left ? 0 : 2) * L;
    const int32_t* oy = d.turn_off + (left ? 1 : 3) * L;
    const int xp = wrapn((int)i - ox[T], N), yp = wrapn((int)j - oy[T], N);
    const int Tk = wrapn(asc ? (int)T - k : (int)T + k, L);
    *pi = wrapn((int)xp + ox[Tk], N);
    *pj = wrapn((int)yp + oy[Tk], N);
    *pT = Tk;
    return true;
  }
  const bool fam_x = d.family[T] == 0;
  const bool asc = (d.fwd[T] > 0) == (mu == NHP_SF);
  const int16_t* sk = d.skew + (size_t)T * N;
  const int c = fam_x ? i : j;
  const int other = fam_x ? j : i;
  const int xp = wrapn((int)other - sk[c], N);
  const int step = asc ? c : N - 1 - c;  // the kernels walk N-1 .. 0 when descending
  if (k > step) return false;
  const int c2 = asc ? step - k : N - 1 - (step - k);
  const int o2 = wrapn((int)xp + sk[c2], N);
  *pi = fam_x ? c2 : o2;
  *pj = fam_x ? o2 : c2;
  *pT = T;
  return true;
}

// k-th pose after (i, j, T) on the curve of maneuver mu, in the maneuver's
// direction of travel; false if the curve has no such pose (a turn closes
// after L - 1 steps, a straight line ends at its far end).
__device__ bool successor(const DevPlan& d, int mu, int i, int j, int T, int k, int* qi, int* qj, int* qT) {
  const int N = d.nx, L = d.nt;
  if (mu != NHP_SF && mu != NHP_SB) {
    if (k >= L) return false;
    const bool left = (mu == NHP_LF || mu == NHP_LB);
    const bool asc = (mu == NHP_LF || mu == NHP_RB);
    const int32_t* ox = d.turn_off + (left ? 0 : 2) * L;
    const int32_t* oy = d.turn_off + (left ? 1 : 3) * L;
    const int xp = wrapn(i - ox[T], N), yp = wrapn(j - oy[T], N);
    const int Tk = wrapn(asc ? T + k : T - k, L);
    *qi = wrapn(xp + ox[Tk], N);
    *qj = wrapn(yp + oy[Tk], N);
    *qT = Tk;
    return true;
  }
  const bool fam_x = d.family[T] == 0;
  const bool asc = (d.fwd[T] > 0) == (mu == NHP_SF);
  const int16_t* sk = d.skew + (size_t)T * N;
  const int c = fam_x ? i : j;
  const int other = fam_x ? j : i;
  const int xp = wrapn(other - sk[c], N);
  // position along the sweep: upward lines start at 0, downward ones at 0 in
  // the wall and then N - 1, N - 2, ...
  const int step = asc ? c : (c == 0 ? 0 : N - c);
  if (step + k > N - 1) return false;
  const int s2 = step + k;
  const int c2 = asc ? s2 : (s2 == 0 ? 0 : N - s2);
  const int o2 = wrapn(xp + sk[c2], N);
  *qi = fam_x ? c2 : o2;
  *qj = fam_x ? o2 : c2;
  *qT = T;
  return true;
}

// Seeds of a start set: block s walks start s's maneuver in progress (thread
// k takes the k-th pose; a block-wide saturating prefix sum gives the edge
// sums), lowers V at every reachable pose to cost + edge sum and records the
// seed; a start at rest seeds its own pose only.
__global__ __launch_bounds__(kThreads) void seed_kernel(DevPlan d) {
  __shared__ uint32_t red32[6][kWaves];
  const int s = blockIdx.x, k = threadIdx.x;
  const nhp_start st = d.starts[s];
  const int mu = st.maneuver;
  int qi = (int)st.i, qj = (int)st.j, qT = (int)st.T;
  bool ok = k == 0;
  if (k > 0 && mu >= 0 && k < d.seed_slots) ok = successor(d, mu, (int)st.i, (int)st.j, (int)st.T, k, &qi, &qj, &qT);
  // weight of the edge leaving pose k (source weight), summed over 0..k
  uint32_t w[1] = {kInf};
  if (ok && mu >= 0) w[0] = weight(d.B[pose_index(d.nx, qi, qj, qT)], d.edge_len[(size_t)mu * d.nt + qT]);
  uint32_t incl[1] = {w[0]};
  block_scan_sat<1>(incl, red32);
  // edge sum from pose 0 to pose k: the inclusive sum through pose k - 1
  __shared__ uint32_t sums[kThreads];
  sums[k] = incl[0];
  __syncthreads();
  const uint32_t E = k == 0 ? 0u : sums[k - 1];
  uint32_t* sd = d.seeds + ((size_t)s * d.seed_slots + k) * kSeedWords;
  const bool seed = ok && E != kInf && d.B[pose_index(d.nx, qi, qj, qT)] != kHard;
  if (k < d.seed_slots) {
    const uint32_t q = (uint32_t)pose_index(d.nx, qi, qj, qT);
    const uint32_t v = sadd(st.cost_q10, E);
    sd[0] = seed ? q : kNoSeed;
    sd[1] = v;
    sd[2] = (uint32_t)s;
    sd[3] = (uint32_t)k;
    if (seed) atomicMin(d.V + q, v);
  }
}

// Grid-wide barrier of the back-tracking workgroups (one per scheduled
// maneuver): thread 0 counts its workgroup in (a release, after its
// exchange writes) and polls, a bounded number of times, until `target`
// workgroups have arrived.  False when it gave up.
constexpr uint32_t kMaxPolls = 1u << 24;
__device__ bool group_barrier(uint32_t* counter, uint32_t target, uint32_t* flag) {
  if (threadIdx.x == 0) {
    uint32_t ok = 1, polls = 0;
    __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    while (__hip_atomic_load(counter, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++polls > kMaxPolls) {
        ok = 0;
        break;
      }
      if (polls < 4096)
        __builtin_amdgcn_s_sleep(1);
      else
        __builtin_amdgcn_s_sleep(32);
    }
    *flag = ok;
  }
  __syncthreads();
  const bool ok = *flag != 0;
  __syncthreads();
  return ok;
}

__device__ __forceinline__ uint32_t load_shared_word(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// GROUP: workgroup g examines the candidates of schedule position g only and
// the workgroups exchange their best (key, value, step cost) through the
// words after the step list; every workgroup then takes the same decision.
// Workgroup 0 writes the result.
template <bool GROUP, int NT = kThreads>
__device__ __forceinline__ void extract_body(const ExArgs& x, uint32_t (*red32)[NT / 64], uint64_t* red64,
                                             uint32_t* flag) {
  constexpr int NW = NT / 64;
  const DevPlan& d = x.d;
  const int N = d.nx, L = d.nt;
  const int tid = threadIdx.x;
  uint32_t* out = d.extract;
  const bool writer = !GROUP || blockIdx.x == 0;
  uint32_t* sync = out + kExHeader + (size_t)NHP_MAX_STEPS_DEVICE * kExStepWords;

  int ci, cj, cT;
  if (x.n_goals > 0) {
    // ---- goal set: smallest V + penalty, ties to the earlier goal ----
    uint64_t key = ~0ull;
    for (int k = tid; k < x.n_goals; k += NT) {
      const uint32_t* g = d.goals + 4 * (size_t)k;
      const size_t q = pose_index(N, (int)g[0], (int)g[1], (int)g[2]);
      const uint32_t v = d.V[q];
      if (d.B[q] == kHard || v == kInf) continue;
      const uint64_t k2 = ((uint64_t)sadd(v, g[3]) << 12) | (uint64_t)k;
      key = k2 < key ? k2 : key;
    }
    key = block_min_u64<NW>(key, red64);
    if (key == ~0ull) {
      if (tid == 0 && writer) {
        out[0] = (uint32_t)(-NHP_EUNREACH);
        out[1] = 0;
      }
      return;
    }
    const uint32_t* g = d.goals + 4 * (size_t)(key & 4095);
    ci = (int)g[0];
    cj = (int)g[1];
    cT = (int)g[2];
    if (tid == 0 && writer) {
      out[2] = ci;
      out[3] = cj;
      out[4] = cT;
      out[5] = d.V[pose_index(N, ci, cj, cT)];
      out[6] = (uint32_t)(key >> 12);
      out[7] = (uint32_t)(key & 4095);
    }
  } else {
    // ---- goal search over the (2r+1)^3 window ----
    const int r = x.radius, W = 2 * r + 1, nc = W * W * W;
    uint64_t key = ~0ull;
    for (int c = tid; c < nc; c += NT) {
      const int dx = c % W - r, dy = (c / W) % W - r, dt = c / (W * W) - r;
      const int i = modn((int)x.gi + dx, N), j = modn((int)x.gj + dy, N), T = modn((int)x.gt + dt, L);
      const size_t q = pose_index(N, i, j, T);
      const uint32_t v = d.V[q];
      if (d.B[q] == kHard || v == kInf) continue;
      const int ax = dx < 0 ? -dx : dx, ay = dy < 0 ? -dy : dy, at = dt < 0 ? -dt : dt;
      const uint64_t pen = (uint64_t)x.w_xy * (uint64_t)(ax + ay) + (uint64_t)x.w_t * (uint64_t)at;
      const uint32_t score = sadd(v, pen >= kInf ? kInf : (uint32_t)pen);
      const uint64_t k2 = ((uint64_t)score << 32) | ((uint64_t)(ax + ay + at) << 18) |
                          ((uint64_t)(dt + r) << 12) | ((uint64_t)(dy + r) << 6) | (uint64_t)(dx + r);
      key = k2 < key ? k2 : key;
    }
    key = block_min_u64<NW>(key, red64);
    if (key == ~0ull) {
      if (tid == 0 && writer) {
        out[0] = (uint32_t)(-NHP_EUNREACH);
        out[1] = 0;
      }
      return;
    }
    ci = modn((int)x.gi + (int)(key & 63) - r, N);
    cj = modn((int)x.gj + (int)((key >> 6) & 63) - r, N);
    cT = modn((int)x.gt + (int)((key >> 12) & 63) - r, L);
    if (tid == 0 && writer) {
      out[2] = ci;
      out[3] = cj;
      out[4] = cT;
      out[5] = d.V[pose_index(N, ci, cj, cT)];
      out[6] = (uint32_t)(key >> 32);
      out[7] = 0;
    }
  }

  // ---- back-tracking ----
  uint32_t n = 0, status = 0;
  const int k = tid + 1;
  int seed_hit = -1;  // seed slot the plan ends at (start sets)
  // value of the current pose: read once here, then handed on by the thread
  // that finds the next pose (with the step's cost), so a step waits for one
  // round of loads only
  uint32_t vcur = d.V[pose_index(N, ci, cj, cT)];
  for (uint32_t iter = 0;; iter++) {
    if (x.n_starts > 0) {
      // the first seed (start order, then along a maneuver in progress) at
      // this pose whose value is the current value ends the plan
      const uint32_t cur = (uint32_t)pose_index(N, ci, cj, cT);
      uint64_t hit = ~0ull;
      const int slots = x.n_starts * d.seed_slots;
      for (int e = tid; e < slots; e += NT) {
        const uint32_t* sd = d.seeds + (size_t)e * kSeedWords;
        if (sd[0] == cur && sd[1] == vcur) hit = hit < (uint64_t)e ? hit : (uint64_t)e;
      }
      hit = block_min_u64<NW>(hit, red64);
      if (hit != ~0ull) {
        seed_hit = (int)hit;
        break;
      }
    } else if ((uint32_t)ci == x.si && (uint32_t)cj == x.sj && (uint32_t)cT == x.st) {
      break;
    }
    // every step strictly lowers the value (edges cost >= 1), so a plan from
    // a swept volume ends well within the step buffer; the bound only stops
    // a walk over a value volume that no sweep produced
    if (iter > NHP_MAX_STEPS_DEVICE || vcur == kInf) {
      status = (uint32_t)(-NHP_EUNREACH);
      break;
    }
    // candidates k = tid + 1 of every scheduled maneuver (GROUP: of this
    // workgroup's one): all loads first
    constexpr int M = GROUP ? 1 : 6;
    uint32_t w[M], vq[M];
    bool ok[M];
#pragma unroll
    for (int m = 0; m < M; m++) {
      const int pos = GROUP ? (int)blockIdx.x : m;
      w[m] = kInf;
      vq[m] = kInf;
      ok[m] = false;
      if (pos < d.n_schedule) {
        const int mu = d.schedule[pos];
        int pi = 0, pj = 0, pT = 0;
        ok[m] = predecessor(d, mu, ci, cj, cT, k, &pi, &pj, &pT);
        if (ok[m]) {
          const size_t q = pose_index(N, pi, pj, pT);
          w[m] = weight(d.B[q], d.edge_len[(size_t)mu * L + pT]);
          vq[m] = d.V[q];
        }
      }
    }
    block_scan_sat<M, NW>(w, red32);  // w[m] becomes the edge sum E_k
    uint64_t best = ~0ull;
#pragma unroll
    for (int m = 0; m < M; m++) {
      const int pos = GROUP ? (int)blockIdx.x : m;
      if (pos < d.n_schedule) {
        const uint32_t cand = sadd(sadd(vq[m], d.ct[d.schedule[pos]]), w[m]);
        if (ok[m] && cand != kInf) {
          const uint64_t k2 = ((uint64_t)cand << 14) | ((uint64_t)pos << 11) | (uint64_t)k;
          best = k2 < best ? k2 : best;
        }
      }
    }
    best = block_min_u64<NW>(best, red64);
    // the thread holding the best candidate hands on its pose's value and
    // the step's cost (ct + edge sum)
    if (best != ~0ull && k == (int)(best & 2047)) {
      const int bpos = (int)((best >> 11) & 7);
#pragma unroll
      for (int m = 0; m < M; m++) {
        if ((GROUP ? (int)blockIdx.x : m) == bpos) {
          red32[0][0] = vq[m];
          red32[0][1] = sadd(d.ct[d.schedule[bpos]], w[m]);
        }
      }
    }
    __syncthreads();
    uint32_t vnext = red32[0][0], cost = red32[0][1];
    __syncthreads();  // red32 is reused by the next step's scan
    if (GROUP) {
      // exchange the workgroups' bests (double-buffered by step parity, so a
      // fast workgroup's next writes never meet a slow one's reads)
      uint32_t* mine = sync + 1 + ((iter & 1) * 6 + blockIdx.x) * 4;
      if (tid == 0) {
        mine[0] = (uint32_t)best;
        mine[1] = (uint32_t)(best >> 32);
        mine[2] = vnext;
        mine[3] = cost;
      }
      if (!group_barrier(sync, gridDim.x * (iter + 1), flag)) {
        status = (uint32_t)(-NHP_EHIP);
        break;
      }
      // the four words of all 6 slots read in one round (the area always
      // holds 6; slots past the grid are read and ignored), then the best
      // of the grid's workgroups taken
      uint32_t ex[6][4];
      const uint32_t* slots = sync + 1 + (iter & 1) * 6 * 4;
#pragma unroll
      for (int g = 0; g < 6; g++) {
#pragma unroll
        for (int m = 0; m < 4; m++) ex[g][m] = load_shared_word(slots + g * 4 + m);
      }
#pragma unroll
      for (int g = 0; g < 6; g++)
        asm volatile("" : "+v"(ex[g][0]), "+v"(ex[g][1]), "+v"(ex[g][2]), "+v"(ex[g][3]));  // all arrived first
      best = ~0ull;
#pragma unroll
      for (int g = 0; g < 6; g++) {
        if (g < (int)gridDim.x) {
          const uint64_t kg = (uint64_t)ex[g][0] | ((uint64_t)ex[g][1] << 32);
          if (kg < best) {
            best = kg;
            vnext = ex[g][2];
            cost = ex[g][3];
          }
        }
      }
    }
    if (best == ~0ull) {
      status = (uint32_t)(-NHP_EUNREACH);
      break;
    }
    const int pos = (int)((best >> 11) & 7), kb = (int)(best & 2047);
    const int mu = d.schedule[pos];
    int pi, pj, pT;
    predecessor(d, mu, ci, cj, cT, kb, &pi, &pj, &pT);
    if (tid == 0 && writer && n < NHP_MAX_STEPS_DEVICE) {
      uint32_t* s = out + kExHeader + (size_t)n * kExStepWords;
      s[0] = mu;
      s[1] = kb;
      s[2] = pi;
      s[3] = pj;
      s[4] = pT;
      s[5] = ci;
      s[6] = cj;
      s[7] = cT;
      s[8] = cost;
    }
    n++;
    ci = pi;
    cj = pj;
    cT = pT;
    vcur = vnext;
  }
  if (seed_hit >= 0 && status == 0) {
    // a seed inside a maneuver in progress: that maneuver is the first step
    const uint32_t* sd = d.seeds + (size_t)seed_hit * kSeedWords;
    const nhp_start st = d.starts[sd[2]];
    if (sd[3] > 0) {
      if (tid == 0 && writer && n < NHP_MAX_STEPS_DEVICE) {
        uint32_t* o = out + kExHeader + (size_t)n * kExStepWords;
        o[0] = (uint32_t)st.maneuver;
        o[1] = sd[3];
        o[2] = st.i;
        o[3] = st.j;
        o[4] = st.T;
        o[5] = ci;
        o[6] = cj;
        o[7] = cT;
        o[8] = sd[1] - st.cost_q10;
      }
      n++;
    }
  }
  if (tid == 0 && writer) {
    out[0] = status;
    out[1] = n;
  }
}

// one workgroup per scheduled maneuver (see extract_body), NT threads: at
// least one per candidate, i.e. more than the longest curve (max(nx, ntheta) - 1
// poses), in as few waves as that allows
template <int NT>
__global__ __launch_bounds__(NT) void extract_kernel(ExArgs x) {
  __shared__ uint32_t red32[6][NT / 64];
  __shared__ uint64_t red64[NT / 64];
  __shared__ uint32_t flag;
  extract_body<true, NT>(x, red32, red64, &flag);
}

__global__ void clear_word_kernel(uint32_t* w) { *w = 0; }

// one workgroup per plan
__global__ __launch_bounds__(kThreads) void extract_batch_kernel(const ExArgs* __restrict__ args) {
  __shared__ uint32_t red32[6][kWaves];
  __shared__ uint64_t red64[kWaves];
  const ExArgs x = args[blockIdx.x];
  extract_body<false>(x, red32, red64, nullptr);
}

// ---- reachability (App. C): goal search and back-tracking on level bits ----

__device__ __forceinline__ bool reach_bit(const ReachExArgs& x, int m, int i, int j, int T) {
  const int N = x.d.nx;
  const uint32_t word = x.levels[(size_t)m * x.vol_words + ((size_t)T * N + j) * x.W + (i >> 5)];
  return ((word >> (i & 31)) & 1u) == 0u;  // a clear bit is reachable
}

__device__ __forceinline__ bool hard_bit(const ReachExArgs& x, int i, int j, int T) {
  const int N = x.d.nx;
  return (x.hard[((size_t)T * N + j) * x.W + (i >> 5)] >> (i & 31)) & 1u;
}

// smallest m with the pose reachable (levels are nested), or -1
__device__ int pose_level(const ReachExArgs& x, int i, int j, int T) {
  int hi = x.n_levels - 1;
  if (!reach_bit(x, hi, i, j, T)) return -1;
  int lo = 0;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (reach_bit(x, mid, i, j, T))
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

// Goal window: smallest (level, |dx|+|dy|+|dT|, dT, dy, dx).  Back-tracking
// from a pose of level m: for the scheduled maneuvers in schedule order, the
// nearest pose up the curve (through free poses) of level m - 1.
__global__ __launch_bounds__(kThreads) void reach_extract_kernel(ReachExArgs x) {
  __shared__ uint64_t red64[kWaves];
  __shared__ int first_hard[6];
  const DevPlan& d = x.d;
  const int N = d.nx, L = d.nt;
  const int tid = threadIdx.x;
  uint32_t* out = x.out;
  const int r = x.radius, Wd = 2 * r + 1, nc = Wd * Wd * Wd;
  uint64_t key = ~0ull;
  for (int c = tid; c < nc; c += kThreads) {
    const int dx = c % Wd - r, dy = (c / Wd) % Wd - r, dt = c / (Wd * Wd) - r;
    const int i = modn((int)x.gi + dx, N), j = modn((int)x.gj + dy, N), T = modn((int)x.gt + dt, L);
    const int lv = pose_level(x, i, j, T);
    if (lv < 0) continue;
    const int ax = dx < 0 ? -dx : dx, ay = dy < 0 ? -dy : dy, at = dt < 0 ? -dt : dt;
    const uint64_t k2 = ((uint64_t)lv << 25) | ((uint64_t)(ax + ay + at) << 18) | ((uint64_t)(dt + r) << 12) |
                        ((uint64_t)(dy + r) << 6) | (uint64_t)(dx + r);
    key = k2 < key ? k2 : key;
  }
  key = block_min_u64(key, red64);
  if (key == ~0ull) {
    if (tid == 0) {
      out[0] = (uint32_t)(-NHP_EUNREACH);
      out[1] = 0;
    }
    return;
  }
  int ci = modn((int)x.gi + (int)(key & 63) - r, N);
  int cj = modn((int)x.gj + (int)((key >> 6) & 63) - r, N);
  int cT = modn((int)x.gt + (int)((key >> 12) & 63) - r, L);
  int m = (int)(key >> 25);
  if (tid == 0) {
    out[2] = ci;
    out[3] = cj;
    out[4] = cT;
    out[5] = m;
  }
  uint32_t n = 0, status = 0;
  const int k = tid + 1;
  while (m > 0) {
    if (tid < 6) first_hard[tid] = 0x7fffffff;
    __syncthreads();
    int pi[6], pj[6], pT[6];
    bool ok[6];
#pragma unroll
    for (int pos = 0; pos < 6; pos++) {
      ok[pos] = pos < d.n_schedule && predecessor(d, d.schedule[pos], ci, cj, cT, k, &pi[pos], &pj[pos], &pT[pos]);
      if (ok[pos] && hard_bit(x, pi[pos], pj[pos], pT[pos])) atomicMin(&first_hard[pos], k);
    }
    __syncthreads();
    uint64_t best = ~0ull;
#pragma unroll
    for (int pos = 0; pos < 6; pos++) {
      if (ok[pos] && k < first_hard[pos] && reach_bit(x, m - 1, pi[pos], pj[pos], pT[pos])) {
        const uint64_t k2 = ((uint64_t)pos << 11) | (uint64_t)k;
        best = k2 < best ? k2 : best;
      }
    }
    best = block_min_u64(best, red64);
    if (best == ~0ull) {
      status = (uint32_t)(-NHP_EUNREACH);
      break;
    }
    const int pos = (int)(best >> 11), kb = (int)(best & 2047);
    const int mu = d.schedule[pos];
    int qi, qj, qT;
    predecessor(d, mu, ci, cj, cT, kb, &qi, &qj, &qT);
    if (tid == 0 && n < (uint32_t)kReachMaxSteps) {
      uint32_t* st = out + kExHeader + (size_t)n * kExStepWords;
      st[0] = mu;
      st[1] = kb;
      st[2] = qi;
      st[3] = qj;
      st[4] = qT;
      st[5] = ci;
      st[6] = cj;
      st[7] = cT;
      st[8] = 1;
    }
    n++;
    ci = qi;
    cj = qj;
    cT = qT;
    m--;
  }
  if (tid == 0) {
    out[0] = status;
    out[1] = n;
  }
}

}  // namespace

hipError_t launch_reach_extract(const ReachExArgs& x, hipStream_t s) {
  hipLaunchKernelGGL(reach_extract_kernel, dim3(1), dim3(kThreads), 0, s, x);
  return hipGetLastError();
}

hipError_t launch_extract(const ExArgs& x, hipStream_t s) {
  if (x.d.n_schedule < 1 || x.d.n_schedule > 6) return hipErrorInvalidValue;
  // the barrier counter starts at zero (a kernel, not a memset node, so the
  // call may be captured)
  hipLaunchKernelGGL(clear_word_kernel, dim3(1), dim3(1), 0, s,
                     x.d.extract + kExHeader + (size_t)NHP_MAX_STEPS_DEVICE * kExStepWords);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int len = x.d.nx > x.d.nt ? x.d.nx : x.d.nt;
  if (len <= 256)
    hipLaunchKernelGGL(extract_kernel<256>, dim3(x.d.n_schedule), dim3(256), 0, s, x);
  else if (len <= 512)
    hipLaunchKernelGGL(extract_kernel<512>, dim3(x.d.n_schedule), dim3(512), 0, s, x);
  else
    hipLaunchKernelGGL(extract_kernel<1024>, dim3(x.d.n_schedule), dim3(1024), 0, s, x);
  return hipGetLastError();
}

hipError_t launch_seed(const DevPlan& d, int n_starts, hipStream_t s) {
  hipLaunchKernelGGL(seed_kernel, dim3(n_starts), dim3(kThreads), 0, s, d);
  return hipGetLastError();
}

// ---- extract area of extract_path_noalloc ----
// One extract area (header, step list, barrier counter and exchange area) per
// device, in a file-scope device array instead of a plan's workspace, for
// callers that cannot allocate.  Every call on a device shares its copy.
static __device__ __align__(256) uint32_t scratch[kNoAllocExtractWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device
}  // namespace

hipError_t noalloc_extract_area(int device, uint32_t** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    // the array's name is a host-side stand-in: its device address comes
    // from the runtime, once per device, with that device current
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = static_cast<uint32_t*>(ptr);
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

hipError_t launch_extract_batch(const ExArgs* d_args, int n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(extract_batch_kernel, dim3(n), dim3(kThreads), 0, s, d_args);
  return hipGetLastError();
}

}  // namespace nhp
