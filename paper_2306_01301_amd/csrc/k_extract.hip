// k_extract.hip -- goal search (Sec. IX) and back-tracking (Sec. X, eq. 32)
// in one single-workgroup kernel, so the value volume never leaves the
// device and the serial back-tracking loop pays no launch per step.
//
// Back-tracking step ("Bellman iteration in reverse"): for every scheduled
// maneuver mu, thread t examines the pose p_k, k = t + 1, up the mu-curve
// through the current pose; a block-wide saturating prefix sum gives the
// edge sum E_k from p_k to the current pose, the candidate is
// V(p_k) + ct_mu + E_k, and a block-wide minimum of the packed key
// (candidate, schedule position, k) picks the next pose.  Curves are at most
// 1024 poses long, so one thread per candidate suffices.
#include "nhp_internal.h"

namespace nhp {
namespace {

constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / 64;

__device__ __forceinline__ uint32_t sadd(uint32_t a, uint32_t b) { return __builtin_elementwise_add_sat(a, b); }

__device__ __forceinline__ int wrapn(long v, int n) {
  long r = v % n;
  return (int)(r < 0 ? r + n : r);
}

__device__ __forceinline__ uint32_t weight(uint32_t code, uint32_t Lq) {
  if (code == kHard) return kInf;
  return (uint32_t)(((uint64_t)Lq * (256u + 4u * code) + 128u) >> 8);
}

// inclusive saturating prefix sum over the block, k-th thread gets sum of 0..k
__device__ uint32_t block_scan_sat(uint32_t x, uint32_t* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x = sadd(x, y);
  }
  if (lane == 63) red[wave] = x;
  __syncthreads();
  if (wave == 0) {
    uint32_t t = lane < kWaves ? red[lane] : 0u;
#pragma unroll
    for (int o = 1; o < kWaves; o <<= 1) {
      const uint32_t y = __shfl_up(t, o, 64);
      if (lane >= o) t = sadd(t, y);
    }
    if (lane < kWaves) red[lane] = t;
  }
  __syncthreads();
  if (wave > 0) x = sadd(x, red[wave - 1]);
  __syncthreads();
  return x;
}

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
  for (int w = 1; w < kWaves; w++) r = red[w] < r ? red[w] : r;
  __syncthreads();
  return r;
}

struct ExArgs {
  DevPlan d;
  uint32_t si, sj, st, gi, gj, gt;
  int radius;
  uint32_t w_xy, w_t;
};

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
    const int xp = wrapn((long)i - ox[T], N), yp = wrapn((long)j - oy[T], N);
    const int Tk = wrapn(asc ? (long)T - k : (long)T + k, L);
    *pi = wrapn((long)xp + ox[Tk], N);
    *pj = wrapn((long)yp + oy[Tk], N);
    *pT = Tk;
    return true;
  }
  const bool fam_x = d.family[T] == 0;
  const bool asc = (d.fwd[T] > 0) == (mu == NHP_SF);
  const int16_t* sk = d.skew + (size_t)T * N;
  const int c = fam_x ? i : j;
  const int other = fam_x ? j : i;
  const int xp = wrapn((long)other - sk[c], N);
  const int step = asc ? c : N - 1 - c;  // the kernels walk N-1 .. 0 when descending
  if (k > step) return false;
  const int c2 = asc ? step - k : N - 1 - (step - k);
  const int o2 = wrapn((long)xp + sk[c2], N);
  *pi = fam_x ? c2 : o2;
  *pj = fam_x ? o2 : c2;
  *pT = T;
  return true;
}

__global__ __launch_bounds__(kThreads) void extract_kernel(ExArgs x) {
  __shared__ uint32_t red32[kWaves];
  __shared__ uint64_t red64[kWaves];
  const DevPlan& d = x.d;
  const int N = d.nx, L = d.nt;
  const int tid = threadIdx.x;
  uint32_t* out = d.extract;

  // ---- goal search over the (2r+1)^3 window ----
  const int r = x.radius, W = 2 * r + 1, nc = W * W * W;
  uint64_t key = ~0ull;
  for (int c = tid; c < nc; c += kThreads) {
    const int dx = c % W - r, dy = (c / W) % W - r, dt = c / (W * W) - r;
    const int i = wrapn((long)x.gi + dx, N), j = wrapn((long)x.gj + dy, N), T = wrapn((long)x.gt + dt, L);
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
  key = block_min_u64(key, red64);
  if (key == ~0ull) {
    if (tid == 0) {
      out[0] = (uint32_t)(-NHP_EUNREACH);
      out[1] = 0;
    }
    return;
  }
  int ci = wrapn((long)x.gi + (int)(key & 63) - r, N);
  int cj = wrapn((long)x.gj + (int)((key >> 6) & 63) - r, N);
  int cT = wrapn((long)x.gt + (int)((key >> 12) & 63) - r, L);
  if (tid == 0) {
    out[2] = ci;
    out[3] = cj;
    out[4] = cT;
    out[5] = d.V[pose_index(N, ci, cj, cT)];
    out[6] = (uint32_t)(key >> 32);
  }

  // ---- back-tracking ----
  uint32_t n = 0, status = 0;
  const int k = tid + 1;
  for (uint32_t iter = 0;; iter++) {
    if ((uint32_t)ci == x.si && (uint32_t)cj == x.sj && (uint32_t)cT == x.st) break;
    // every step strictly lowers the value (edges cost >= 1), so a plan from
    // a swept volume ends well within the step buffer; the bound only stops
    // a walk over a value volume that no sweep produced
    if (iter > NHP_MAX_STEPS_DEVICE || d.V[pose_index(N, ci, cj, cT)] == kInf) {
      status = (uint32_t)(-NHP_EUNREACH);
      break;
    }
    uint64_t best = ~0ull;
    for (int pos = 0; pos < d.n_schedule; pos++) {
      const int mu = d.schedule[pos];
      int pi = 0, pj = 0, pT = 0;
      const bool ok = predecessor(d, mu, ci, cj, cT, k, &pi, &pj, &pT);
      uint32_t w = kInf, vq = kInf;
      if (ok) {
        const size_t q = pose_index(N, pi, pj, pT);
        w = weight(d.B[q], d.edge_len[(size_t)mu * L + pT]);
        vq = d.V[q];
      }
      const uint32_t E = block_scan_sat(w, red32);
      const uint32_t cand = sadd(sadd(vq, d.ct[mu]), E);
      if (ok && cand != kInf) {
        const uint64_t k2 = ((uint64_t)cand << 14) | ((uint64_t)pos << 11) | (uint64_t)k;
        best = k2 < best ? k2 : best;
      }
    }
    best = block_min_u64(best, red64);
    if (best == ~0ull) {
      status = (uint32_t)(-NHP_EUNREACH);
      break;
    }
    const int pos = (int)((best >> 11) & 7), kb = (int)(best & 2047);
    const uint32_t cand = (uint32_t)(best >> 14);
    const int mu = d.schedule[pos];
    int pi, pj, pT;
    predecessor(d, mu, ci, cj, cT, kb, &pi, &pj, &pT);
    if (tid == 0 && n < NHP_MAX_STEPS_DEVICE) {
      uint32_t* s = out + kExHeader + (size_t)n * kExStepWords;
      s[0] = mu;
      s[1] = kb;
      s[2] = pi;
      s[3] = pj;
      s[4] = pT;
      s[5] = ci;
      s[6] = cj;
      s[7] = cT;
      s[8] = cand - d.V[pose_index(N, pi, pj, pT)];  // ct + edge sum (no saturation below INF)
    }
    n++;
    ci = pi;
    cj = pj;
    cT = pT;
  }
  if (tid == 0) {
    out[0] = status;
    out[1] = n;
  }
}

}  // namespace

hipError_t launch_extract(const DevPlan& d, uint32_t si, uint32_t sj, uint32_t st, uint32_t gi, uint32_t gj,
                          uint32_t gt, int radius, uint32_t w_xy, uint32_t w_t, hipStream_t s) {
  ExArgs x{d, si, sj, st, gi, gj, gt, radius, w_xy, w_t};
  hipLaunchKernelGGL(extract_kernel, dim3(1), dim3(kThreads), 0, s, x);
  return hipGetLastError();
}

}  // namespace nhp
