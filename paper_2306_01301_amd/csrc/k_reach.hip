// k_reach.hip -- reachability by maneuver count (App. C, Insert 2) for
// gfx950, on bit volumes (32 poses of one row per word).
//
// With hard obstacles only and every maneuver costing one transition, a pose
// needs one bit per maneuver count m: reachable with at most m maneuvers or
// not.  In the paper's convention a set bit means "not reachable", so along
// a maneuver curve the carried bit v is updated per pose by
//     v = (v AND R_m(pose)) OR hard(pose),   out(pose) = v
// and R_{m+1} is the AND over the scheduled maneuvers' outputs (every
// maneuver of a cycle reads R_m).  All level volumes R_0 .. R_n are kept for
// back-tracking.
//
// Kernels:
//   * rendering: the hard image as bits, then per heading plane the OR of the
//     image under the vehicle box (sideways samples, then lengthwise samples
//     of the sideways plane staged in LDS); a sample shifted by dx reads two
//     words and funnels them with one alignbit.
//   * turn curves: 32 curves per lane (one word of a row of curve origins),
//     the curve split into S sections of P steps held in registers (the
//     shortest sections whose lanes fit a workgroup of 256); both
//     maneuvers of a circle family (forward and backward along it) run on the
//     same registers; section results meet in LDS (the three passes of the
//     Sections technique, App. D, Inserts 6-8, done in one kernel).  A lane's
//     32 curves sit at a bit offset of the row, so loads funnel two words and
//     stores take the neighbour lane's word through a cross-lane permute, so
//     every store writes one whole aligned word.
//   * straight lines: one workgroup per heading plane, the plane's level bits,
//     hard bits and output bits in LDS with rows along the sweep coordinate
//     (transposed in 32 x 32 bit blocks for the x-major family), one thread
//     per 32 lines and direction carrying the lines' bits in one word.
#include "nhp_internal.h"

namespace nhp {
namespace {

__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, int r) {
  return __builtin_amdgcn_alignbit(hi, lo, (uint32_t)r);  // ({hi, lo} >> r)[31:0]
}

__device__ __forceinline__ int wrapn(int v, int n) {
  v += (v < 0) ? n : 0;
  return v - ((v >= n) ? n : 0);
}

// ---- rendering ----

// img[j][w]: bit t set when image(32 w + t, j) is hard, or in the one-cell
// walls of row 0 and column 0 (put into the image before dilation).
__global__ __launch_bounds__(256) void reach_image_kernel(const uint8_t* __restrict__ image, uint32_t* __restrict__ img,
                                                          int N, int W) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N * W) return;
  const int j = q / W, w = q % W;
  const uint8_t* row = image + (size_t)j * N + 32 * w;
  uint32_t bits = 0;
#pragma unroll 8
  for (int t = 0; t < 32; t++) bits |= (row[t] == kHard ? 1u : 0u) << t;
  if (j == 0) bits = ~0u;
  if (w == 0) bits |= 1u;
  img[q] = bits;
}

// OR over the samples (packed dx | dy << 16, reduced mod N) of a bit plane
// `src` (N rows of W words) at word w of row j.
__device__ __forceinline__ uint32_t or_samples(const uint32_t* src, const int32_t* tp, int n, int j, int w, int N,
                                               int W) {
  uint32_t acc = 0;
  for (int g = 0; g < n; g++) {
    const int32_t t = tp[g];
    const int row = wrapn(j + (int)((uint32_t)t >> 16), N);
    const int pos = wrapn(32 * w + (int)(t & 0xffff), N);
    const int q = pos >> 5, r = pos & 31;
    const int q1 = (q + 1 == W) ? 0 : q + 1;
    acc |= funnel(src[row * W + q1], src[row * W + q], r);
  }
  return acc;
}

// One workgroup per heading plane: the sideways OR into an LDS plane, then
// the lengthwise OR into the obstacle bits; the wall poses are forced hard.
__global__ __launch_bounds__(256) void reach_render_kernel(const uint32_t* __restrict__ img, const int32_t* __restrict__ taps,
                                                           uint32_t* __restrict__ hard, int N, int W, int n_side,
                                                           int n_len) {
  __shared__ int32_t ts[kMaxTaps], tl[kMaxTaps];
  __shared__ uint32_t side[kReachMaxN * (kReachMaxN / 32)];
  const int T = blockIdx.x;
  const int32_t* tp = taps + (size_t)T * (n_side + n_len);
  for (int g = threadIdx.x; g < n_side; g += blockDim.x) ts[g] = tp[g];
  for (int g = threadIdx.x; g < n_len; g += blockDim.x) tl[g] = tp[n_side + g];
  __syncthreads();
  const int NW = N * W;
  for (int q = threadIdx.x; q < NW; q += blockDim.x) side[q] = or_samples(img, ts, n_side, q / W, q % W, N, W);
  __syncthreads();
  uint32_t* out = hard + (size_t)T * NW;
  for (int q = threadIdx.x; q < NW; q += blockDim.x) {
    const int j = q / W, w = q % W;
    uint32_t b = or_samples(side, tl, n_len, j, w, N, W);
    if (j == 0) b = ~0u;
    if (w == 0) b |= 1u;
    out[q] = b;
  }
}

// Obstacle bits from a code volume (code 255 = hard), walls forced.
__global__ __launch_bounds__(256) void reach_pack_kernel(const uint8_t* __restrict__ codes, uint32_t* __restrict__ hard,
                                                         int N, int W, size_t words) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= words) return;
  const int w = (int)(q % W);
  const int j = (int)((q / W) % N);
  const uint8_t* c = codes + q * 32;
  uint32_t bits = 0;
#pragma unroll 8
  for (int t = 0; t < 32; t++) bits |= (c[t] == kHard ? 1u : 0u) << t;
  if (j == 0) bits = ~0u;
  if (w == 0) bits |= 1u;
  hard[q] = bits;
}

// R_0: nothing reachable but the start.
__global__ __launch_bounds__(256) void reach_start_kernel(uint32_t* __restrict__ R, size_t words, uint32_t start) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < words; q += stride)
    R[q] = (q == (start >> 5)) ? ~(1u << (start & 31)) : ~0u;
}

// ---- turn curves ----

struct TurnJob {
  const uint32_t* rin;
  uint32_t* rout;
  const uint32_t* hard;
  const int32_t* offx;  // offsets of the family's curves, reduced mod N
  const int32_t* offy;
  int N, L, W, Wp, rows, S;
  int fwd_on, bwd_on;  // the maneuver walking up the headings / down
  int store;           // 1: write R_{m+1}; 0: AND into it
};

// Lane layout of a workgroup: section sec, row slot rr, word w:
// thread = (sec * rows + rr) * Wp + w, Wp = W rounded up to a power of two,
// so the Wp lanes of one (sec, rr) sit together inside one wave.
// The most threads (sections x rows x words) per workgroup; shorter sections
// put more lanes to work (at 128 x 128 x 512: 0.30 ms for eight cycles with
// 256, 0.35 with 128, 0.50 with 64, 0.32 with 512).
constexpr int kTurnThreads = 256;
template <int P>
__global__ __launch_bounds__(kTurnThreads) void reach_turn_kernel(TurnJob a) {
  __shared__ int32_t sox[kReachMaxL], soy[kReachMaxL];
  __shared__ uint32_t aggD[kTurnThreads], aggF[kTurnThreads], aggB[kTurnThreads];
  const int tid = threadIdx.x;
  for (int t = tid; t < a.L; t += blockDim.x) {
    sox[t] = a.offx[t];
    soy[t] = a.offy[t];
  }
  __syncthreads();
  const int N = a.N, L = a.L, W = a.W, S = a.S;
  const int G = a.rows * a.Wp;
  const int g = tid % G, sec = tid / G;
  const int w = g % a.Wp, rr = g / a.Wp;
  const int yp = blockIdx.x * a.rows + rr;
  const bool live = w < W && yp < N;
  const int wl = w < W ? w : 0;  // idle lanes read valid words
  const int yl = yp < N ? yp : 0;

  uint32_t vi[P], h[P];
#pragma unroll
  for (int k = 0; k < P; k++) {
    const int s = sec * P + k;
    if (s < L) {
      const int ox = sox[s];
      const int row = wrapn(yl + soy[s], N);
      const int q = wrapn(wl + (ox >> 5), W), r = ox & 31;
      const int q1 = (q + 1 == W) ? 0 : q + 1;
      const size_t base = ((size_t)s * N + row) * W;
      vi[k] = funnel(a.rin[base + q1], a.rin[base + q], r);
      h[k] = funnel(a.hard[base + q1], a.hard[base + q], r);
    } else {
      vi[k] = ~0u;  // steps past the curve: identity maps
      h[k] = 0u;
    }
  }
  // section summaries: D = OR of the hard bits (the carried bit is then
  // replaced), F / B = the section's output from an unreachable entry,
  // walking up / down the headings
  uint32_t D = 0, F = ~0u, Bk = ~0u;
#pragma unroll
  for (int k = 0; k < P; k++) {
    D |= h[k];
    F = (F & vi[k]) | h[k];
  }
#pragma unroll
  for (int k = P - 1; k >= 0; k--) Bk = (Bk & vi[k]) | h[k];
  aggD[sec * G + g] = D;
  aggF[sec * G + g] = F;
  aggB[sec * G + g] = Bk;
  __syncthreads();
  // bit entering this section: once around the circle from "unreachable",
  // starting with this section and ending with the one before it
  uint32_t cf = ~0u, cb = ~0u;
  if (a.fwd_on) {
    int s2 = sec;
    for (int t = 0; t < S; t++) {
      cf = (cf | aggD[s2 * G + g]) & aggF[s2 * G + g];
      s2 = (s2 + 1 == S) ? 0 : s2 + 1;
    }
  }
  if (a.bwd_on) {
    int s2 = sec;
    for (int t = 0; t < S; t++) {
      cb = (cb | aggD[s2 * G + g]) & aggB[s2 * G + g];
      s2 = (s2 == 0) ? S - 1 : s2 - 1;
    }
  }
  uint32_t o[P];
  uint32_t v = cf;
#pragma unroll
  for (int k = 0; k < P; k++) {
    v = (v & vi[k]) | h[k];
    o[k] = a.fwd_on ? v : ~0u;
  }
  if (a.bwd_on) {
    v = cb;
#pragma unroll
    for (int k = P - 1; k >= 0; k--) {
      v = (v & vi[k]) | h[k];
      o[k] &= v;
    }
  }
  // store: output word (w + q) of the row gets the top bits of this lane's
  // word and the bottom bits of the lane before it (w - 1, cyclically)
  const int lane = tid & 63;
  const int src = (lane - w) + (w == 0 ? W - 1 : (w < W ? w - 1 : 0));
#pragma unroll
  for (int k = 0; k < P; k++) {
    const uint32_t prev = __shfl(o[k], src, 64);
    const int s = sec * P + k;
    if (s < L && live) {
      const int ox = sox[s];
      const int row = wrapn(yl + soy[s], N);
      const int q = wrapn(wl + (ox >> 5), W), r = ox & 31;
      const uint32_t val = r ? funnel(o[k], prev, 32 - r) : o[k];
      uint32_t* dst = a.rout + ((size_t)s * N + row) * W + q;
      *dst = a.store ? val : (*dst & val);
    }
  }
}

// ---- straight lines ----

struct StraightJob {
  const uint32_t* rin;
  uint32_t* rout;
  const uint32_t* hard;
  const int16_t* skew;
  const int32_t* family;
  const int32_t* fwd;
  int N, W;
  int sf_on, sb_on, store;
};

// Line x' of plane T visits, at sweep coordinate c, the pose (c, x' + B(c))
// for the x-major family and (x' + B(c), c) for the y-major one (eq. 23);
// SF walks c upward when J > 0, SB the other way, and a downward walk starts
// at c = 0 (in the wall) and continues N - 1, N - 2, ...
//
// One workgroup per heading plane.  The plane's level and hard bits go to
// LDS as a matrix whose row c holds the poses of sweep coordinate c: the
// plane itself for the y-major family, its transpose for the x-major one
// (built from 32 x 32 bit blocks).  Then lines x' = 32 g .. 32 g + 31 sit at 32
// consecutive columns 32 g + B(c) .. of row c, so one thread carries the 32
// lines' bits in one word: per step it funnels the window out of two words
// and applies v = (v AND R) OR hard to all 32 lines at once; the lines that
// are reachable clear their output bits with two LDS atomic ANDs (windows of
// neighbouring groups share words).  The output matrix is transposed back
// for the x-major family as it is stored.  (The transposes work on 32 x 32
// bit blocks in registers: N is a multiple of 32.)
// Transpose of 32 x 32 bit blocks of a matrix of N rows of W words (bit t
// of word w of row r is column 32 w + t), 32 lanes per block: lane r loads
// row r of block (rows 32 X.., word Y), five butterfly stages swap the
// off-diagonal halves, quarters, ... between lane pairs, and lane r then
// holds row 32 Y + r, word X of the transpose.  `put` receives (row, word,
// value).  Every lane of the workgroup must call it (the stages shuffle).
template <typename Put>
__device__ __forceinline__ void transpose_blocks(const uint32_t* src, int W, Put put) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n_waves = blockDim.x >> 6;
  const int r = lane & 31, n_blocks = W * W, per_round = 2 * n_waves;
  const int rounds = (n_blocks + per_round - 1) / per_round;
  for (int it = 0; it < rounds; it++) {
    const int blk = it * per_round + 2 * wave + (lane >> 5);
    const bool ok = blk < n_blocks;
    const int X = ok ? blk / W : 0, Y = ok ? blk % W : 0;
    uint32_t v = ok ? src[(32 * X + r) * W + Y] : 0u;
    const uint32_t masks[5] = {0x0000FFFFu, 0x00FF00FFu, 0x0F0F0F0Fu, 0x33333333u, 0x55555555u};
#pragma unroll
    for (int st = 0; st < 5; st++) {
      const int j = 16 >> st;
      const uint32_t other = __shfl_xor(v, j, 64);
      if ((r & j) == 0) {
        v ^= (((v >> j) ^ other) & masks[st]) << j;
      } else {
        v ^= ((other >> j) ^ v) & masks[st];
      }
    }
    if (ok) put(32 * Y + r, X, v);
  }
}

constexpr int kStraightThreads = 256;
__global__ __launch_bounds__(kStraightThreads) void reach_straight_kernel(StraightJob a) {
  extern __shared__ uint32_t lds[];
  const int N = a.N, W = a.W, NW = N * W;
  uint32_t* Rp = lds;
  uint32_t* Hp = lds + NW;
  uint32_t* Op = lds + 2 * NW;
  int16_t* sk = reinterpret_cast<int16_t*>(lds + 3 * NW);
  const int T = blockIdx.x;
  const size_t plane = (size_t)T * NW;
  const bool fam_x = a.family[T] == 0;
  const bool sf_up = a.fwd[T] > 0;
  if (!fam_x) {
    for (int q = threadIdx.x; q < NW; q += blockDim.x) {
      Rp[q] = a.rin[plane + q];
      Hp[q] = a.hard[plane + q];
    }
  } else {
    // row c of the LDS matrices = column c of the plane: each matrix is read
    // into the output area first, then transposed block by block
    for (int m = 0; m < 2; m++) {
      const uint32_t* src = (m == 0 ? a.rin : a.hard) + plane;
      uint32_t* dst = m == 0 ? Rp : Hp;
      for (int q = threadIdx.x; q < NW; q += blockDim.x) Op[q] = src[q];
      __syncthreads();
      transpose_blocks(Op, W, [&](int row, int w, uint32_t v) { dst[row * W + w] = v; });
      __syncthreads();
    }
  }
  for (int q = threadIdx.x; q < NW; q += blockDim.x) Op[q] = ~0u;
  for (int c = threadIdx.x; c < N; c += blockDim.x) sk[c] = a.skew[(size_t)T * N + c];
  __syncthreads();
  // Walkers: (group of 32 lines, direction, section of the walk).  A section
  // maps the entering bits v to (v AND A) OR B (the paper's section value and
  // distance for bits, App. D); sections compose as (A1 A2, B1 A2 | B2).
  const int walkers = 2 * W;
  const int S = blockDim.x / walkers;  // sections per walk (at least 8: W <= 16)
  const int len = (N + S - 1) / S;
  uint32_t* aggA = Op + NW + N / 2 + 1;  // after the skew table
  uint32_t* aggB = aggA + blockDim.x;
  const int item = threadIdx.x % walkers, sec = threadIdx.x / walkers;
  const int g = item % W, dir = item / W;
  const bool on = sec < S && (dir == 0 ? a.sf_on : a.sb_on);
  const bool up = (dir == 0) ? sf_up : !sf_up;
  const int k0 = sec * len, k1 = (k0 + len) < N ? (k0 + len) : N;
  // bits of the 32 lines' poses at walk step k: level window, hard window,
  // and where they sit (word q of row c at bit r, the rest in word q1)
  auto window = [&](int k, uint32_t& rw, uint32_t& hw, int& rb, int& q, int& q1, int& r) {
    const int c = up ? k : (k == 0 ? 0 : N - k);
    const int col = wrapn(32 * g + (int)sk[c], N);
    q = col >> 5;
    r = col & 31;
    q1 = (q + 1 == W) ? 0 : q + 1;
    rb = c * W;
    rw = funnel(Rp[rb + q1], Rp[rb + q], r);
    hw = funnel(Hp[rb + q1], Hp[rb + q], r);
  };
  if (on) {
    uint32_t A = ~0u, B = 0u;
    for (int k = k0; k < k1; k++) {
      uint32_t rw, hw;
      int rb, q, q1, r;
      window(k, rw, hw, rb, q, q1, r);
      A &= rw;
      B = (B & rw) | hw;
    }
    aggA[threadIdx.x] = A;
    aggB[threadIdx.x] = B;
  }
  __syncthreads();
  if (on) {
    uint32_t v = ~0u;  // every line enters from the wall unreachable
    for (int t = 0; t < sec; t++) v = (v & aggA[t * walkers + item]) | aggB[t * walkers + item];
    for (int k = k0; k < k1; k++) {
      uint32_t rw, hw;
      int rb, q, q1, r;
      window(k, rw, hw, rb, q, q1, r);
      v = (v & rw) | hw;
      const uint32_t reach = ~v;  // line t reaches column col + t of row c
      if (reach) {
        atomicAnd(&Op[rb + q], ~(reach << r));
        if (r) atomicAnd(&Op[rb + q1], ~(reach >> (32 - r)));
      }
    }
  }
  __syncthreads();
  if (!fam_x) {
    for (int q = threadIdx.x; q < NW; q += blockDim.x)
      a.rout[plane + q] = a.store ? Op[q] : (a.rout[plane + q] & Op[q]);
  } else {
    // transposed back on the way out
    uint32_t* out = a.rout + plane;
    const bool store = a.store != 0;
    transpose_blocks(Op, W, [&](int row, int w, uint32_t v) {
      uint32_t* dst = out + (size_t)row * W + w;
      *dst = store ? v : (*dst & v);
    });
  }
}

template <int P>
hipError_t launch_turn_t(const TurnJob& j, int blocks, int threads, hipStream_t s) {
  hipLaunchKernelGGL(reach_turn_kernel<P>, dim3(blocks), dim3(threads), 0, s, j);
  return hipGetLastError();
}

bool has(const uint8_t* schedule, int n, int mu) {
  for (int k = 0; k < n; k++)
    if (schedule[k] == mu) return true;
  return false;
}

}  // namespace

hipError_t launch_reach_render(const ReachDev& r, const uint8_t* image, int n_side, int n_len, hipStream_t s) {
  const int NW = r.N * r.W;
  hipLaunchKernelGGL(reach_image_kernel, dim3((NW + 255) / 256), dim3(256), 0, s, image, r.img, r.N, r.W);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reach_render_kernel, dim3(r.L), dim3(256), 0, s, r.img, r.taps, r.hard, r.N, r.W, n_side, n_len);
  return hipGetLastError();
}

hipError_t launch_reach_pack(const ReachDev& r, const uint8_t* codes, hipStream_t s) {
  const size_t blocks = (r.vol_words + 255) / 256;
  hipLaunchKernelGGL(reach_pack_kernel, dim3((unsigned)blocks), dim3(256), 0, s, codes, r.hard, r.N, r.W,
                     r.vol_words);
  return hipGetLastError();
}

hipError_t launch_reach_start(const ReachDev& r, uint32_t start_index, hipStream_t s) {
  size_t blocks = (r.vol_words + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(reach_start_kernel, dim3((unsigned)blocks), dim3(256), 0, s, r.levels, r.vol_words, start_index);
  return hipGetLastError();
}

// The straight kernel's LDS can exceed the default dynamic limit (up to
// 101 KB at N = 512); set once per device before any launch or capture.
hipError_t prepare_reach_kernels() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(reach_straight_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (3 * kReachMaxN * (kReachMaxN / 32) + kReachMaxN / 2 + 1 + 2 * kStraightThreads) * 4);
}

hipError_t launch_reach_cycle(const ReachDev& r, const uint8_t* schedule, int n_schedule, uint32_t m, hipStream_t s) {
  const uint32_t* rin = r.levels + (size_t)m * r.vol_words;
  uint32_t* rout = r.levels + (size_t)(m + 1) * r.vol_words;
  int store = 1;
  // turn families: left circles (LF up the headings, LB down), right
  // circles (RB up, RF down), eqs. (25)-(28)
  // the shortest sections (most parallel lanes) whose lanes fit a workgroup
  int Wp = 1;
  while (Wp < r.W) Wp <<= 1;
  int P = 4;
  while (P < 32 && ((r.L + P - 1) / P) * Wp > kTurnThreads) P <<= 1;
  const int S = (r.L + P - 1) / P;
  if (S * Wp > kTurnThreads) return hipErrorInvalidValue;  // the plan's checks keep L and N below this
  int rows = kTurnThreads / (Wp * S);
  if (rows < 1) rows = 1;
  const int threads = S * rows * Wp, blocks = (r.N + rows - 1) / rows;
  for (int fam = 0; fam < 2; fam++) {
    const int up = fam == 0 ? NHP_LF : NHP_RB, down = fam == 0 ? NHP_LB : NHP_RF;
    const bool fwd_on = has(schedule, n_schedule, up), bwd_on = has(schedule, n_schedule, down);
    if (!fwd_on && !bwd_on) continue;
    TurnJob j{};
    j.rin = rin;
    j.rout = rout;
    j.hard = r.hard;
    j.offx = r.turn_off + (fam == 0 ? 0 : 2) * r.L;
    j.offy = r.turn_off + (fam == 0 ? 1 : 3) * r.L;
    j.N = r.N;
    j.L = r.L;
    j.W = r.W;
    j.Wp = Wp;
    j.rows = rows;
    j.S = S;
    j.fwd_on = fwd_on;
    j.bwd_on = bwd_on;
    j.store = store;
    store = 0;
    hipError_t e;
    switch (P) {
      case 4: e = launch_turn_t<4>(j, blocks, threads, s); break;
      case 8: e = launch_turn_t<8>(j, blocks, threads, s); break;
      case 16: e = launch_turn_t<16>(j, blocks, threads, s); break;
      case 32: e = launch_turn_t<32>(j, blocks, threads, s); break;
      default: e = hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
  }
  const bool sf = has(schedule, n_schedule, NHP_SF), sb = has(schedule, n_schedule, NHP_SB);
  if (sf || sb) {
    StraightJob j{};
    j.rin = rin;
    j.rout = rout;
    j.hard = r.hard;
    j.skew = r.skew;
    j.family = r.family;
    j.fwd = r.fwd;
    j.N = r.N;
    j.W = r.W;
    j.sf_on = sf;
    j.sb_on = sb;
    j.store = store;
    // three bit matrices, the skew table (rounded up to words), two section
    // aggregates per thread
    const size_t lds = ((size_t)3 * r.N * r.W + r.N / 2 + 1 + 2 * kStraightThreads) * 4;
    hipLaunchKernelGGL(reach_straight_kernel, dim3(r.L), dim3(kStraightThreads), lds, s, j);
    return hipGetLastError();
  }
  return hipSuccess;
}

}  // namespace nhp
