// k_sweep.hip -- the maneuver kernels (Sec. VIII.B, Insert 1) for gfx950.
//
// One maneuver kernel relaxes every pose once along the curves of one
// maneuver.  Per pose p in curve order, with u = V(p) and w = weight of the
// edge leaving p:
//     out = min(v, u)            stored to V(p)   (INF if p is hard)
//     v   = min(v, u + ct) + w   carried to the next pose
// Each pose is an affine min-plus map v -> min(v + D, C) with D = w and
// C = u + ct + w (a hard pose is (INF, INF), a reset), and these maps compose
// associatively: (D1, C1) then (D2, C2) = (D1 + D2, min(C1 + D2, C2)).  That
// is the section value / section distance pair of the paper's Sections
// technique (App. D, Inserts 3-5).  All additions saturate at INF.
//
// Work decomposition (one HBM read and one write per pose):
//   * a workgroup owns 64 curves (one per lane) over their full length;
//   * wave w of the S waves holds steps [wP, (w+1)P) of every curve in
//     registers (values, and the obstacle codes packed 4 per register);
//   * each wave composes its section into one (D, C) per curve, the S pairs
//     meet in LDS, and each wave derives the value entering its section:
//     for turns the fixed point of the cyclic composition (equal to the
//     paper's two loops around the circle), for straights the composition of
//     the sections before it, starting from INF at the wall;
//   * each wave replays its section from registers and stores.
// Turn curves and y-major straight lines put the 64 lanes on 64 consecutive
// x of one row, so every load and store is a contiguous row segment.  The
// x-major straight family (|tan| <= 1) puts the lanes on a column instead;
// those planes are loaded and stored row-wise into an LDS tile per wave and
// transposed there.
#include "nhp_internal.h"

namespace nhp {
namespace {

__device__ __forceinline__ uint32_t sadd(uint32_t a, uint32_t b) { return __builtin_elementwise_add_sat(a, b); }
__device__ __forceinline__ uint32_t umin(uint32_t a, uint32_t b) { return a < b ? a : b; }

// Edge weight (Lq * (256 + 4 code) + 128) >> 8, infinite for a hard code.
// base = 256 Lq + 128, lq4 = 4 Lq (Lq <= 2^21 keeps the sum below 2^32).
__device__ __forceinline__ uint32_t weight(uint32_t code, uint32_t base, uint32_t lq4) {
  const uint32_t w = (base + lq4 * code) >> 8;
  return code == kHard ? kInf : w;
}

__device__ __forceinline__ uint32_t code_of(const uint32_t* packed, int k) {
  return (packed[k >> 2] >> ((k & 3) * 8)) & 0xffu;
}

typedef uint16_t code2 __attribute__((ext_vector_type(2)));

// Value volume access by 32-bit cell index.  The byte offset is formed in
// 32 bits (volumes hold at most 2^30 poses), so the access is a uniform
// 64-bit base plus a 32-bit per-lane offset (global_load ... saddr).
__device__ __forceinline__ uint32_t ld_value(const uint32_t* V, uint32_t cell) {
  return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(V) + (cell << 2));
}
__device__ __forceinline__ void st_value(uint32_t* V, uint32_t cell, uint32_t v) {
  *reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(V) + (cell << 2)) = v;
}

__device__ __forceinline__ uint32_t code_of(const code2* packed, int k) { return packed[k >> 1][k & 1]; }

// Workgroup index spread over the 8 XCDs so that consecutive tiles (which
// share row segments at their edges) land on the same XCD and its L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int per = n >> 3, rem = n & 7, x = b & 7, k = b >> 3;
  return x * per + (x < rem ? x : rem) + k;
}

// Workgroup barrier that waits only for this wave's LDS operations, not for
// its outstanding global loads (__syncthreads waits for both), so loads
// issued for the next chunk stay in flight across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

struct SweepArgs {
  uint32_t* V;
  const uint8_t* B;
  int N;       // cells per side
  int L;       // curve length (N_theta for turns, N for straights)
  uint32_t ct;
};

// Value entering this wave's section: cyclic fixed point (turns) or the
// composition of the earlier sections from INF (straights).
template <bool CYCLIC>
__device__ __forceinline__ uint32_t section_carry(const uint32_t (*aggD)[64], const uint32_t (*aggC)[64],
                                                  int S, int wave, int lane) {
  uint32_t C = kInf;
  if (CYCLIC) {
    int s = wave;
    for (int t = 0; t < S; t++) {
      C = umin(sadd(C, aggD[s][lane]), aggC[s][lane]);
      s = (s + 1 == S) ? 0 : s + 1;
    }
  } else {
    for (int s = 0; s < wave; s++) C = umin(sadd(C, aggD[s][lane]), aggC[s][lane]);
  }
  return C;
}

// Row-coalesced sweep: turns (CYCLIC) and y-major straights.
//   turns:     block -> (x tile, y'); step k -> plane T_k, offsets (ox, oy)
//   straights: block -> (x tile, plane); step k -> row c_k, column x' + B(c_k)
template <int P, bool CYCLIC>
__global__ __launch_bounds__(1024) void row_sweep_kernel(SweepArgs a, const int32_t* __restrict__ offx,
                                                        const int32_t* __restrict__ offy, int asc,
                                                        uint32_t lq_base, uint32_t lq4,
                                                        // straights only:
                                                        const int16_t* __restrict__ skew,
                                                        const int32_t* __restrict__ planes,
                                                        const uint32_t* __restrict__ edge_len,
                                                        const int32_t* __restrict__ fwd, int mu_forward) {
  __shared__ uint32_t aggD[16][64];
  __shared__ uint32_t aggC[16][64];
  __shared__ uint32_t wlut[256];  // edge weight by obstacle code (INF for hard)
  const int S = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int N = a.N, L = a.L;
  const int tiles_x = (N + 63) >> 6;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tx = tile % tiles_x;
  const int outer = tile / tiles_x;  // y' (turns) or plane slot (straights)
  const int xp = tx * 64 + lane;
  const bool active = xp < N;

  int T0 = 0;
  uint32_t base = lq_base, l4 = lq4;
  int dir = asc;
  const int16_t* sk = nullptr;
  if (!CYCLIC) {
    T0 = planes[outer];
    const uint32_t Lq = edge_len[T0];
    base = 256u * Lq + 128u;
    l4 = 4u * Lq;
    dir = (fwd[T0] > 0) == (mu_forward != 0);
    sk = skew + (size_t)T0 * N;
  }
  for (int c = threadIdx.x; c < 256; c += blockDim.x) wlut[c] = weight((uint32_t)c, base, l4);

  uint32_t u[P];
  uint32_t code[P];

  // Step k of this wave's section touches row `row` of plane T, columns
  // (xp + shift) mod N: a uniform row base plus a small per-lane column.
  // Sections are P steps; steps past the curve length (when S P > L) are
  // identity maps that touch no memory.
  auto step_geometry = [&](int k, int& T, int& row, int& shift) {
    int step = wave * P + k;
    step = step < L ? step : L - 1;
    if (CYCLIC) {
      T = dir ? step : (L - 1 - step);
      shift = offx[T];
      row = outer + offy[T];
      row -= (row >= N) ? N : 0;
    } else {
      T = T0;
      const int c = dir ? step : (L - 1 - step);
      shift = sk[c];
      shift += (shift < 0) ? N : 0;
      row = c;
    }
  };
  const int n_real = (L - wave * P) < P ? (L - wave * P) : P;  // real steps of this wave

  // Load this wave's section of the 64 curves.  Lanes past the grid edge
  // read a valid cell, so the loads carry no branch.
  const int xl = active ? xp : N - 1;
#pragma unroll
  for (int k = 0; k < P; k++) {
    int T, row, shift;
    step_geometry(k, T, row, shift);
    const uint32_t rbase = ((uint32_t)T * (uint32_t)N + (uint32_t)row) * (uint32_t)N;
    int i = xl + shift;
    i -= (i >= N) ? N : 0;
    // lanes are independent curves: an idle lane computes on its clamped
    // cell and never stores, so loaded values need no masking
    const uint32_t cell = rbase + (uint32_t)i;
    u[k] = ld_value(a.V, cell);
    code[k] = a.B[cell];
  }

  __syncthreads();  // weight table ready
  // weights replace the codes in place; compose the section into (D, C):
  // min(C + w, u + ct + w) = min(C, u + ct) + w (saturating add is monotone)
  uint32_t D = 0, C = kInf;
#pragma unroll
  for (int k = 0; k < P; k++) code[k] = wlut[code[k]];
#pragma unroll
  for (int k = 0; k < P; k++) {
    if (k < n_real) {
      C = sadd(umin(C, sadd(u[k], a.ct)), code[k]);
      D = sadd(D, code[k]);
    }
  }
  aggD[wave][lane] = D;
  aggC[wave][lane] = C;
  __syncthreads();
  uint32_t v = section_carry<CYCLIC>(aggD, aggC, S, wave, lane);

  // replay: a hard pose has weight INF, and w >> 31 (arithmetic) is then all
  // ones, which forces its output to INF
#pragma unroll
  for (int k = 0; k < P; k++) {
    const uint32_t w = code[k];
    const uint32_t uu = u[k];
    u[k] = umin(v, uu) | (uint32_t)((int32_t)w >> 31);
    v = sadd(umin(v, sadd(uu, a.ct)), w);
  }
  // recompute the column of every step rather than keeping P of them live
  int xs = xp;
  asm volatile("" : "+v"(xs));
  if (active) {
#pragma unroll
    for (int k = 0; k < P; k++) {
      if (k < n_real) {
        int T, row, shift;
        step_geometry(k, T, row, shift);
        const uint32_t rbase = ((uint32_t)T * (uint32_t)N + (uint32_t)row) * (uint32_t)N;
        int i = xs + shift;
        i -= (i >= N) ? N : 0;
        st_value(a.V, rbase + (uint32_t)i, u[k]);
      }
    }
  }
}

// x-major straights (|tan| <= 1): line x' visits (c, x' + B(c)), so lines
// that are neighbours in x' sit in different rows at every step and a lane
// per line would read a column.  A workgroup of 4 waves owns 64 lines and
// walks them along c in chunks of Q columns.  Per chunk the cells owned by
// its lines form a sheared band of at most 64 + Q rows; they are loaded row
// by row (contiguous segments, each cell exactly once) into an LDS tile, the
// four waves scan Q/4 columns each for all 64 lines (section composition in
// LDS, carry from the previous chunk), write the results back into the tile,
// and the tile is stored row by row.
template <int Q>
__global__ __launch_bounds__(256) void xmajor_sweep_kernel(SweepArgs a, const int16_t* __restrict__ skew,
                                                          const int32_t* __restrict__ planes,
                                                          const uint32_t* __restrict__ edge_len,
                                                          const int32_t* __restrict__ fwd, int mu_forward) {
  constexpr int LINES = 64;
  constexpr int R = LINES + Q;        // rows a chunk can touch (|B(c+1) - B(c)| <= 1)
  constexpr int PITCH = Q + 1;        // odd pitch: a column read by 64 lanes hits 64 banks
  constexpr int SUB = Q / 4;          // columns per wave
  constexpr int ITER = (R * Q + 255) / 256;
  static_assert(256 % Q == 0, "Q must divide 256");
  __shared__ uint32_t tV[R * PITCH];
  __shared__ uint8_t tB[R * PITCH];
  __shared__ int32_t tS[Q];
  __shared__ uint32_t aggD[4][64];
  __shared__ uint32_t aggC[4][64];
  __shared__ uint32_t wlut[256];
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int N = a.N;
  const int tiles_x = (N + LINES - 1) / LINES;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int x0 = (tile % tiles_x) * LINES;
  const int T = planes[tile / tiles_x];
  const uint32_t plane = (uint32_t)T * (uint32_t)N * (uint32_t)N;
  const uint32_t Lq = edge_len[T];
  wlut[tid] = weight((uint32_t)tid, 256u * Lq + 128u, 4u * Lq);
  const int dir = (fwd[T] > 0) == (mu_forward != 0);
  const int16_t* sk = skew + (size_t)T * N;
  const int kk = tid % Q;       // column of this thread in the load/store phases
  const int r0 = tid / Q;       // first row of this thread; rows r0 + it * (256 / Q)
  const bool line_ok = x0 + lane < N;

  uint32_t carry = kInf;        // value carried along line x0 + lane into the chunk
  for (int k0 = 0; k0 < N; k0 += Q) {
    const int nq = (N - k0) < Q ? (N - k0) : Q;
    const int c_first = dir ? k0 : (N - 1 - k0);
    const int c_last = dir ? (k0 + nq - 1) : (N - 1 - (k0 + nq - 1));
    const int b_first = sk[c_first], b_last = sk[c_last];
    const int bmin = b_first < b_last ? b_first : b_last;
    const int rows = LINES + (b_first > b_last ? b_first - b_last : b_last - b_first);
    int rowbase = (x0 + bmin) % N;
    rowbase += (rowbase < 0) ? N : 0;
    const int my_c = dir ? (k0 + kk) : (N - 1 - (k0 + kk));
    const bool col_ok = kk < nq;
    const int my_b = col_ok ? (int)sk[my_c] : 0;
    if (tid < Q) tS[tid] = my_b;

    // load the band: every owned cell once, rows as contiguous segments
    uint32_t lv[ITER], lc[ITER];
    uint32_t cell[ITER];
    bool own[ITER];
#pragma unroll
    for (int it = 0; it < ITER; it++) {
      const int r = r0 + it * (256 / Q);
      const int t = r + bmin - my_b;
      own[it] = col_ok && r < rows && t >= 0 && t < LINES && x0 + t < N;
      int row = rowbase + r;
      row = row >= N ? row % N : row;
      cell[it] = own[it] ? plane + (uint32_t)row * (uint32_t)N + (uint32_t)my_c : plane;
      lv[it] = ld_value(a.V, cell[it]);
      lc[it] = a.B[cell[it]];
    }
#pragma unroll
    for (int it = 0; it < ITER; it++) {
      if (own[it]) {
        const int r = r0 + it * (256 / Q);
        tV[r * PITCH + kk] = lv[it];
        tB[r * PITCH + kk] = (uint8_t)lc[it];
      }
    }
    __syncthreads();

    // scan: wave w takes columns [w SUB, (w+1) SUB) of the chunk for all 64 lines
    uint32_t u[SUB], w[SUB];
    int rr[SUB];
#pragma unroll
    for (int q = 0; q < SUB; q++) {
      const int kq = wave * SUB + q;
      const bool ok = kq < nq;
      rr[q] = ok ? lane + tS[kq] - bmin : 0;  // in [0, rows) for real columns
      u[q] = ok ? tV[rr[q] * PITCH + kq] : kInf;
      w[q] = ok ? wlut[tB[rr[q] * PITCH + kq]] : 0u;
    }
    uint32_t D = 0, C = kInf;
#pragma unroll
    for (int q = 0; q < SUB; q++) {
      const bool ok = wave * SUB + q < nq;
      C = ok ? sadd(umin(C, sadd(u[q], a.ct)), w[q]) : C;
      D = sadd(D, w[q]);
    }
    aggD[wave][lane] = D;
    aggC[wave][lane] = C;
    __syncthreads();
    uint32_t v = carry;
    for (int s = 0; s < wave; s++) v = umin(sadd(v, aggD[s][lane]), aggC[s][lane]);
#pragma unroll
    for (int q = 0; q < SUB; q++) {
      const int kq = wave * SUB + q;
      if (kq < nq && line_ok) {
        tV[rr[q] * PITCH + kq] = umin(v, u[q]) | (uint32_t)((int32_t)w[q] >> 31);
        v = sadd(umin(v, sadd(u[q], a.ct)), w[q]);
      }
    }
    for (int s = 0; s < 4; s++) carry = umin(sadd(carry, aggD[s][lane]), aggC[s][lane]);
    __syncthreads();

    // store the band back
#pragma unroll
    for (int it = 0; it < ITER; it++) {
      if (own[it]) {
        const int r = r0 + it * (256 / Q);
        st_value(a.V, cell[it], tV[r * PITCH + kk]);
      }
    }
    __syncthreads();
  }
}

__global__ void init_kernel(uint32_t* __restrict__ V, size_t n4, uint32_t start) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n4; q += stride) {
    const size_t e = q * 4;
    uint4 v = make_uint4(kInf, kInf, kInf, kInf);
    if (start >= e && start < e + 4) {
      const uint32_t o = (uint32_t)(start - e);
      if (o == 0) v.x = 0;
      if (o == 1) v.y = 0;
      if (o == 2) v.z = 0;
      if (o == 3) v.w = 0;
    }
    reinterpret_cast<uint4*>(V)[q] = v;
  }
}

__global__ void walls_kernel(uint8_t* __restrict__ B, int N, int L) {
  // one block per plane: row j = 0 and column i = 0 are hard
  const size_t base = (size_t)blockIdx.x * N * N;
  for (int k = threadIdx.x; k < N; k += blockDim.x) {
    B[base + k] = (uint8_t)kHard;
    B[base + (size_t)k * N] = (uint8_t)kHard;
  }
}

// Steps per wave: the smallest power of two in [8, 64] that splits the curve
// into at most 16 sections (16 waves of a 1024-thread workgroup).
constexpr int XQ = 32;  // columns per x-major chunk

int pick_section(int len) {
  int P = 8;
  while (P < 64 && P * 16 < len) P <<= 1;
  return (P * 16 >= len) ? P : 0;
}

template <bool CYCLIC>
hipError_t launch_row(int P, dim3 grid, dim3 block, hipStream_t s, SweepArgs a, const int32_t* offx,
                      const int32_t* offy, int asc, uint32_t base, uint32_t l4, const int16_t* skew,
                      const int32_t* planes, const uint32_t* edge_len, const int32_t* fwd, int mu_fwd) {
  switch (P) {
    case 64:
      hipLaunchKernelGGL((row_sweep_kernel<64, CYCLIC>), grid, block, 0, s, a, offx, offy, asc, base, l4, skew, planes,
                         edge_len, fwd, mu_fwd);
      break;
    case 32:
      hipLaunchKernelGGL((row_sweep_kernel<32, CYCLIC>), grid, block, 0, s, a, offx, offy, asc, base, l4, skew, planes,
                         edge_len, fwd, mu_fwd);
      break;
    case 16:
      hipLaunchKernelGGL((row_sweep_kernel<16, CYCLIC>), grid, block, 0, s, a, offx, offy, asc, base, l4, skew, planes,
                         edge_len, fwd, mu_fwd);
      break;
    case 8:
      hipLaunchKernelGGL((row_sweep_kernel<8, CYCLIC>), grid, block, 0, s, a, offx, offy, asc, base, l4, skew, planes,
                         edge_len, fwd, mu_fwd);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_init(const DevPlan& d, uint32_t start_index, hipStream_t s) {
  const size_t NR = (size_t)d.nx * d.nx * d.nt;  // a multiple of 64: nx and nt are multiples of 8
  const size_t n4 = NR / 4;
  size_t blocks = (n4 + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(init_kernel, dim3((unsigned)blocks), dim3(256), 0, s, d.V, n4, start_index);
  return hipGetLastError();
}

hipError_t launch_force_walls(const DevPlan& d, hipStream_t s) {
  hipLaunchKernelGGL(walls_kernel, dim3(d.nt), dim3(256), 0, s, d.B, d.nx, d.nt);
  return hipGetLastError();
}

hipError_t launch_sweep(const DevPlan& d, int mu, hipStream_t s) {
  const int N = d.nx, L = d.nt;
  const int tiles_x = (N + 63) / 64;
  SweepArgs a{d.V, d.B, N, L, d.ct[mu]};
  if (mu == NHP_SF || mu == NHP_SB) {
    const int P = pick_section(N);
    if (!P) return hipErrorInvalidValue;
    const int S = (N + P - 1) / P;
    a.L = N;
    const int mu_fwd = (mu == NHP_SF);
    const uint32_t* el = d.edge_len + (size_t)mu * L;
    hipError_t e = hipSuccess;
    if (d.n_planes_y > 0) {
      e = launch_row<false>(P, dim3(tiles_x * d.n_planes_y), dim3(64 * S), s, a, nullptr, nullptr, 0, 0, 0, d.skew,
                            d.planes + d.n_planes_x, el, d.fwd, mu_fwd);
      if (e != hipSuccess) return e;
    }
    if (d.n_planes_x > 0) {
      hipLaunchKernelGGL((xmajor_sweep_kernel<XQ>), dim3(tiles_x * d.n_planes_x), dim3(256), 0, s, a, d.skew,
                         d.planes, el, d.fwd, mu_fwd);
      e = hipGetLastError();
    }
    return e;
  }
  const int P = pick_section(L);
  if (!P) return hipErrorInvalidValue;
  const int S = (L + P - 1) / P;
  const bool left = (mu == NHP_LF || mu == NHP_LB);
  const int asc = (mu == NHP_LF || mu == NHP_RB);  // eqs. (25)-(28): LF, RB step to T+1
  const int32_t* offx = d.turn_off + (left ? 0 : 2) * L;
  const int32_t* offy = d.turn_off + (left ? 1 : 3) * L;
  const uint32_t Lq = d.turn_lq[mu];
  return launch_row<true>(P, dim3(tiles_x * N), dim3(64 * S), s, a, offx, offy, asc, 256u * Lq + 128u, 4u * Lq,
                          nullptr, nullptr, nullptr, nullptr, 0);
}

}  // namespace nhp
