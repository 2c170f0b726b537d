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
// A unit of work is a job (one maneuver of one plan); a batched launch
// covers the tiles of many jobs, each block finding its job by a binary
// search over the jobs' first block.
// Turn curves and y-major straight lines put the 64 lanes on 64 consecutive
// x of one row, so every load and store is a contiguous row segment.  The
// x-major straight family (|tan| <= 1) puts the lanes on a column instead;
// those planes are loaded and stored row-wise into an LDS tile per wave and
// transposed there.
#include <atomic>

#include "nhp_internal.h"

// Structured buffer access to the sweep kernels' volumes: the record index is
// the pose index for both the 4-byte values and the 1-byte codes, so one
// per-lane index addresses both (the hardware applies the record size), and
// indices at or past the record count read 0 and drop stores instead of
// touching memory.  (The compiler's structured-buffer operations, declared
// by their intrinsic names.)
__device__ uint32_t buffer_load_u32(__amdgpu_buffer_rsrc_t r, uint32_t index, uint32_t voffset, uint32_t soffset,
                                    int aux) __asm("llvm.amdgcn.struct.ptr.buffer.load.i32");
__device__ uint8_t buffer_load_u8(__amdgpu_buffer_rsrc_t r, uint32_t index, uint32_t voffset, uint32_t soffset,
                                  int aux) __asm("llvm.amdgcn.struct.ptr.buffer.load.i8");
__device__ void buffer_store_u32(uint32_t v, __amdgpu_buffer_rsrc_t r, uint32_t index, uint32_t voffset,
                                 uint32_t soffset, int aux) __asm("llvm.amdgcn.struct.ptr.buffer.store.i32");

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

// A column in [0, 2N) reduced to [0, N): the unsigned i - N wraps above i
// whenever i < N, so the smaller of the two is the reduced column.
__device__ __forceinline__ uint32_t wrap_col(uint32_t i, int N) {
  const uint32_t j = i - (uint32_t)N;
  return j < i ? j : i;
}

// Index of the pose at column (x + shift) mod N of the row starting at pose
// rb (a multiple of N).  For a power-of-two N the geometry table holds
// g = rb | shift, and the pose is g + x with the carry out of the column
// bits dropped: the low bits of g + x spliced onto the high bits of g
// (one bitfield insert).
template <bool POW2>
__device__ __forceinline__ uint32_t row_cell(uint32_t g, uint32_t x, uint32_t shift, int N) {
  if (POW2) {
    const uint32_t m = (uint32_t)N - 1u;
    uint32_t r;
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "s"(m), "v"(g + x), "v"(g));  // (sum & m) | (g & ~m)
    return r;
  }
  return g + wrap_col(x + shift, N);
}

constexpr int kBufferWord3 = 0x00020000;  // descriptor word 3 for untyped access on gfx9-family GPUs

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct RowBuffers {
  __amdgpu_buffer_rsrc_t V, B;
};
__device__ __forceinline__ RowBuffers row_buffers(const SweepJob& a) {
  return {__builtin_amdgcn_make_buffer_rsrc(a.V, (short)4, (int)a.n_poses, kBufferWord3),
          __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(a.B), (short)1, (int)a.n_poses, kBufferWord3)};
}

// A job's tables are global memory; saying so lets the compiler read them
// with global rather than generic loads (a job read from a batched job
// table otherwise reaches them through generic pointers).
template <typename T>
using GlobalPtr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ GlobalPtr<T> as_global(T* p) {
  return (GlobalPtr<T>)p;
}

// Workgroup index spread over the 8 XCDs so that consecutive tiles (which
// share row segments at their edges) land on the same XCD and its L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int per = n >> 3, rem = n & 7, x = b & 7, k = b >> 3;
  return x * per + (x < rem ? x : rem) + k;
}

// Tile of workgroup slot b of n: XCD-aware (order 1) or launch order (order 2).
__device__ __forceinline__ int tile_of(int b, int n, int order) { return order == 2 ? b : xcd_tile(b, n); }

// Value entering this wave's section: the cyclic fixed point (turns) or the
// composition of the earlier sections from INF (straights).  Sections are
// visited in increasing order (forward) or decreasing order (the second
// maneuver of a fused pair, which walks the curves backwards).
template <bool BACKWARD = false>
__device__ __forceinline__ uint32_t section_carry(const uint32_t (*aggD)[64], const uint32_t (*aggC)[64], int S,
                                                  int wave, int lane, bool cyclic) {
  uint32_t C = kInf;
  if (cyclic) {
    // once around, starting with this section and ending with the one before it
    int s = wave;
    for (int t = 0; t < S; t++) {
      C = umin(sadd(C, aggD[s][lane]), aggC[s][lane]);
      if (BACKWARD)
        s = (s == 0) ? S - 1 : s - 1;
      else
        s = (s + 1 == S) ? 0 : s + 1;
    }
  } else if (BACKWARD) {
    for (int s = S - 1; s > wave; s--) C = umin(sadd(C, aggD[s][lane]), aggC[s][lane]);
  } else {
    for (int s = 0; s < wave; s++) C = umin(sadd(C, aggD[s][lane]), aggC[s][lane]);
  }
  return C;
}

struct RowShared {
  uint32_t aggD[16][64];
  uint32_t aggC[16][64];
  uint32_t aggD2[16][64];  // second maneuver of a fused pair
  uint32_t aggC2[16][64];
  uint32_t wlut[256];      // edge weight by obstacle code (INF for hard)
  uint32_t wlut2[256];     // the same for the second maneuver
  uint32_t row_base[1024]; // per step: index of the first pose of the row it reads
                           // (power-of-two N: OR the column offset below)
  uint16_t shift[1024];    // per step: column offset of curve x' (reduced mod N)
};

// The scan phases of one section held in registers, then its stores.
// GUARD: the curve length is not a multiple of P, so the last section has
// fewer than P real steps and the steps past the curve are skipped (without
// it every section is full and the loops carry no conditions).
// Write elision: a pass changes few poses once the search front has gone
// by (about 5 % of the poses and 11 % of the 128-byte lines per pass of a
// 512^3 maze plan), so a wave does not store a step whose 64 values are all
// unchanged (memory already holds them).  The test is per wave and step: a
// ballot in the replay, one bit per step, and a uniform branch at the store
// (no per-lane work; a step with any change stores all its lanes).
template <int P, bool FUSED, bool GUARD, bool POW2, bool ELIDE>
__device__ __forceinline__ void scan_section(const SweepJob& a, const RowBuffers& buf, RowShared& sh,
                                             uint32_t (&u)[P], uint32_t (&code)[P], int n_real, int S, int wave,
                                             int lane, bool cyclic, bool active, int xp, int first, int N) {
  uint32_t packed[FUSED ? P / 4 : 1];
  uint32_t changed = 0;  // bit k: some lane's value at step k changed (wave-uniform)
  static_assert(!ELIDE || P <= 32, "one bit per step");
  {
    // weights replace the codes; compose the section into (D, C):
    // min(C + w, u + ct + w) = min(C, u + ct) + w (saturating add is monotone).
    // A fused pair keeps the codes, packed four to a register, for the
    // second maneuver's weights (packing after the loads have landed, so it
    // does not hold the loads back).
    uint32_t D = 0, C = kInf;
    if (FUSED) {
#pragma unroll
      for (int q = 0; q < P / 4; q++)
      {
        packed[q] = code[4 * q] | (code[4 * q + 1] << 8) | (code[4 * q + 2] << 16) | (code[4 * q + 3] << 24);
        asm volatile("" : "+v"(packed[q]));  // keep the packed form (not P live codes)
      }
    }
#pragma unroll
    for (int k = 0; k < P; k++) code[k] = sh.wlut[code[k]];
#pragma unroll
    for (int k = 0; k < P; k++) {
      if (!GUARD || k < n_real) {
        C = sadd(umin(C, sadd(u[k], a.ct)), code[k]);
        D = sadd(D, code[k]);
      }
    }
    sh.aggD[wave][lane] = D;
    sh.aggC[wave][lane] = C;
  }
  __syncthreads();
  {
    uint32_t v = section_carry(sh.aggD, sh.aggC, S, wave, lane, cyclic);
    // replay: a hard pose has weight INF, and w >> 31 (arithmetic) is then
    // all ones, which forces its output to INF (weights of other codes stay
    // below 2^24).  A fused pair forces it only in the second replay: until
    // then a hard pose's value only ever enters a step whose weight is INF,
    // which returns INF whatever the value, so it cannot change any result.
#pragma unroll
    for (int k = 0; k < P; k++) {
      const uint32_t w = code[k];
      const uint32_t uu = u[k];
      u[k] = FUSED ? umin(v, uu) : (umin(v, uu) | (uint32_t)((int32_t)w >> 31));
      if (ELIDE) {
        // fold each step's mask into its bit now (not 32 masks held in registers)
        changed = (uint32_t)__builtin_amdgcn_readfirstlane(
            (int)(changed | ((__builtin_amdgcn_ballot_w64(u[k] != uu) != 0ull ? 1u : 0u) << k)));
      }
      v = sadd(umin(v, sadd(uu, a.ct)), w);
    }
    if (FUSED) {
      // second maneuver: the steps of the section in reverse order, its
      // weights replacing the codes
      uint32_t D2 = 0, C2 = kInf;
#pragma unroll
      for (int k = P - 1; k >= 0; k--) {
        if (!GUARD || k < n_real) {
          code[k] = sh.wlut2[(packed[k >> 2] >> (8 * (k & 3))) & 0xffu];
          C2 = sadd(umin(C2, sadd(u[k], a.ct2)), code[k]);
          D2 = sadd(D2, code[k]);
        }
      }
      sh.aggD2[wave][lane] = D2;
      sh.aggC2[wave][lane] = C2;
    }
  }
  if (FUSED) {
    __syncthreads();
    uint32_t v = section_carry<true>(sh.aggD2, sh.aggC2, S, wave, lane, cyclic);
#pragma unroll
    for (int k = P - 1; k >= 0; k--) {
      if (!GUARD || k < n_real) {
        const uint32_t w = code[k];
        const uint32_t uu = u[k];
        u[k] = umin(v, uu) | (uint32_t)((int32_t)w >> 31);
        if (ELIDE) {
          changed = (uint32_t)__builtin_amdgcn_readfirstlane(
              (int)(changed | ((__builtin_amdgcn_ballot_w64(u[k] != uu) != 0ull ? 1u : 0u) << k)));
        }
        v = sadd(umin(v, sadd(uu, a.ct2)), w);
      }
    }
  }
  // recompute the pose of every step rather than keeping P of them live
  int xs = xp;
  asm volatile("" : "+v"(xs));
  if (active) {
#pragma unroll
    for (int k = 0; k < P; k++) {
      if ((!GUARD || k < n_real) && (!ELIDE || ((changed >> k) & 1u))) {
        buffer_store_u32(u[k], buf.V,
                         row_cell<POW2>(sh.row_base[first + k], (uint32_t)xs, POW2 ? 0u : sh.shift[first + k], N), 0,
                         0, 0);
      }
    }
  }
}

// Sections of 64 steps (curves of up to 1024 poses in 16 waves): the first
// 32 values of a section stay in registers and the other 32 in LDS (128 KB
// for 16 waves), the codes are packed four to a register as they arrive
// (loaded in groups of 16, so that few byte loads hold registers at once),
// and each use reads its weight from the LDS table.  The compiler barriers
// every 8 steps tie the table and LDS reads to the carried value, so only a
// few are live at once (holding all 64 values and weights would spill).
template <int P, bool FUSED, bool GUARD, bool POW2>
__device__ __forceinline__ void scan_section_wide(const SweepJob& a, const RowBuffers& buf, RowShared& sh, int n_real,
                                                  int S, int wave, int lane, bool cyclic, bool active, int xp,
                                                  int first, int L, int N) {
  constexpr int G = 16;      // codes per load group
  constexpr int H = P / 2;   // values kept in registers
  __shared__ uint32_t upper[16][P - H][64];
  // write elision, as in scan_section: bit k of changed[k / 32] says some
  // lane's value at step k changed (wave-uniform)
  uint32_t changed[(P + 31) / 32] = {};
  auto note = [&](int k, uint32_t before, uint32_t after) {
    changed[k >> 5] = (uint32_t)__builtin_amdgcn_readfirstlane(
        (int)(changed[k >> 5] | ((__builtin_amdgcn_ballot_w64(after != before) != 0ull ? 1u : 0u) << (k & 31))));
  };
  uint32_t (*hi)[64] = upper[wave];
  uint32_t u[H], packed[P / 4];
  const int xl = active ? xp : N - 1;
  {
    uint32_t uh[P - H];
#pragma unroll
    for (int k = 0; k < P; k++) {
      const int s = first + k;
      const uint32_t v =
          buffer_load_u32(buf.V, row_cell<POW2>(sh.row_base[s], (uint32_t)xl, POW2 ? 0u : sh.shift[s], N), 0, 0, 0);
      if (k < H)
        u[k] = v;
      else
        uh[k - H] = v;
    }
#pragma unroll
    for (int h = 0; h < P / G; h++) {
      asm volatile("" ::: "memory");
      int xg = xl;
      asm volatile("" : "+v"(xg));  // recompute the cells rather than keep P of them
      uint32_t c[G];
#pragma unroll
      for (int e = 0; e < G; e++) {
        const int k = h * G + e;
        const int s = first + k;
        c[e] = buffer_load_u8(buf.B, row_cell<POW2>(sh.row_base[s], (uint32_t)xg, POW2 ? 0u : sh.shift[s], N), 0, 0,
                              0);
      }
#pragma unroll
      for (int q = 0; q < G / 4; q++) {
        packed[h * (G / 4) + q] = c[4 * q] | (c[4 * q + 1] << 8) | (c[4 * q + 2] << 16) | (c[4 * q + 3] << 24);
        asm volatile("" : "+v"(packed[h * (G / 4) + q]));
      }
    }
#pragma unroll
    for (int k = 0; k < P - H; k++) hi[k][lane] = uh[k];  // a wave reads back only its own slots
  }
  auto weight_of = [&](int k) { return sh.wlut[(packed[k >> 2] >> (8 * (k & 3))) & 0xffu]; };
  {
    uint32_t D = 0, C = kInf;
#pragma unroll
    for (int k = 0; k < P; k++) {
      if ((k & 7) == 0) asm volatile("" : "+v"(C), "+v"(D)::"memory");
      // a step past the curve (GUARD) is the identity map: weight 0, value INF
      const bool real = !GUARD || k < n_real;
      const uint32_t w = real ? weight_of(k) : 0u;
      const uint32_t uk = real ? (k < H ? u[k] : hi[k - H][lane]) : kInf;
      C = sadd(umin(C, sadd(uk, a.ct)), w);
      D = sadd(D, w);
    }
    sh.aggD[wave][lane] = D;
    sh.aggC[wave][lane] = C;
  }
  __syncthreads();
  {
    // opaque: the replay recomputes u + ct and the weights rather than the
    // compiler keeping the compose phase's copies
#pragma unroll
    for (int q = 0; q < P / 4; q++) asm volatile("" : "+v"(packed[q]));
#pragma unroll
    for (int k = 0; k < H; k++) asm volatile("" : "+v"(u[k]));
    uint32_t v = section_carry(sh.aggD, sh.aggC, S, wave, lane, cyclic);
#pragma unroll
    for (int k = 0; k < P; k++) {
      if ((k & 7) == 0) asm volatile("" : "+v"(v)::"memory");
      const bool real = !GUARD || k < n_real;
      const uint32_t w = real ? weight_of(k) : 0u;
      const uint32_t uu = real ? (k < H ? u[k] : hi[k - H][lane]) : kInf;
      // (a fused pair forces hard poses to INF only in its second replay)
      const uint32_t out = FUSED ? umin(v, uu) : (umin(v, uu) | (uint32_t)((int32_t)w >> 31));
      note(k, uu, out);
      if (k < H)
        u[k] = out;
      else
        hi[k - H][lane] = out;
      v = sadd(umin(v, sadd(uu, a.ct)), w);
    }
  }
  if (FUSED) {
    // second maneuver: the steps in reverse order with its own weights
    auto weight2_of = [&](int k) { return sh.wlut2[(packed[k >> 2] >> (8 * (k & 3))) & 0xffu]; };
    {
#pragma unroll
      for (int q = 0; q < P / 4; q++) asm volatile("" : "+v"(packed[q]));
      uint32_t D2 = 0, C2 = kInf;
#pragma unroll
      for (int k = P - 1; k >= 0; k--) {
        if ((k & 7) == 7) asm volatile("" : "+v"(C2), "+v"(D2)::"memory");
        const bool real = !GUARD || k < n_real;
        const uint32_t w = real ? weight2_of(k) : 0u;
        const uint32_t uk = real ? (k < H ? u[k] : hi[k - H][lane]) : kInf;
        C2 = sadd(umin(C2, sadd(uk, a.ct2)), w);
        D2 = sadd(D2, w);
      }
      sh.aggD2[wave][lane] = D2;
      sh.aggC2[wave][lane] = C2;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < P / 4; q++) asm volatile("" : "+v"(packed[q]));
#pragma unroll
    for (int k = 0; k < H; k++) asm volatile("" : "+v"(u[k]));
    uint32_t v = section_carry<true>(sh.aggD2, sh.aggC2, S, wave, lane, cyclic);
#pragma unroll
    for (int k = P - 1; k >= 0; k--) {
      if ((k & 7) == 7) asm volatile("" : "+v"(v)::"memory");
      const bool real = !GUARD || k < n_real;
      const uint32_t w = real ? weight2_of(k) : 0u;
      const uint32_t uu = real ? (k < H ? u[k] : hi[k - H][lane]) : kInf;
      const uint32_t out = umin(v, uu) | (uint32_t)((int32_t)w >> 31);
      note(k, uu, out);
      if (k < H)
        u[k] = out;
      else
        hi[k - H][lane] = out;
      v = sadd(umin(v, sadd(uu, a.ct2)), w);
    }
  }
  int xs = xp;
  asm volatile("" : "+v"(xs));
  if (active) {
#pragma unroll
    for (int k = 0; k < P; k++) {
      if ((k & 7) == 0) asm volatile("" ::: "memory");
      if ((!GUARD || k < n_real) && ((changed[k >> 5] >> (k & 31)) & 1u)) {
        buffer_store_u32(k < H ? u[k] : hi[k - H][lane], buf.V,
                         row_cell<POW2>(sh.row_base[first + k], (uint32_t)xs, POW2 ? 0u : sh.shift[first + k], N), 0,
                         0, 0);
      }
    }
  }
}

// A turn job's step geometry is the same in every tile of the job: the
// plane, column offset and row offset of step s = threadIdx.x (a workgroup of
// 64 S threads covers the S P steps, since P <= 64).  The kernels read it
// once per job, so a turn tile's set-up reads no global memory and its loads
// are issued while the previous tile's stores are still draining (a global
// read there would first wait for every earlier store).
struct TurnGeo {
  uint32_t Tn;  // plane T times N
  int shift;    // column offset of the curve through x' = 0
  int oy;       // row offset of that curve from y'
};
template <int P>
__device__ __forceinline__ TurnGeo turn_geo(const SweepJob& a) {
  TurnGeo g{0u, 0, 0};
  const int L = a.L, s = threadIdx.x;
  if (a.cyclic && s < ((L + P - 1) / P) * P) {
    const int sc = s < L ? s : L - 1;  // steps past the curve repeat the last one
    const int T = a.dir ? sc : (L - 1 - sc);
    g.Tn = (uint32_t)T * (uint32_t)a.N;
    g.shift = as_global(a.offx)[T];
    g.oy = as_global(a.offy)[T];
  }
  return g;
}

// Row-coalesced sweep of one tile (64 curves) of a job: turns (cyclic) and
// y-major straights.
//   turns:     tile -> (x tile, y'); step k -> plane T_k, offsets (ox, oy)
//   straights: tile -> (x tile, plane slot); step k -> row c_k, column x' + B(c_k)
// FUSED (turns): after the first maneuver the second one, on the same curves
// in the opposite direction, runs on the values still held in registers, so
// the pair costs one read and one write per pose.
// The workgroup has exactly one wave per section (64 S threads: the
// launchers size it so); a workgroup of another size skips the tile.
// POW2: N is a power of two.  g: the job's turn geometry (turn_geo).
template <int P, bool FUSED, bool GUARD, bool POW2>
__device__ __forceinline__ void row_sweep_tile(const SweepJob& a, int tile, RowShared& sh, const TurnGeo& g) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int N = a.N, L = a.L;
  const bool cyclic = a.cyclic != 0;
  const int S = (L + P - 1) / P;  // sections of this job
  if ((int)blockDim.x != 64 * S) return;  // uniform over the workgroup
  const int tx = tile % a.tiles_x;
  const int outer = tile / a.tiles_x;  // y' (turns) or plane slot (straights)
  const int xp = tx * 64 + lane;
  const bool active = xp < N;
  const RowBuffers buf = row_buffers(a);

  int T0 = 0;
  uint32_t Lq = a.lq;
  int dir = a.dir;
  GlobalPtr<const int16_t> sk = nullptr;
  if (!cyclic) {
    T0 = as_global(a.planes)[outer];
    Lq = as_global(a.edge_len)[T0];
    dir = (as_global(a.fwd)[T0] > 0) == (a.mu_forward != 0);
    sk = as_global(a.skew) + (size_t)T0 * N;
  }
  for (int c = threadIdx.x; c < 256; c += blockDim.x) {
    sh.wlut[c] = weight((uint32_t)c, 256u * Lq + 128u, 4u * Lq);
    if (FUSED) sh.wlut2[c] = weight((uint32_t)c, 256u * a.lq2 + 128u, 4u * a.lq2);
  }
  // Step s of a curve touches row `row` of plane T at column (x' + shift)
  // mod N: a row base shared by the 64 lanes plus a small per-lane column.
  // The geometry of all steps goes to LDS once per workgroup.
  // Steps past the curve (the last section's tail when L is not a multiple
  // of P) repeat the geometry of the last step, so loads need no clamp.
  // (one step per thread: S P <= 64 S threads)
  if (const int s = threadIdx.x; s < S * P) {
    uint32_t Tn;
    int row, shift;
    if (cyclic) {
      Tn = g.Tn;
      shift = g.shift;
      row = outer + g.oy;
      row -= (row >= N) ? N : 0;
    } else {
      Tn = (uint32_t)T0 * (uint32_t)N;
      const int sc = s < L ? s : L - 1;
      const int c = dir ? sc : (L - 1 - sc);
      shift = sk[c];
      shift += (shift < 0) ? N : 0;
      row = c;
    }
    const uint32_t rb = (Tn + (uint32_t)row) * (uint32_t)N;
    if (POW2) {
      sh.row_base[s] = rb | (uint32_t)shift;
    } else {
      sh.row_base[s] = rb;
      sh.shift[s] = (uint16_t)shift;
    }
  }
  __syncthreads();  // weight table and geometry ready

  // Sections are P steps; steps past the curve length (when S P > L) are
  // identity maps that touch no memory.
  const int n_real = (L - wave * P) < P ? (L - wave * P) : P;  // real steps of this wave
  const int first = wave * P;
  if constexpr (P >= 64) {
    scan_section_wide<P, FUSED, GUARD, POW2>(a, buf, sh, n_real, S, wave, lane, cyclic, active, xp, first, L, N);
    return;
  }
  uint32_t u[P];
  uint32_t code[P];
  {
    // Load this wave's section of the 64 curves.  Lanes past the grid edge
    // read a valid cell, so the loads carry no branch; lanes are independent
    // curves, so an idle lane's values are never stored.
    const int xl = active ? xp : N - 1;
#pragma unroll
    for (int k = 0; k < P; k++) {
      // the geometry reads take constant offsets from one address (steps past
      // the curve have a copy of the last step's geometry)
      const int s = first + k;
      const uint32_t cell = row_cell<POW2>(sh.row_base[s], (uint32_t)xl, POW2 ? 0u : sh.shift[s], N);
      u[k] = buffer_load_u32(buf.V, cell, 0, 0, 0);
      code[k] = buffer_load_u8(buf.B, cell, 0, 0, 0);
    }
  }
  scan_section<P, FUSED, GUARD, POW2, (P <= 32)>(a, buf, sh, u, code, n_real, S, wave, lane, cyclic, active, xp, first, N);
}

// x-major straights (|tan| <= 1): line x' visits (c, x' + B(c)), so lines
// that are neighbours in x' sit in different rows at every step and a lane
// per line would read a column.  A workgroup of NT / 64 waves owns 64 lines
// and walks them along c in chunks of Q columns.  Per chunk the cells owned
// by its lines form a sheared band of at most 64 + Q - 1 rows; they are read
// row by row (contiguous segments, each cell exactly once) and written to an
// LDS tile indexed by (line, column), the waves scan Q / NW columns each for
// all 64 lines (section composition in LDS, carry from the previous chunk),
// write the results back into the tile, and the band is stored row by row.
// A band cell that no line of the tile owns gets a record index past the
// end of the plane (its load reads nothing and its store is dropped) and an
// LDS slot in a spare row, so no lane branches.  The tile is double
// buffered, so a chunk's stores and the next chunk's loads need no barrier
// between them.
template <int Q, int NT, int BUFS>
struct XShared {
  static constexpr int LINES = 64;
  static constexpr int NW = NT / 64;    // waves
  static constexpr int PITCH = Q + 1;   // odd pitch: lanes reading one column of 64 lines hit 64 banks
  static constexpr int SLOTS = (LINES + 1) * PITCH;  // 64 lines and the spare row
  // codes: rows of Q bytes padded to an odd number of words, so the byte
  // reads of one column of 64 lines also fall in distinct banks
  static constexpr int PITCH_B = 4 * (Q / 4 + ((Q / 4) % 2 == 0 ? 1 : 0));
  static constexpr int SLOTS_B = (LINES + 1) * PITCH_B;
  uint32_t tV[BUFS][SLOTS];
  uint8_t tB[BUFS][SLOTS_B];
  uint32_t aggD[NW][64];
  uint32_t aggC[NW][64];
  uint32_t wlut[256];
  int16_t skew[1024];  // B(c, T) of this plane
};

template <int Q, int NT, int BUFS>
__device__ __forceinline__ void xmajor_sweep_tile(const SweepJob& a, int tile, XShared<Q, NT, BUFS>& sh) {
  using X = XShared<Q, NT, BUFS>;
  constexpr int LINES = X::LINES, PITCH = X::PITCH, PITCH_B = X::PITCH_B, NW = X::NW;
  static_assert((PITCH_B / 4) % 2 == 1 && PITCH_B % 4 == 0 && PITCH_B >= Q, "odd word pitch for the codes");
  constexpr int SUB = Q / NW;   // columns per wave
  constexpr int ROWS = NT / Q;  // band rows per load round (a column per thread)
  constexpr int ITER = (LINES + Q - 1 + ROWS - 1) / ROWS;
  static_assert(NT % Q == 0 && Q % NW == 0 && Q % 4 == 0, "Q must divide the thread count and split over the waves");
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int N = a.N;
  const uint32_t NN = (uint32_t)N * (uint32_t)N;
  const int x0 = (tile % a.tiles_x) * LINES;
  const int T = as_global(a.planes)[tile / a.tiles_x];
  // this plane's values and codes as record arrays indexed by row * N + column
  const __amdgpu_buffer_rsrc_t bV =
      __builtin_amdgcn_make_buffer_rsrc(a.V + (size_t)T * NN, (short)4, (int)NN, kBufferWord3);
  const __amdgpu_buffer_rsrc_t bB =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(a.B) + (size_t)T * NN, (short)1, (int)NN, kBufferWord3);
  const uint32_t Lq = as_global(a.edge_len)[T];
  for (int c = tid; c < 256; c += NT) sh.wlut[c] = weight((uint32_t)c, 256u * Lq + 128u, 4u * Lq);
  const int dir = (as_global(a.fwd)[T] > 0) == (a.mu_forward != 0);
  const GlobalPtr<const int16_t> skg = as_global(a.skew) + (size_t)T * N;
  for (int c = tid; c < N; c += NT) sh.skew[c] = skg[c];
  __syncthreads();
  const int16_t* sk = sh.skew;
  const int kk = tid % Q;  // column of this thread in the load/store phases
  const int r0 = tid / Q;  // first band row of this thread; rows r0 + it * ROWS
  const int t_lim = (N - x0) < LINES ? (N - x0) : LINES;  // lines of this tile inside the grid
  const uint32_t spare = LINES * PITCH + kk;               // LDS slot for cells no line owns
  const uint32_t spare_b = LINES * PITCH_B + kk;
  constexpr uint32_t kNoRecord = 0xFFFFFFFFu;

  uint32_t carry = kInf;  // value carried along line x0 + lane into the chunk
  int buf = 0;
  for (int k0 = 0; k0 < N; k0 += Q, buf = (BUFS == 2) ? (buf ^ 1) : 0) {
    uint32_t* tV = sh.tV[buf];
    uint8_t* tB = sh.tB[buf];
    const int nq = (N - k0) < Q ? (N - k0) : Q;
    const int c_first = dir ? k0 : (N - 1 - k0);
    const int c_last = dir ? (k0 + nq - 1) : (N - 1 - (k0 + nq - 1));
    const int b_first = sk[c_first], b_last = sk[c_last];
    const int bmin = b_first < b_last ? b_first : b_last;
    // grid row of band row 0, reduced mod N (|B| < N, so x0 + bmin is in (-N, 2N))
    int band0 = x0 + bmin;
    band0 += (band0 < 0) ? N : 0;
    band0 -= (band0 >= N) ? N : 0;
    const bool col_ok = kk < nq;
    const int my_c = dir ? (k0 + kk) : (N - 1 - (k0 + kk));
    const int my_b = sk[col_ok ? my_c : c_first];
    const uint32_t tl = col_ok ? (uint32_t)t_lim : 0u;
    int row = band0 + r0;
    row -= (row >= N) ? N : 0;
    const uint32_t rel0 = (uint32_t)row * (uint32_t)N + (uint32_t)(col_ok ? my_c : 0);
    const int t0 = r0 + bmin - my_b;

    // load the band: band row r holds line t = r + bmin - B(c) of column c
    uint32_t lv[ITER], lc[ITER];
    {
      uint32_t rel = rel0;
      int t = t0;
#pragma unroll
      for (int it = 0; it < ITER; it++) {
        const uint32_t idx = (uint32_t)t < tl ? rel : kNoRecord;
        lv[it] = buffer_load_u32(bV, idx, 0, 0, 0);
        lc[it] = buffer_load_u8(bB, idx, 0, 0, 0);
        t += ROWS;
        rel = wrap_col(rel + (uint32_t)(ROWS * N), (int)NN);  // ROWS rows down, wrapping around the plane
      }
    }
    {
      // the slots are recomputed rather than kept from the loads (registers)
      int t = t0;
      asm volatile("" : "+v"(t));
#pragma unroll
      for (int it = 0; it < ITER; it++) {
        const bool own = (uint32_t)t < tl;
        tV[own ? (uint32_t)(t * PITCH + kk) : spare] = lv[it];
        tB[own ? (uint32_t)(t * PITCH_B + kk) : spare_b] = (uint8_t)lc[it];
        t += ROWS;
      }
    }
    __syncthreads();

    // scan: wave w takes columns [w SUB, (w+1) SUB) of the chunk for all 64 lines
    const int line_slot = lane * PITCH + wave * SUB;
    const int line_slot_b = lane * PITCH_B + wave * SUB;
    uint32_t u[SUB], w[SUB];
#pragma unroll
    for (int q = 0; q < SUB; q++) {
      const bool ok = wave * SUB + q < nq;  // uniform
      u[q] = ok ? tV[line_slot + q] : kInf;
      w[q] = ok ? sh.wlut[tB[line_slot_b + q]] : 0u;
    }
    uint32_t D = 0, C = kInf;
#pragma unroll
    for (int q = 0; q < SUB; q++) {
      C = sadd(umin(C, sadd(u[q], a.ct)), w[q]);
      D = sadd(D, w[q]);
    }
    sh.aggD[wave][lane] = D;
    sh.aggC[wave][lane] = C;
    __syncthreads();
    uint32_t v = carry;
    for (int s = 0; s < wave; s++) v = umin(sadd(v, sh.aggD[s][lane]), sh.aggC[s][lane]);
#pragma unroll
    for (int q = 0; q < SUB; q++) {
      if (wave * SUB + q < nq) {
        tV[line_slot + q] = umin(v, u[q]) | (uint32_t)((int32_t)w[q] >> 31);
        v = sadd(umin(v, sadd(u[q], a.ct)), w[q]);
      }
    }
    for (int s = 0; s < NW; s++) carry = umin(sadd(carry, sh.aggD[s][lane]), sh.aggC[s][lane]);
    __syncthreads();

    // store the band back (cells no line owns have no record: dropped)
    {
      uint32_t rel = rel0;
      int t = t0;
      asm volatile("" : "+v"(t), "+v"(rel));
#pragma unroll
      for (int it = 0; it < ITER; it++) {
        const bool own = (uint32_t)t < tl;
        buffer_store_u32(tV[own ? (uint32_t)(t * PITCH + kk) : spare], bV, own ? rel : kNoRecord, 0, 0, 0);
        t += ROWS;
        rel = wrap_col(rel + (uint32_t)(ROWS * N), (int)NN);
      }
    }
    if (BUFS == 1) __syncthreads();  // every wave has read the tile before the next chunk writes it
  }
}

// x-major straights on grids of at least 32 cells: the same 64 lines and
// chunks of 32 columns, with the band kept in LDS in its memory layout (band
// row by band row) rather than transposed on the way in.  A thread moves 4
// adjacent columns of a band row (one 16-byte load of values, one 4-byte
// load of codes) into 4 consecutive LDS words and one code word, with no
// per-cell arithmetic; the scan reads line t's cell of column c at band row
// t + B(c) - bmin, an offset that is the same for every line of the column,
// so a column read is one address per lane plus a wave-uniform offset.
// Rows of 33 value words and 9 code words: the 64 lines of one column sit in
// consecutive band rows, which an odd pitch spreads over distinct banks.
// The stores read the band back the same way: one 16-byte store where the
// tile owns all 4 cells of a group, and one store of the owned run where it
// owns only some of them (a group of a band row can hold the last lines of
// this tile and the first of the next); band rows whose values did not change
// are not stored.  PREF: the next chunk's band is loaded into registers while
// the current one is scanned and stored, so each workgroup keeps loads in
// flight through its whole loop.

template <int Q_, int NT, int BUFS>
struct XBand {
  static constexpr int Q = Q_;                          // chunk columns
  static constexpr int NW = NT / 64;                    // waves
  static constexpr int SUB = 8;                         // columns a wave scans
  static constexpr int WPG = Q / SUB;                   // waves per group of 64 lines
  static constexpr int LINES = 64 * (NW / WPG);         // lines of a tile
  static constexpr int GW = Q / 4;                      // 4-column groups per band row
  static constexpr int ROWS = NT / GW;                  // band rows per load round
  static constexpr int BROWS = LINES + Q;               // band rows held (at least LINES + Q - 1)
  static constexpr int ITER = (BROWS + ROWS - 1) / ROWS;  // load rounds
  static constexpr int PV = Q + 1;                      // value words per band row (odd)
  static constexpr int PBW = Q / 4 + 1;                 // code words per band row (odd)
  uint32_t tV[BUFS][BROWS * PV];
  uint32_t tB[BUFS][BROWS * PBW];
  uint32_t aggD[NW][64];
  uint32_t aggC[NW][64];
  uint32_t wlut[256];
  alignas(16) int16_t skew[1024];  // B(c, T) of this plane (read 8 entries at a time)
  int16_t first_col[1024];         // first column c with |B(c) - B(0)| = i (B is monotone in unit steps)
  uint8_t dirty[2][BROWS];         // band rows holding a changed value, by chunk parity
};

// Where this thread's group of 4 columns sits in a chunk's band: record
// index of its first cell in band row r0, and the lines (relative to the
// tile) that own its outer cells in that row (one more per ROWS rows down).
struct BandGroup {
  uint32_t base;
  int lo, hi;  // smallest and largest owner: the owners of a group form a run of consecutive lines
  bool ok;     // the group lies inside the chunk's columns
};

// `chunks` counts the chunks this workgroup has swept (across tiles): its
// parity selects the band-row change flags of a chunk, which start cleared.
template <int Q_, int NT, int BUFS, bool PREF>
__device__ __forceinline__ void xmajor_band_tile(const SweepJob& a, int tile, XBand<Q_, NT, BUFS>& sh,
                                                 uint32_t& chunks) {
  using X = XBand<Q_, NT, BUFS>;
  constexpr int Q = X::Q, LINES = X::LINES, NW = X::NW, GW = X::GW, ROWS = X::ROWS, ITER = X::ITER;
  constexpr int PV = X::PV, PBW = X::PBW, BROWS = X::BROWS, SUB = X::SUB, WPG = X::WPG;
  static_assert(BUFS == 1 || BUFS == 2, "one or two band buffers");
  static_assert(NT % GW == 0 && Q % SUB == 0 && NW % WPG == 0, "groups tile the threads; columns split over the waves");
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int csec = wave % WPG;            // this wave's column section of a chunk (SUB columns)
  const int gfirst = wave - csec;         // first wave of this wave's group of 64 lines
  const int line = (wave / WPG) * 64 + lane;  // the line this lane scans (relative to the tile)
  const int N = a.N;
  const uint32_t NN = (uint32_t)N * (uint32_t)N;
  const int x0 = (tile % a.tiles_x) * LINES;
  const int T = as_global(a.planes)[tile / a.tiles_x];
  // this plane's values and codes, addressed by byte offset
  const __amdgpu_buffer_rsrc_t rV =
      __builtin_amdgcn_make_buffer_rsrc(a.V + (size_t)T * NN, (short)0, (int)(NN * 4u), kBufferWord3);
  const __amdgpu_buffer_rsrc_t rB =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(a.B) + (size_t)T * NN, (short)0, (int)NN, kBufferWord3);
  const uint32_t Lq = as_global(a.edge_len)[T];
  for (int c = tid; c < 256; c += NT) sh.wlut[c] = weight((uint32_t)c, 256u * Lq + 128u, 4u * Lq);
  const int dir = (as_global(a.fwd)[T] > 0) == (a.mu_forward != 0);
  const GlobalPtr<const int16_t> skg = as_global(a.skew) + (size_t)T * N;
  const int b0 = skg[0];
  const bool incr = skg[N - 1] >= b0;  // B ascends with the column (else descends)
  for (int c = tid; c < N; c += NT) {
    const int b = skg[c];
    sh.skew[c] = (int16_t)b;
    if (c == 0 || b != skg[c - 1]) sh.first_col[b >= b0 ? b - b0 : b0 - b] = (int16_t)c;
  }
  __syncthreads();
  const int16_t* sk = sh.skew;
  const int gw = tid % GW;  // column group of this thread in the load and store phases
  const int r0 = tid / GW;  // first band row of this thread; rows r0 + it * ROWS
  const int gs = dir ? gw : GW - 1 - gw;  // the group's place in the band row (memory order)
  const int t_lim = (N - x0) < LINES ? (N - x0) : LINES;  // lines of this tile inside the grid
  constexpr uint32_t kNoOffset = 0xFFFFFFF0u;  // past the end of either plane: loads nothing

  // chunk k0 walks memory columns k0 .. k0 + nq - 1 (dir) or N - 1 - k0
  // down to N - k0 - nq; band row 0 is grid row x0 + bmin (mod N), where
  // bmin is the smallest B over the chunk (B is monotone: at one end)
  // grid row of band row 0: x0 + bmin reduced mod N (|B| < N, x0 < N)
  auto band_row0 = [&](int bmin) {
    int row = x0 + bmin;
    row += (row < 0) ? N : 0;
    return row - (row >= N ? N : 0);
  };
  // (and brange, the difference of B between the chunk's ends)
  auto chunk_bmin = [&](int k0, int nq, int& brange) {
    const int b_first = sk[dir ? k0 : (N - 1 - k0)];
    const int b_last = sk[dir ? (k0 + nq - 1) : (N - k0 - nq)];
    brange = __builtin_amdgcn_readfirstlane(b_first < b_last ? b_last - b_first : b_first - b_last);
    return __builtin_amdgcn_readfirstlane(b_first < b_last ? b_first : b_last);
  };
  auto group_of = [&](int k0, int nq, int bmin, BandGroup& g) {
    g.ok = 4 * gw < nq;
    const int cw = g.ok ? (dir ? (k0 + 4 * gw) : (N - 4 - k0 - 4 * gw)) : 0;
    const int row = band_row0(bmin) + r0;  // r0 < ROWS <= N: at most one wrap
    g.base = (uint32_t)(row - (row >= N ? N : 0)) * (uint32_t)N + (uint32_t)cw;
    const int t_0 = r0 + bmin - sk[cw], t_3 = r0 + bmin - sk[cw + 3];  // owners of the outer cells
    g.lo = t_0 < t_3 ? t_0 : t_3;
    g.hi = t_0 < t_3 ? t_3 : t_0;
  };
  // a group some line of the tile owns in band row r0 + it ROWS is loaded;
  // the others load nothing
  auto load_band = [&](const BandGroup& g, u32x4 (&lv)[ITER], uint32_t (&lc)[ITER]) {
    uint32_t base = g.base;
#pragma unroll
    for (int it = 0; it < ITER; it++) {
      if (BROWS % ROWS != 0 && r0 + it * ROWS >= BROWS) break;  // past the rows held (uniform per wave)
      const bool any = g.ok && g.hi + it * ROWS >= 0 && g.lo + it * ROWS < t_lim;
      lv[it] = __builtin_amdgcn_raw_buffer_load_b128(rV, any ? base * 4u : kNoOffset, 0, 0);
      lc[it] = __builtin_amdgcn_raw_buffer_load_b32(rB, any ? base : kNoOffset, 0, 0);
      base = wrap_col(base + (uint32_t)(ROWS * N), (int)NN);  // ROWS rows down, wrapping around the plane
    }
  };
  auto put_band = [&](int buf, const u32x4 (&lv)[ITER], const uint32_t (&lc)[ITER]) {
    uint32_t* dv = sh.tV[buf] + r0 * PV + 4 * gs;
    uint32_t* db = sh.tB[buf] + r0 * PBW + gs;
#pragma unroll
    for (int it = 0; it < ITER; it++) {
      if (BROWS % ROWS != 0 && r0 + it * ROWS >= BROWS) break;
#pragma unroll
      for (int m = 0; m < 4; m++) dv[it * ROWS * PV + m] = lv[it][m];
      db[it * ROWS * PBW] = lc[it];
    }
  };

  u32x4 lv[ITER];
  uint32_t lc[ITER];
  BandGroup g;
  int nq = N < Q ? N : Q;
  int brange;
  int bmin = chunk_bmin(0, nq, brange);
  group_of(0, nq, bmin, g);
  if (PREF) load_band(g, lv, lc);
  uint32_t carry = kInf;  // value carried along line x0 + line into the chunk
  int buf = 0;
  for (int k0 = 0; k0 < N; k0 += Q, buf = (BUFS == 2) ? (buf ^ 1) : 0) {
    if (!PREF) load_band(g, lv, lc);
    put_band(buf, lv, lc);
    // groups the tile owns in part (the last lines of this tile and the
    // first of the next, or the reverse, in one band row): a band row's
    // owned cells run between two columns, where B(c) - bmin passes the row
    // (first line) and the row minus t_lim (past the last line), and those
    // lie inside the chunk only for the first brange rows after band row 0
    // and after band row t_lim.  One lane of the last wave per such (row,
    // edge) finds the column from the first-column table (here, so that the
    // read overlaps the scan) and, when it falls inside a group, writes that
    // group's owned cells one by one after the whole groups are stored; the
    // other waves store whole groups only.
    int pg_slot = -1;       // LDS slot of the partial group's first cell (-1: none)
    int pg_rho = 0;         // its band row
    uint32_t pg_rec = 0;    // its record index
    uint32_t pg_own = 0;    // owned cells of the group, bit m for memory column gm + m
    if (wave == NW - 1) {
      const int r = lane & 31;
      if (r < brange) {  // uniform per half-wave
        const bool last = lane >= 32;
        const int rho = last ? t_lim + r : r;
        // |B - B(0)| at the first column past the edge, in memory order
        const int v = last ? (incr ? r + 1 + bmin - b0 : b0 - (r + bmin))
                           : (incr ? rho + bmin + 1 - b0 : b0 - (rho + bmin));
        const int cb = sh.first_col[v];
        if (cb & 3) {
          const int gm = cb & ~3;  // memory column of the group
          int row = band_row0(bmin) + rho;
          while (row >= N) row -= N;  // rho < BROWS: at most BROWS / N + 1 wraps
          pg_rec = (uint32_t)row * (uint32_t)N + (uint32_t)gm;
          pg_slot = rho * PV + (gm - (dir ? k0 : (N - k0 - Q)));
          pg_rho = rho;
          // the cells before cb are owned when ownership stops there (the
          // first line's edge with B ascending, the last line's with B
          // descending), else the cells from cb on
          const uint32_t before = (1u << (cb & 3)) - 1u;
          pg_own = (last != incr) ? before : (0xFu & ~before);
        }
      }
    }
    BandGroup gn;
    int nq_n = 0, bmin_n = 0, brange_n = 0;
    if (PREF && k0 + Q < N) {
      nq_n = (N - k0 - Q) < Q ? (N - k0 - Q) : Q;
      bmin_n = chunk_bmin(k0 + Q, nq_n, brange_n);
      group_of(k0 + Q, nq_n, bmin_n, gn);
      load_band(gn, lv, lc);
    }
    __syncthreads();

    // scan: wave w takes chunk columns [w SUB, (w+1) SUB) for all 64 lines;
    // line `lane` at chunk column k is band row lane + B(c_k) - bmin.  A
    // chunk's column count is a multiple of 8 (so is N), so a wave's columns
    // are all inside the chunk or all past it (an identity section).
    const bool wok = csec * SUB < nq;  // uniform
    const uint32_t* tV = sh.tV[buf];
    const uint8_t* tB = reinterpret_cast<const uint8_t*>(sh.tB[buf]);
    // change flags: this chunk's set is clear (it was cleared during the
    // previous chunk); clear the other set for the next chunk (the previous
    // chunk's stores read it, and every wave finished them before the
    // barrier above)
    const int par = (int)(chunks & 1u);
    for (int i = tid; i < BROWS; i += NT) sh.dirty[par ^ 1][i] = 0;
    uint32_t u[SUB], w[SUB];
    int soff[SUB];  // wave-uniform part of each column's value slot
    int orow[SUB];  // band row of line 0 at each column (wave-uniform)
    if (wok) {
      // the wave's 8 columns are 8 consecutive entries of the skew table
      // (ascending when dir, else descending), 16-byte aligned: one read,
      // unpacked in scalar registers
      const int cs = dir ? (k0 + csec * SUB) : (N - SUB - k0 - csec * SUB);
      const uint4 s8 = *reinterpret_cast<const uint4*>(sk + cs);
      const uint32_t sw[4] = {(uint32_t)__builtin_amdgcn_readfirstlane((int)s8.x),
                              (uint32_t)__builtin_amdgcn_readfirstlane((int)s8.y),
                              (uint32_t)__builtin_amdgcn_readfirstlane((int)s8.z),
                              (uint32_t)__builtin_amdgcn_readfirstlane((int)s8.w)};
      int offb[SUB];
#pragma unroll
      for (int q = 0; q < SUB; q++) {
        const int k = csec * SUB + q;
        const int e = dir ? q : (SUB - 1 - q);
        const int o = (int)(int16_t)(sw[e >> 1] >> (16 * (e & 1))) - bmin;  // band row of line 0
        const int pos = dir ? k : (Q - 1 - k);                              // column in the band row
        soff[q] = o * PV + pos;
        orow[q] = o;
        offb[q] = line * (4 * PBW) + (o * (4 * PBW) + pos);
      }
      uint32_t code[SUB];
#pragma unroll
      for (int q = 0; q < SUB; q++) {
        u[q] = tV[line * PV + soff[q]];
        code[q] = tB[offb[q]];
      }
#pragma unroll
      for (int q = 0; q < SUB; q++) w[q] = sh.wlut[code[q]];
    } else {
#pragma unroll
      for (int q = 0; q < SUB; q++) {
        u[q] = kInf;
        w[q] = 0u;
        soff[q] = 0;
        orow[q] = 0;
      }
    }
    uint32_t D = 0, C = kInf;
#pragma unroll
    for (int q = 0; q < SUB; q++) {
      C = sadd(umin(C, sadd(u[q], a.ct)), w[q]);
      D = sadd(D, w[q]);
    }
    sh.aggD[wave][lane] = D;
    sh.aggC[wave][lane] = C;
    __syncthreads();
    uint32_t v = carry;
    for (int s = gfirst; s < wave; s++) v = umin(sadd(v, sh.aggD[s][lane]), sh.aggC[s][lane]);
    if (wok) {
      uint32_t* tVw = sh.tV[buf];
      int lpv = line * PV;
      asm volatile("" : "+v"(lpv));  // the slots are recomputed here rather than kept from the reads (registers)
#pragma unroll
      for (int q = 0; q < SUB; q++) {
        const uint32_t out = umin(v, u[q]) | (uint32_t)((int32_t)w[q] >> 31);
        tVw[lpv + soff[q]] = out;
        // flag the band row of a changed value (most columns change none:
        // then the wave writes no flag)
        if (__builtin_amdgcn_ballot_w64(out != u[q]) != 0ull && out != u[q]) sh.dirty[par][line + orow[q]] = 1;
        v = sadd(umin(v, sadd(u[q], a.ct)), w[q]);
      }
    }
    for (int s = gfirst; s < gfirst + WPG; s++) carry = umin(sadd(carry, sh.aggD[s][lane]), sh.aggC[s][lane]);
    __syncthreads();

    // store the band: a group the tile owns whole in one 16-byte store, then
    // the owned cells of the partly owned groups found above; a band row
    // whose values all stayed as loaded is not stored (memory holds them)
    {
      uint32_t pv[4];
      if (pg_slot >= 0 && !sh.dirty[par][pg_rho]) pg_slot = -1;
      if (pg_slot >= 0) {
#pragma unroll
        for (int m = 0; m < 4; m++) pv[m] = sh.tV[buf][pg_slot + m];
      }
      const uint32_t* sv = sh.tV[buf] + r0 * PV + 4 * gs;
      uint32_t base = g.base;
#pragma unroll
      for (int it = 0; it < ITER; it++) {
        if (BROWS % ROWS != 0 && r0 + it * ROWS >= BROWS) break;
        u32x4 val;
#pragma unroll
        for (int m = 0; m < 4; m++) val[m] = sv[it * ROWS * PV + m];
        const bool all = g.ok && g.lo + it * ROWS >= 0 && g.hi + it * ROWS < t_lim;
        if (sh.dirty[par][r0 + it * ROWS]) __builtin_amdgcn_raw_buffer_store_b128(val, rV, all ? base * 4u : kNoOffset, 0, 0);
        base = wrap_col(base + (uint32_t)(ROWS * N), (int)NN);
      }
      if (pg_slot >= 0) {
        // the owned cells are a run of 1 to 3 at one end of the group: one
        // store of the run's length (each cell a separate memory request
        // costs more than the cells' bytes)
        const int m0 = __builtin_ctz(pg_own), len = __builtin_popcount(pg_own);
        const uint32_t off = (pg_rec + (uint32_t)m0) * 4u;
        const uint32_t a0 = m0 ? pv[1] : pv[0];
        const uint32_t a1 = m0 == 0 ? pv[1] : (m0 == 1 ? pv[2] : pv[3]);
        const uint32_t a2 = m0 ? pv[3] : pv[2];
        typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
        typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));
        if (len == 1) __builtin_amdgcn_raw_buffer_store_b32(m0 == 3 ? pv[3] : (m0 == 2 ? pv[2] : a0), rV, off, 0, 0);
        if (len == 2) __builtin_amdgcn_raw_buffer_store_b64(u32x2{m0 ? pv[2] : pv[0], m0 ? pv[3] : pv[1]}, rV, off, 0, 0);
        if (len == 3) __builtin_amdgcn_raw_buffer_store_b96(u32x3{a0, a1, a2}, rV, off, 0, 0);
      }
    }
    if (BUFS == 1) __syncthreads();  // every wave has read the band before the next chunk writes it
    chunks++;
    if (PREF) {
      g = gn;
      nq = nq_n;
      bmin = bmin_n;
      brange = brange_n;
    } else if (k0 + Q < N) {
      nq = (N - k0 - Q) < Q ? (N - k0 - Q) : Q;
      bmin = chunk_bmin(k0 + Q, nq, brange);
      group_of(k0 + Q, nq, bmin, g);
    }
  }
}

// The job a block of a batched launch works on: jobs are listed in order of
// their first block, so a binary search over `first_block` finds it.
__device__ __forceinline__ int find_job(const SweepJob* __restrict__ jobs, int n_jobs, int t) {
  int lo = 0, hi = n_jobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].first_block <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Workgroups stay resident and walk the tiles (the grid is capped near the
// number that fits the chip at once): a tile's stores drain while the next
// tile's loads are issued, and no workgroup launch separates them.  The
// barrier keeps the LDS tables of the previous tile until every wave is done
// with them.
template <int P, bool FUSED, bool GUARD, bool POW2>
__global__ __launch_bounds__(1024) void row_sweep_kernel(SweepJob job) {
  __shared__ RowShared sh;
  const TurnGeo g = turn_geo<P>(job);
  for (int b = blockIdx.x; b < job.blocks; b += gridDim.x) {
    __syncthreads();
    row_sweep_tile<P, FUSED, GUARD, POW2>(job, tile_of(b, job.blocks, job.order), sh, g);
  }
}

template <int P, bool FUSED, bool GUARD, bool POW2>
__global__ __launch_bounds__(1024) void row_sweep_batch_kernel(const SweepJob* __restrict__ jobs, int n_jobs,
                                                                 int total_blocks, int order) {
  __shared__ RowShared sh;
  int jg = -1;  // job whose turn geometry g holds
  TurnGeo g{0u, 0, 0};
  for (int b = blockIdx.x; b < total_blocks; b += gridDim.x) {
    __syncthreads();
    const int t = tile_of(b, total_blocks, order);
    const int j = __builtin_amdgcn_readfirstlane(find_job(jobs, n_jobs, t));
    const SweepJob job = jobs[j];
    if (j != jg) {
      g = turn_geo<P>(job);
      jg = j;
    }
    row_sweep_tile<P, FUSED, GUARD, POW2>(job, t - job.first_block, sh, g);
  }
}

// Launch-shape knobs (nhp_set_knob; 0 = built-in choice).
std::atomic<int> g_knob[kKnobs];

int knob(int k, int builtin) {
  const int v = g_knob[k].load(std::memory_order_relaxed);
  return v ? v : builtin;
}

// Resident workgroups for a row launch: 256 CUs times the workgroups of
// `waves` waves that fit one CU (built-in: at most 16 waves per CU at these
// register counts, 32 for the small sections).
int row_grid(int blocks, int waves, int P) {
  const int builtin = (P >= 32 ? 16 : 32) / waves;
  const int per_cu = knob(NHP_KNOB_ROW_WG_PER_CU, builtin > 0 ? builtin : 1);
  const int cap = 256 * per_cu;
  return blocks < cap ? blocks : cap;
}

// x-major workgroups may walk several tiles.  A tile's stores read only the
// LDS band, and the next tile writes its band after the barrier that follows
// its weight and skew tables, so a wave still storing never sees it
// overwritten.  Grids of at least 32 cells take band tiles
// (xmajor_band_tile), smaller ones the transposed tile.  Occupancy asked of
// the register allocator: the waves per SIMD that the LDS allows.
constexpr int XBQ = 32;          // band tiles: chunk columns
constexpr int XBNT = 256;        // band tiles: workgroup threads
constexpr bool XBPREF = true;    // band tiles: load the next chunk while scanning this one
constexpr int kLdsBytes = 160 * 1024;

// Band tiles resident per CU: what the LDS allows, at most 20 waves.  More
// (the LDS allows 28 waves of 4-wave tiles with one buffer) gain no time and
// evict band rows that neighbouring tiles share from the L2 before both have
// read them: 1.15 times the algorithmic fetch at 6 or 7 tiles per CU against
// 1.04 at 5.
template <int Q, int NT, int BUFS>
constexpr int xband_wg_per_cu() {
  const int by_lds = kLdsBytes / (int)sizeof(XBand<Q, NT, BUFS>);
  const int by_waves = 20 / (NT / 64) > 0 ? 20 / (NT / 64) : 1;
  return by_lds < by_waves ? by_lds : by_waves;
}
template <int Q, int NT, int BUFS>
constexpr int xband_waves_per_simd() { return xband_wg_per_cu<Q, NT, BUFS>() * (NT / 64) / 4; }

// Band tile launches give each tile a workgroup of its own (up to 16 per CU
// in the grid, of which the occupancy above keeps 5 resident): the
// dispatcher hands the next tile to whichever CU frees a slot first, which
// evens out tiles of uneven cost better than a fixed round-robin over
// resident workgroups (2-5 % faster at 1024 sides, 0-3 % at 512).
constexpr int kXBandGridPerCU = 16;

template <int Q, int NT, int BUFS>
__global__ __launch_bounds__(NT, (xband_waves_per_simd<Q, NT, BUFS>())) void xmajor_band_kernel(SweepJob job) {
  __shared__ XBand<Q, NT, BUFS> sh;
  for (int i = threadIdx.x; i < 2 * XBand<Q, NT, BUFS>::BROWS; i += NT) sh.dirty[i & 1][i >> 1] = 0;
  uint32_t chunks = 0;  // (the tile's first barrier orders the clearing before any flag is set)
  for (int b = blockIdx.x; b < job.blocks; b += gridDim.x)
    xmajor_band_tile<Q, NT, BUFS, XBPREF>(job, tile_of(b, job.blocks, job.order), sh, chunks);
}

template <int Q, int NT, int BUFS>
__global__ __launch_bounds__(NT, (xband_waves_per_simd<Q, NT, BUFS>())) void xmajor_band_batch_kernel(
    const SweepJob* __restrict__ jobs, int n_jobs, int order) {
  __shared__ XBand<Q, NT, BUFS> sh;
  const int t = tile_of(blockIdx.x, gridDim.x, order);
  const int j = __builtin_amdgcn_readfirstlane(find_job(jobs, n_jobs, t));
  const SweepJob job = jobs[j];
  for (int i = threadIdx.x; i < 2 * XBand<Q, NT, BUFS>::BROWS; i += NT) sh.dirty[i & 1][i >> 1] = 0;
  uint32_t chunks = 0;
  xmajor_band_tile<Q, NT, BUFS, XBPREF>(job, t - job.first_block, sh, chunks);
}

// (six transposed tiles of 27 KB fit a CU)
template <int Q, int NT, int BUFS>
__global__ __launch_bounds__(NT, 6) void xmajor_sweep_kernel(SweepJob job) {
  __shared__ XShared<Q, NT, BUFS> sh;
  for (int b = blockIdx.x; b < job.blocks; b += gridDim.x)
    xmajor_sweep_tile<Q, NT, BUFS>(job, tile_of(b, job.blocks, job.order), sh);
}

template <int Q, int NT, int BUFS>
__global__ __launch_bounds__(NT, 6) void xmajor_sweep_batch_kernel(const SweepJob* __restrict__ jobs, int n_jobs,
                                                                  int order) {
  __shared__ XShared<Q, NT, BUFS> sh;
  const int t = tile_of(blockIdx.x, gridDim.x, order);
  const int j = __builtin_amdgcn_readfirstlane(find_job(jobs, n_jobs, t));
  const SweepJob job = jobs[j];
  xmajor_sweep_tile<Q, NT, BUFS>(job, t - job.first_block, sh);
}

// Resident x-major workgroups: what fits a CU at once, times 256 CUs.
int xmajor_grid(int blocks, int per_cu) {
  const int cap = 256 * knob(NHP_KNOB_XMAJOR_WG_PER_CU, per_cu);
  return blocks < cap ? blocks : cap;
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

// Batched init: job k fills V of plan k (n4[k] uint4 words, start index
// start[k]); blocks stride over all plans' words.
__global__ void init_batch_kernel(const InitJob* __restrict__ jobs, int n_jobs) {
  for (int k = 0; k < n_jobs; k++) {
    const InitJob j = jobs[k];
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < j.n4; q += stride) {
      const size_t e = q * 4;
      uint4 v = make_uint4(kInf, kInf, kInf, kInf);
      if (j.start >= e && j.start < e + 4) {
        const uint32_t o = (uint32_t)(j.start - e);
        if (o == 0) v.x = 0;
        if (o == 1) v.y = 0;
        if (o == 2) v.z = 0;
        if (o == 3) v.w = 0;
      }
      reinterpret_cast<uint4*>(j.V)[q] = v;
    }
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

// transposed x-major tiles (grids under 32 cells): chunks of 32 columns,
// 256 threads per workgroup
constexpr int XQ = 32;   // x-major chunk columns
constexpr int XNT = 256;  // x-major workgroup threads
constexpr int XBUFS_BUILTIN = 2;  // x-major tile buffers unless a knob says otherwise
constexpr int XB_BUFS_BUILTIN = 1;  // the same for band tiles

}  // namespace

// Whether the x-major kernel takes band tiles for grids of side N: a load
// round covers XBNT / (XBQ / 4) band rows, which must not exceed N (one wrap).
bool xmajor_wide(int N) { return N >= XBNT / (XBQ / 4); }

// Lines per x-major tile for grids of side N.
int xmajor_lines(int N) { return xmajor_wide(N) ? XBand<XBQ, XBNT, 1>::LINES : 64; }

namespace {

}  // namespace

// Steps per wave chosen for a curve length (0 = not set), process-wide.
static std::atomic<uint8_t> g_section_steps[1025];

int set_knob(int k, int v) {
  if (k < 0 || k >= kKnobs) return NHP_EINVAL;
  static const int lo[kKnobs] = {1, 1, 1, 1}, hi[kKnobs] = {8, 16, 2, 2};
  if (v != 0 && (v < lo[k] || v > hi[k])) return NHP_EINVAL;
  g_knob[k].store(v, std::memory_order_relaxed);
  return NHP_OK;
}

int get_knob(int k) { return (k < 0 || k >= kKnobs) ? -1 : g_knob[k].load(std::memory_order_relaxed); }

bool valid_section(int len, int P) { return (P == 8 || P == 16 || P == 32 || P == 64) && (len + P - 1) / P <= 16; }

// Steps per wave: the tuned choice for this curve length, else the smallest
// power of two in [8, 64] that splits the curve into at most 16 sections
// (16 waves of a 1024-thread workgroup).
int pick_section(int len) {
  if (len >= 1 && len <= 1024) {
    const int t = g_section_steps[len].load(std::memory_order_relaxed);
    if (t && valid_section(len, t)) return t;
  }
  int P = 8;
  while (P < 64 && P * 16 < len) P <<= 1;
  return (P * 16 >= len) ? P : 0;
}

int set_section_steps(int len, int P) {
  if (len < 1 || len > 1024) return NHP_EINVAL;
  if (P != 0 && !valid_section(len, P)) return NHP_EINVAL;
  g_section_steps[len].store((uint8_t)P, std::memory_order_relaxed);
  return NHP_OK;
}

void schedule_passes(const uint8_t* schedule, int n, uint64_t first, uint64_t count, bool pairs,
                     std::vector<Pass>& out) {
  const uint64_t end = first + count;
  for (uint64_t k = first; k < end;) {
    const int a = schedule[k % (uint64_t)n];
    if (pairs && k + 1 < end && fusable(a, schedule[(k + 1) % (uint64_t)n])) {
      out.push_back(Pass{(int8_t)a, (int8_t)schedule[(k + 1) % (uint64_t)n]});
      k += 2;
    } else {
      out.push_back(Pass{(int8_t)a, (int8_t)-1});
      k += 1;
    }
  }
}

bool can_fuse(const DevPlan& d) { return pick_section(d.nt) > 0; }

// The jobs of one pass of one plan: a row job (turns, or the y-major
// straight planes) and, for straights, an x-major job.  Returns the number of
// jobs written (0..2), blocks counts each job's workgroups; -1 for a pair
// that cannot share a pass (the caller splits it).
int make_sweep_jobs(const DevPlan& d, Pass pass, SweepJob* row, SweepJob* xmaj) {
  if (pass.mu2 >= 0 && !(fusable(pass.mu, pass.mu2) && can_fuse(d))) return -1;
  const int mu = pass.mu;
  const int N = d.nx, L = d.nt;
  const int tiles_x = (N + 63) / 64;
  SweepJob j{};
  j.V = d.V;
  j.B = d.B;
  j.N = N;
  j.n_poses = (uint32_t)N * (uint32_t)N * (uint32_t)L;
  j.ct = d.ct[mu];
  j.tiles_x = tiles_x;
  j.order = knob(NHP_KNOB_TILE_ORDER, 1);
  int n = 0;
  if (mu == NHP_SF || mu == NHP_SB) {
    j.L = N;
    j.cyclic = 0;
    j.skew = d.skew;
    j.edge_len = d.edge_len + (size_t)mu * L;
    j.fwd = d.fwd;
    j.mu_forward = (mu == NHP_SF);
    j.P = pick_section(N);
    SweepJob y = j, x = j;
    y.planes = d.planes + d.n_planes_x;
    y.blocks = tiles_x * d.n_planes_y;
    x.planes = d.planes;
    x.tiles_x = (N + xmajor_lines(N) - 1) / xmajor_lines(N);
    x.blocks = x.tiles_x * d.n_planes_x;
    x.P = 0;
    row->blocks = 0;
    xmaj->blocks = 0;
    if (y.blocks) *row = y;
    if (x.blocks) *xmaj = x;
    n = (y.blocks > 0) + (x.blocks > 0);
  } else {
    const bool left = (mu == NHP_LF || mu == NHP_LB);
    j.L = L;
    j.cyclic = 1;
    j.dir = (mu == NHP_LF || mu == NHP_RB);  // eqs. (25)-(28): LF and RB step to T+1
    j.offx = d.turn_off + (left ? 0 : 2) * L;
    j.offy = d.turn_off + (left ? 1 : 3) * L;
    j.lq = d.turn_lq[mu];
    j.P = pick_section(L);
    if (pass.mu2 >= 0) {
      j.fused = 1;
      j.ct2 = d.ct[pass.mu2];
      j.lq2 = d.turn_lq[pass.mu2];
    }
    j.blocks = tiles_x * N;
    *row = j;
    xmaj->blocks = 0;
    n = 1;
  }
  return n;
}

template <bool FUSED, bool GUARD, bool POW2>
hipError_t launch_row_job_t(const SweepJob& j, hipStream_t s) {
  const int waves = (j.L + j.P - 1) / j.P;
  const dim3 grid(row_grid(j.blocks, waves, j.P)), block(64 * waves);
  switch (j.P) {
    case 64: hipLaunchKernelGGL((row_sweep_kernel<64, FUSED, GUARD, POW2>), grid, block, 0, s, j); break;
    case 32: hipLaunchKernelGGL((row_sweep_kernel<32, FUSED, GUARD, POW2>), grid, block, 0, s, j); break;
    case 16: hipLaunchKernelGGL((row_sweep_kernel<16, FUSED, GUARD, POW2>), grid, block, 0, s, j); break;
    case 8: hipLaunchKernelGGL((row_sweep_kernel<8, FUSED, GUARD, POW2>), grid, block, 0, s, j); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

template <bool FUSED, bool GUARD>
hipError_t launch_row_job_g(const SweepJob& j, hipStream_t s) {
  return is_pow2(j.N) ? launch_row_job_t<FUSED, GUARD, true>(j, s) : launch_row_job_t<FUSED, GUARD, false>(j, s);
}

hipError_t launch_row_job(const SweepJob& j, hipStream_t s) {
  const bool guard = j.L % j.P != 0;
  if (j.fused) return guard ? launch_row_job_g<true, true>(j, s) : launch_row_job_g<true, false>(j, s);
  return guard ? launch_row_job_g<false, true>(j, s) : launch_row_job_g<false, false>(j, s);
}

hipError_t launch_init(const DevPlan& d, uint32_t start_index, hipStream_t s) {
  const size_t NR = (size_t)d.nx * d.nx * d.nt;  // a multiple of 64: nx and nt are multiples of 8
  const size_t n4 = NR / 4;
  size_t blocks = (n4 + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(init_kernel, dim3((unsigned)blocks), dim3(256), 0, s, d.V, n4, start_index);
  return hipGetLastError();
}

hipError_t launch_init_batch(const InitJob* d_jobs, int n_jobs, size_t max_n4, hipStream_t s) {
  size_t blocks = (max_n4 + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(init_batch_kernel, dim3((unsigned)blocks), dim3(256), 0, s, d_jobs, n_jobs);
  return hipGetLastError();
}

hipError_t launch_force_walls(const DevPlan& d, hipStream_t s) {
  hipLaunchKernelGGL(walls_kernel, dim3(d.nt), dim3(256), 0, s, d.B, d.nx, d.nt);
  return hipGetLastError();
}

hipError_t launch_sweep(const DevPlan& d, Pass pass, hipStream_t s) { return launch_sweep_part(d, pass, 3, s); }

hipError_t launch_sweep_part(const DevPlan& d, Pass pass, int parts, hipStream_t s) {
  SweepJob row{}, xmaj{};
  if (make_sweep_jobs(d, pass, &row, &xmaj) < 0) {
    // a pair that cannot share a pass: one pass each
    const hipError_t e = launch_sweep(d, Pass{pass.mu, (int8_t)-1}, s);
    return e != hipSuccess ? e : launch_sweep(d, Pass{pass.mu2, (int8_t)-1}, s);
  }
  if (row.blocks && (parts & 1)) {
    if (!row.P) return hipErrorInvalidValue;
    const hipError_t e = launch_row_job(row, s);
    if (e != hipSuccess) return e;
  }
  if (xmaj.blocks && (parts & 2)) {
    const bool wide = xmajor_wide(xmaj.N);
    const bool one = knob(NHP_KNOB_XMAJOR_BUFFERS, wide ? XB_BUFS_BUILTIN : XBUFS_BUILTIN) == 1;
    if (wide) {
      const dim3 block(XBNT);
      if (one)
        hipLaunchKernelGGL((xmajor_band_kernel<XBQ, XBNT, 1>),
                           dim3(xmajor_grid(xmaj.blocks, kXBandGridPerCU)), block, 0, s, xmaj);
      else
        hipLaunchKernelGGL((xmajor_band_kernel<XBQ, XBNT, 2>),
                           dim3(xmajor_grid(xmaj.blocks, kXBandGridPerCU)), block, 0, s, xmaj);
    } else {
      const dim3 grid(xmajor_grid(xmaj.blocks, 6)), block(XNT);
      if (one)
        hipLaunchKernelGGL((xmajor_sweep_kernel<XQ, XNT, 1>), grid, block, 0, s, xmaj);
      else
        hipLaunchKernelGGL((xmajor_sweep_kernel<XQ, XNT, 2>), grid, block, 0, s, xmaj);
    }
    return hipGetLastError();
  }
  return hipSuccess;
}

template <bool FUSED, bool GUARD, bool POW2>
hipError_t launch_row_batch_t(const SweepJob* d_jobs, int n_jobs, int total_blocks, int P, int waves,
                              hipStream_t s) {
  const dim3 grid(row_grid(total_blocks, waves, P)), block(64 * waves);
  switch (P) {
    case 64:
      hipLaunchKernelGGL((row_sweep_batch_kernel<64, FUSED, GUARD, POW2>), grid, block, 0, s, d_jobs, n_jobs,
                         total_blocks, knob(NHP_KNOB_TILE_ORDER, 1));
      break;
    case 32:
      hipLaunchKernelGGL((row_sweep_batch_kernel<32, FUSED, GUARD, POW2>), grid, block, 0, s, d_jobs, n_jobs,
                         total_blocks, knob(NHP_KNOB_TILE_ORDER, 1));
      break;
    case 16:
      hipLaunchKernelGGL((row_sweep_batch_kernel<16, FUSED, GUARD, POW2>), grid, block, 0, s, d_jobs, n_jobs,
                         total_blocks, knob(NHP_KNOB_TILE_ORDER, 1));
      break;
    case 8:
      hipLaunchKernelGGL((row_sweep_batch_kernel<8, FUSED, GUARD, POW2>), grid, block, 0, s, d_jobs, n_jobs,
                         total_blocks, knob(NHP_KNOB_TILE_ORDER, 1));
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <bool FUSED, bool GUARD>
hipError_t launch_row_batch_g(const SweepJob* d_jobs, int n_jobs, int total_blocks, int P, bool pow2, int waves,
                              hipStream_t s) {
  return pow2 ? launch_row_batch_t<FUSED, GUARD, true>(d_jobs, n_jobs, total_blocks, P, waves, s)
              : launch_row_batch_t<FUSED, GUARD, false>(d_jobs, n_jobs, total_blocks, P, waves, s);
}

hipError_t launch_sweep_batch(const SweepJob* d_jobs, int n_jobs, int total_blocks, int P, bool fused, bool guard,
                              bool pow2, bool xmajor, int waves, hipStream_t s) {
  if (n_jobs == 0) return hipSuccess;
  if (xmajor) {
    const int order = knob(NHP_KNOB_TILE_ORDER, 1);
    const bool one = knob(NHP_KNOB_XMAJOR_BUFFERS, pow2 ? XB_BUFS_BUILTIN : XBUFS_BUILTIN) == 1;
    const dim3 grid(total_blocks);
    // (for x-major launches `pow2` says every job's grid takes band tiles)
    if (pow2 && one)
      hipLaunchKernelGGL((xmajor_band_batch_kernel<XBQ, XBNT, 1>), grid, dim3(XBNT), 0, s, d_jobs, n_jobs, order);
    if (pow2 && !one)
      hipLaunchKernelGGL((xmajor_band_batch_kernel<XBQ, XBNT, 2>), grid, dim3(XBNT), 0, s, d_jobs, n_jobs, order);
    if (!pow2 && one)
      hipLaunchKernelGGL((xmajor_sweep_batch_kernel<XQ, XNT, 1>), grid, dim3(XNT), 0, s, d_jobs, n_jobs, order);
    if (!pow2 && !one)
      hipLaunchKernelGGL((xmajor_sweep_batch_kernel<XQ, XNT, 2>), grid, dim3(XNT), 0, s, d_jobs, n_jobs, order);
    return hipGetLastError();
  }
  if (waves < 1 || waves > 16) return hipErrorInvalidValue;
  if (fused)
    return guard ? launch_row_batch_g<true, true>(d_jobs, n_jobs, total_blocks, P, pow2, waves, s)
                 : launch_row_batch_g<true, false>(d_jobs, n_jobs, total_blocks, P, pow2, waves, s);
  return guard ? launch_row_batch_g<false, true>(d_jobs, n_jobs, total_blocks, P, pow2, waves, s)
               : launch_row_batch_g<false, false>(d_jobs, n_jobs, total_blocks, P, pow2, waves, s);
}

}  // namespace nhp
