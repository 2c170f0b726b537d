// k_render.hip -- obstacle rendering (Sec. VI) for gfx950, and soft
// obstacle costs from a distance transform of the image (Sec. VI-VII).
//
// For every heading plane T the obstacle volume is the maximum of the image
// codes under the vehicle box, taken separably: a sideways pass over the
// left-normal samples into a scratch plane, then a lengthwise pass over the
// heading samples.  The one-cell walls of Sec. V.C sit in row 0 and column 0
// of the image before dilation, and the wall poses themselves are forced
// hard afterwards.  Sample offsets come from the host (one table per plane).
// The image and a scratch plane stay L2-resident; the volume is written
// once.  The value volume's memory serves as the scratch volume.
#include "nhp_internal.h"

namespace nhp {
namespace {

// Sample offsets arrive reduced modulo N (in [0, N)), so one conditional
// subtraction wraps a row.
__device__ __forceinline__ int wrapn(int v, int N) { return v - ((v >= N) ? N : 0); }

__device__ __forceinline__ int tap_dx(int32_t p) { return (int)(p & 0xffff); }
__device__ __forceinline__ int tap_dy(int32_t p) { return (int)((uint32_t)p >> 16); }

// Both passes read rows that are padded to 2N columns (column x holds column
// x mod N), so a sample at column offset dx in [0, N) of pose column i is
// column i + dx of the padded row: no per-lane wrap.  The scratch space (the
// value volume, 4 bytes per pose) holds the padded sideways volume (2 bytes
// per pose) followed by the padded walled image (2 N^2 bytes).
__device__ __forceinline__ uint8_t* padded_image(const RenderJob& r) {
  return r.side + (size_t)2 * r.N * r.N * r.nt;
}

// A thread renders 4 consecutive poses of a row (N is a multiple of 8).  A
// sample's 4 bytes at an arbitrary column come from two aligned words
// funnelled with one byte align, and the maximum runs on the bytes as two
// pairs of 16-bit lanes (even and odd bytes), so a sample costs two word
// loads for 4 poses instead of 4 byte loads.  Sample offsets are the same
// for the whole block (one heading plane): staged in LDS, each is read into
// a scalar register.  Samples are taken 4 at a time with independent loads
// (the count is a run-time value).
typedef unsigned short ushort2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t window4(const uint8_t* row, uint32_t a) {
  const uint32_t* w = reinterpret_cast<const uint32_t*>(row + (a & ~3u));
  return __builtin_amdgcn_alignbyte(w[1], w[0], a & 3u);  // bytes a .. a + 3
}

__device__ __forceinline__ uint32_t max4_over(const uint8_t* __restrict__ src, const int32_t* tp, int n, uint32_t i0,
                                              int j, int N) {
  const uint32_t pitch = 2u * (uint32_t)N;  // a padded plane is below 2^21 bytes
  ushort2_t me = {0, 0}, mo = {0, 0};
  auto take = [&](uint32_t win) {
    me = __builtin_elementwise_max(me, __builtin_bit_cast(ushort2_t, win & 0x00FF00FFu));
    mo = __builtin_elementwise_max(mo, __builtin_bit_cast(ushort2_t, (win >> 8) & 0x00FF00FFu));
  };
  int g = 0;
  for (; g + 4 <= n; g += 4) {
    uint32_t q[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const int32_t t = __builtin_amdgcn_readfirstlane(tp[g + e]);
      q[e] = window4(src + __umul24((uint32_t)wrapn(j + tap_dy(t), N), pitch), i0 + (uint32_t)tap_dx(t));
    }
#pragma unroll
    for (int e = 0; e < 4; e++) take(q[e]);
  }
  for (; g < n; g++) {
    const int32_t t = __builtin_amdgcn_readfirstlane(tp[g]);
    take(window4(src + __umul24((uint32_t)wrapn(j + tap_dy(t), N), pitch), i0 + (uint32_t)tap_dx(t)));
  }
  return __builtin_bit_cast(uint32_t, me) | (__builtin_bit_cast(uint32_t, mo) << 8);
}

// One render job per plan; a block covers kRenderRows rows of one plane:
// block -> (plane, row group); its threads walk the rows' 4-pose groups.
constexpr int kRenderRows = 16;

__device__ __forceinline__ int find_render_job(const RenderJob* __restrict__ jobs, int n_jobs, int t) {
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

// Padded walled image, block b = row b: row 0 and column 0 (in both copies)
// are the walls of Sec. V.C.
__device__ __forceinline__ void pad_row(const RenderJob& r, int b) {
  const int N = r.N;
  uint8_t* P = padded_image(r) + (size_t)b * 2 * N;
  const uint8_t* src = r.image + (size_t)b * N;
  for (int x = threadIdx.x; x < 2 * N; x += blockDim.x) {
    const int xm = x < N ? x : x - N;
    P[x] = (b == 0 || xm == 0) ? (uint8_t)kHard : src[xm];
  }
}

// SIDE: side[T][j][i] = max over sideways samples of the walled image,
// written to both copies of the padded row.  Otherwise B[T][j][i] = max over
// lengthwise samples of side[T], walls forced hard.
template <bool SIDE>
__device__ __forceinline__ void render_rows(const RenderJob& r, int b, int32_t* tp) {
  const int N = r.N, G = N / 4;
  const int groups = (N + kRenderRows - 1) / kRenderRows;
  const int T = b / groups, j0 = (b % groups) * kRenderRows;
  const int j1 = (j0 + kRenderRows) < N ? (j0 + kRenderRows) : N;
  const size_t NN = (size_t)N * N;
  const int n = SIDE ? r.n_side : r.n_len;
  // the plane's sample offsets in LDS (global loads of them would be vector
  // loads: the stores below might alias them)
  const int32_t* tg = r.taps + (size_t)T * (r.n_side + r.n_len) + (SIDE ? 0 : r.n_side);
  for (int g = threadIdx.x; g < n; g += blockDim.x) tp[g] = tg[g];
  __syncthreads();
  const uint8_t* src = SIDE ? padded_image(r) : r.side + (size_t)T * 2 * NN;
  // the loop runs the same number of times in every lane, so the sample
  // offsets stay scalar loads (a lane past the end repeats the last group)
  const int total = (j1 - j0) * G;
  for (int base = 0; base < total; base += blockDim.x) {
    const int item = base + (int)threadIdx.x;
    const bool valid = item < total;
    const int it = valid ? item : total - 1;
    const int j = j0 + it / G;
    const uint32_t i0 = 4u * (uint32_t)(it % G);
    uint32_t m = max4_over(src, tp, n, i0, j, N);
    if (SIDE) {
      uint8_t* row = r.side + ((size_t)T * N + j) * 2 * N;
      if (valid) {
        *reinterpret_cast<uint32_t*>(row + i0) = m;
        *reinterpret_cast<uint32_t*>(row + i0 + N) = m;
      }
    } else {
      if (j == 0) m = 0xFFFFFFFFu;
      if (i0 == 0) m |= kHard;
      if (valid) *reinterpret_cast<uint32_t*>(r.B + (size_t)T * NN + (size_t)j * N + i0) = m;
    }
  }
}

__global__ __launch_bounds__(256) void pad_image_kernel(RenderJob r) { pad_row(r, blockIdx.x); }
__global__ __launch_bounds__(256) void render_side_kernel(RenderJob r) {
  __shared__ int32_t tp[kMaxTaps];
  render_rows<true>(r, blockIdx.x, tp);
}
__global__ __launch_bounds__(256) void render_len_kernel(RenderJob r) {
  __shared__ int32_t tp[kMaxTaps];
  render_rows<false>(r, blockIdx.x, tp);
}

// batched: the pad blocks of job k are N rows starting at pad_first (a
// running sum over the jobs); the pass blocks follow first_block
__global__ __launch_bounds__(256) void pad_image_batch_kernel(const RenderJob* __restrict__ jobs, int n_jobs) {
  int lo = 0, hi = n_jobs - 1, t = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].pad_first <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  pad_row(jobs[lo], t - jobs[lo].pad_first);
}

__global__ __launch_bounds__(256) void render_side_batch_kernel(const RenderJob* __restrict__ jobs, int n_jobs) {
  const int k = find_render_job(jobs, n_jobs, blockIdx.x);
  __shared__ int32_t tp[kMaxTaps];
  render_rows<true>(jobs[k], blockIdx.x - jobs[k].first_block, tp);
}

__global__ __launch_bounds__(256) void render_len_batch_kernel(const RenderJob* __restrict__ jobs, int n_jobs) {
  const int k = find_render_job(jobs, n_jobs, blockIdx.x);
  __shared__ int32_t tp[kMaxTaps];
  render_rows<false>(jobs[k], blockIdx.x - jobs[k].first_block, tp);
}

// ---- soft obstacle costs from a distance transform (Sec. VI-VII) ----
// Squared Euclidean distance to the nearest hard pixel, split the usual
// way: per column the squared distance to the nearest hard row, then per
// row the minimum over columns i' of (i - i')^2 + that column's value.

constexpr uint32_t kFar = 1u << 30;  // no hard pixel in the column

// one thread per column: two passes, down and up
__global__ __launch_bounds__(256) void soft_cols_kernel(const uint8_t* __restrict__ image, uint32_t* __restrict__ g,
                                                        int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int last = -1;  // nearest hard row above, -1 for none
  for (int j = 0; j < n; j++) {
    if (image[(size_t)j * n + i] == kHard) last = j;
    g[(size_t)j * n + i] = last < 0 ? kFar : (uint32_t)((j - last) * (j - last));
  }
  last = -1;  // nearest hard row below
  for (int j = n - 1; j >= 0; j--) {
    if (image[(size_t)j * n + i] == kHard) last = j;
    if (last >= 0) {
      const uint32_t d = (uint32_t)((last - j) * (last - j));
      const size_t x = (size_t)j * n + i;
      g[x] = d < g[x] ? d : g[x];
    }
  }
}

// one workgroup per row: the row of column values in LDS, a minimum over all
// columns per pixel, then the table
__global__ __launch_bounds__(256) void soft_rows_kernel(const uint8_t* __restrict__ image, const uint32_t* __restrict__ g,
                                                        const uint8_t* __restrict__ table, uint32_t len,
                                                        uint8_t* __restrict__ out, int n) {
  __shared__ uint32_t row[1024];
  const int j = blockIdx.x;
  for (int i = threadIdx.x; i < n; i += blockDim.x) row[i] = g[(size_t)j * n + i];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const size_t x = (size_t)j * n + i;
    if (image[x] == kHard) {
      out[x] = (uint8_t)kHard;
      continue;
    }
    uint32_t best = 0xFFFFFFFFu;
    for (int ii = 0; ii < n; ii++) {
      const uint32_t d = (uint32_t)((i - ii) * (i - ii)) + row[ii];
      best = d < best ? d : best;
    }
    out[x] = table[best < len - 1 ? best : len - 1];
  }
}

}  // namespace

hipError_t launch_soft_costs(const uint8_t* image, uint32_t* g_scratch, const uint8_t* table, uint32_t len,
                             uint8_t* out, int n, hipStream_t s) {
  hipLaunchKernelGGL(soft_cols_kernel, dim3((n + 255) / 256), dim3(256), 0, s, image, g_scratch, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(soft_rows_kernel, dim3(n), dim3(256), 0, s, image, g_scratch, table, len, out, n);
  return hipGetLastError();
}

int render_blocks(int N, int nt) { return ((N + kRenderRows - 1) / kRenderRows) * nt; }

hipError_t launch_render(const DevPlan& d, const uint8_t* image, int n_side, int n_len, hipStream_t s) {
  RenderJob r{};
  r.image = image;
  r.side = reinterpret_cast<uint8_t*>(d.V);  // N_R bytes of the 4 N_R-byte value volume
  r.B = d.B;
  r.taps = d.taps;
  r.N = d.nx;
  r.nt = d.nt;
  r.n_side = n_side;
  r.n_len = n_len;
  r.blocks = render_blocks(d.nx, d.nt);
  hipLaunchKernelGGL(pad_image_kernel, dim3(d.nx), dim3(256), 0, s, r);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(render_side_kernel, dim3(r.blocks), dim3(256), 0, s, r);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(render_len_kernel, dim3(r.blocks), dim3(256), 0, s, r);
  return hipGetLastError();
}

hipError_t launch_render_batch(const RenderJob* d_jobs, int n_jobs, int total_blocks, int total_pad_rows,
                               hipStream_t s) {
  if (n_jobs == 0) return hipSuccess;
  hipLaunchKernelGGL(pad_image_batch_kernel, dim3(total_pad_rows), dim3(256), 0, s, d_jobs, n_jobs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(render_side_batch_kernel, dim3(total_blocks), dim3(256), 0, s, d_jobs, n_jobs);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(render_len_batch_kernel, dim3(total_blocks), dim3(256), 0, s, d_jobs, n_jobs);
  return hipGetLastError();
}

}  // namespace nhp
