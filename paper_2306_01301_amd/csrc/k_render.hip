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

// Sample offsets are the same for the whole block (one heading plane): each
// is read once into a scalar register, and the row of a sample (a uniform
// value) is formed in scalar arithmetic.  Samples are taken 8 at a time with
// independent loads (the count is a run-time value).
__device__ __forceinline__ uint32_t max_over(const uint8_t* __restrict__ src, const int32_t* __restrict__ tp, int n,
                                             uint32_t i, int j, int N) {
  const uint32_t pitch = 2u * (uint32_t)N;  // a padded plane is below 2^21 bytes
  uint32_t m = 0;
  int g = 0;
  for (; g + 8 <= n; g += 8) {
    uint32_t q[8];
#pragma unroll
    for (int e = 0; e < 8; e++) {
      const int32_t t = __builtin_amdgcn_readfirstlane(tp[g + e]);
      const uint8_t* row = src + ((uint32_t)wrapn(j + tap_dy(t), N) * pitch + (uint32_t)tap_dx(t));
      q[e] = row[i];
    }
#pragma unroll
    for (int e = 0; e < 8; e++) m = q[e] > m ? q[e] : m;
  }
  for (; g < n; g++) {
    const int32_t t = __builtin_amdgcn_readfirstlane(tp[g]);
    const uint8_t* row = src + ((uint32_t)wrapn(j + tap_dy(t), N) * pitch + (uint32_t)tap_dx(t));
    const uint32_t q = row[i];
    m = q > m ? q : m;
  }
  return m;
}

// One render job per plan; a block covers 256 columns of kRenderRows rows of
// one plane: block -> (plane, row group, column tile).  The plane's sample
// offsets stay in scalar registers over the rows.
constexpr int kRenderRows = 16;
__device__ __forceinline__ void render_pose(const RenderJob& r, int b, int& T, int& j0, int& i) {
  const int tiles = (r.N + 255) >> 8;
  const int groups = (r.N + kRenderRows - 1) / kRenderRows;
  i = (b % tiles) * 256 + threadIdx.x;
  j0 = ((b / tiles) % groups) * kRenderRows;
  T = b / (tiles * groups);
}

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

// side[T][j][i] = max over sideways samples of the walled image, written to
// both copies of the padded row
__device__ __forceinline__ void side_pose(const RenderJob& r, int b) {
  int T, j0, i;
  render_pose(r, b, T, j0, i);
  if (i >= r.N) return;
  const int j1 = (j0 + kRenderRows) < r.N ? (j0 + kRenderRows) : r.N;
  for (int j = j0; j < j1; j++) {
    const uint32_t m = max_over(padded_image(r), r.taps + (size_t)T * 2 * kMaxTaps, r.n_side, (uint32_t)i, j, r.N);
    uint8_t* row = r.side + ((size_t)T * r.N + j) * 2 * r.N;
    row[i] = (uint8_t)m;
    row[i + r.N] = (uint8_t)m;
  }
}

// B[T][j][i] = max over lengthwise samples of side[T]; walls forced hard
__device__ __forceinline__ void len_pose(const RenderJob& r, int b) {
  int T, j0, i;
  render_pose(r, b, T, j0, i);
  if (i >= r.N) return;
  const size_t NN = (size_t)r.N * r.N;
  const int j1 = (j0 + kRenderRows) < r.N ? (j0 + kRenderRows) : r.N;
  for (int j = j0; j < j1; j++) {
    uint32_t m = max_over(r.side + (size_t)T * 2 * NN, r.taps + (size_t)T * 2 * kMaxTaps + kMaxTaps, r.n_len,
                          (uint32_t)i, j, r.N);
    if (i == 0 || j == 0) m = kHard;
    r.B[(size_t)T * NN + (size_t)j * r.N + i] = (uint8_t)m;
  }
}

__global__ __launch_bounds__(256) void pad_image_kernel(RenderJob r) { pad_row(r, blockIdx.x); }
__global__ __launch_bounds__(256) void render_side_kernel(RenderJob r) { side_pose(r, blockIdx.x); }
__global__ __launch_bounds__(256) void render_len_kernel(RenderJob r) { len_pose(r, blockIdx.x); }

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
  side_pose(jobs[k], blockIdx.x - jobs[k].first_block);
}

__global__ __launch_bounds__(256) void render_len_batch_kernel(const RenderJob* __restrict__ jobs, int n_jobs) {
  const int k = find_render_job(jobs, n_jobs, blockIdx.x);
  len_pose(jobs[k], blockIdx.x - jobs[k].first_block);
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

int render_blocks(int N, int nt) { return ((N + 255) / 256) * ((N + kRenderRows - 1) / kRenderRows) * nt; }

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
