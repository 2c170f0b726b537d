// k_render.hip -- obstacle rendering (Sec. VI) for gfx950.
//
// For every heading plane T the obstacle volume is the maximum of the image
// codes under the vehicle box, taken separably: a sideways pass over the
// left-normal samples into a scratch plane, then a lengthwise pass over the
// heading samples.  The one-cell walls of Sec. V.C sit in row 0 and column 0
// of the image before dilation, and the wall poses themselves are forced
// hard afterwards.  Sample offsets come from the host (one table per plane).
// The image (N^2 bytes) and a scratch plane stay L2-resident; the volume is
// written once.  The value volume's memory serves as the scratch volume.
#include "nhp_internal.h"

namespace nhp {
namespace {

// Sample offsets arrive reduced modulo N (in [0, N)), so one conditional
// subtraction wraps a coordinate.
__device__ __forceinline__ int wrapn(int v, int N) { return v - ((v >= N) ? N : 0); }

__device__ __forceinline__ int tap_dx(int32_t p) { return (int)(p & 0xffff); }
__device__ __forceinline__ int tap_dy(int32_t p) { return (int)((uint32_t)p >> 16); }

// Samples of a pass are read 4 at a time with independent loads (the tap
// count is a run-time value, so a plain loop would serialise them).
template <bool WALLED>
__device__ __forceinline__ uint32_t max_over(const uint8_t* __restrict__ src, const int32_t* __restrict__ tp, int n,
                                             int i, int j, int N) {
  uint32_t m = 0;
  int g = 0;
  for (; g + 4 <= n; g += 4) {
    uint32_t q[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const int32_t t = tp[g + e];
      const int y = wrapn(j + tap_dy(t), N), x = wrapn(i + tap_dx(t), N);
      q[e] = src[(size_t)y * N + x];
      if (WALLED) q[e] = (y == 0 || x == 0) ? kHard : q[e];
    }
#pragma unroll
    for (int e = 0; e < 4; e++) m = q[e] > m ? q[e] : m;
  }
  for (; g < n; g++) {
    const int32_t t = tp[g];
    const int y = wrapn(j + tap_dy(t), N), x = wrapn(i + tap_dx(t), N);
    uint32_t q = src[(size_t)y * N + x];
    if (WALLED) q = (y == 0 || x == 0) ? kHard : q;
    m = q > m ? q : m;
  }
  return m;
}

// side[T][j][i] = max over sideways samples of the walled image
__global__ __launch_bounds__(256) void render_side_kernel(const uint8_t* __restrict__ image, uint8_t* __restrict__ side,
                                                          const int32_t* __restrict__ taps, int N, int n_side) {
  const int T = blockIdx.z;
  const int j = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const uint32_t m = max_over<true>(image, taps + (size_t)T * 2 * kMaxTaps, n_side, i, j, N);
  side[((size_t)T * N + j) * N + i] = (uint8_t)m;
}

// B[T][j][i] = max over lengthwise samples of side[T]; walls forced hard
__global__ __launch_bounds__(256) void render_len_kernel(const uint8_t* __restrict__ side, uint8_t* __restrict__ B,
                                                         const int32_t* __restrict__ taps, int N, int n_side,
                                                         int n_len) {
  const int T = blockIdx.z;
  const int j = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  uint32_t m = max_over<false>(side + (size_t)T * N * N, taps + (size_t)T * 2 * kMaxTaps + kMaxTaps, n_len, i, j, N);
  if (i == 0 || j == 0) m = kHard;
  B[((size_t)T * N + j) * N + i] = (uint8_t)m;
}

}  // namespace

hipError_t launch_render(const DevPlan& d, const uint8_t* image, int n_side, int n_len, hipStream_t s) {
  const int N = d.nx;
  const dim3 block(256);
  const dim3 grid((N + 255) / 256, N, d.nt);
  uint8_t* side = reinterpret_cast<uint8_t*>(d.V);  // N_R bytes of the 4 N_R-byte value volume
  hipLaunchKernelGGL(render_side_kernel, grid, block, 0, s, image, side, d.taps, N, n_side);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(render_len_kernel, grid, block, 0, s, side, d.B, d.taps, N, n_side, n_len);
  return hipGetLastError();
}

}  // namespace nhp
