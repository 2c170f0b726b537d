// nhp_internal.h -- private declarations of the HIP planner library.
// Shared only by the library's own translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

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
  std::vector<int32_t> beta, psi, family, fwd, skew;  // skew: [T][y']
  std::vector<uint32_t> edge_len;                     // [mu][T], Q10, gear applied
  // derived device layouts
  std::vector<int32_t> turn_off;  // [4][T]: LEFT x, LEFT y, RIGHT x, RIGHT y, reduced mod nx
  std::vector<int16_t> skew16;    // [T][y'] signed B(y', T)
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
  int32_t* taps;         // [nt][2 * kMaxTaps] packed (dx & 0xffff) | (dy << 16): side then length
  uint32_t* extract;     // result header + steps
  uint32_t ct[6];
  uint32_t turn_lq[6];   // host copy of the (plane-independent) turn edge lengths
  uint8_t schedule[6];
  int n_schedule;
};

// extract buffer layout (uint32 words)
constexpr int kExHeader = 16;  // status, n_steps, best i, j, T, V(best), score, ...
constexpr int kExStepWords = 9;

hipError_t launch_init(const DevPlan& d, uint32_t start_index, hipStream_t s);
hipError_t launch_force_walls(const DevPlan& d, hipStream_t s);
hipError_t launch_sweep(const DevPlan& d, int mu, hipStream_t s);
hipError_t launch_render(const DevPlan& d, const uint8_t* image, int n_side, int n_len, hipStream_t s);
hipError_t launch_extract(const DevPlan& d, uint32_t si, uint32_t sj, uint32_t st, uint32_t gi, uint32_t gj,
                          uint32_t gt, int radius, uint32_t w_xy, uint32_t w_t, hipStream_t s);

}  // namespace nhp
