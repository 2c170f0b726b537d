// nhp_tables.cpp -- host construction of the planner's integer tables,
// Sec. V.C-D of the paper (eqs. 11-31), and of the rendering sample offsets
// (Sec. VI).  Built once per plan in double precision and rounded; the device
// only ever sees integers.
//
// Rounding rules (the paper leaves them open; every one is symmetric so the
// tables are exactly periodic and mirror-symmetric):
//   * trigonometry is evaluated on the first quadrant only and extended by
//     sin(pi - x) = sin(x), sin(x + pi) = -sin(x), cos(x) = sin(x + pi/2);
//   * round() is round-half-away-from-zero everywhere;
//   * the straight family is decided on the integer heading (45 degrees is
//     x-major in all four diagonal directions).
#include <math.h>

#include <map>
#include <mutex>

#include "nhp_internal.h"

namespace nhp {

namespace {

constexpr double kPi = 3.14159265358979323846;

double first_quadrant_sin(int nt, int m) {
  if (m == 0) return 0.0;
  if (4 * m == nt) return 1.0;
  return sin(2.0 * kPi * (double)m / (double)nt);
}

int mod(long a, int n) {
  long r = a % n;
  return (int)(r < 0 ? r + n : r);
}

// eq. (19): plane T is x-major (|tan| <= 1) within 45 degrees of 0 or 180
bool x_major_plane(int L, int T) {
  const int half = mod(T, L / 2);
  return 8 * half <= L || 8 * half >= 3 * L;
}

// round-half-away-from-zero of |v| < 2^31, the value lround gives, without
// the library call: the integer part is truncated and the fraction, which
// the subtraction gives exactly, decides the rounding.
int32_t round_half_away(double v) {
  const double a = fabs(v);
  const long i = (long)a;
  const long k = i + ((a - (double)i) >= 0.5 ? 1 : 0);
  return (int32_t)(v < 0 ? -k : k);
}

}  // namespace

// sin(2 pi T / nt) from the first-quadrant table.
double grid_sin(int nt, long T) {
  const int q = nt / 4;
  const int t = mod(T, nt);
  const int r = t % q;
  switch (t / q) {
    case 0: return first_quadrant_sin(nt, r);
    case 1: return first_quadrant_sin(nt, q - r);
    case 2: return -first_quadrant_sin(nt, r);
    default: return -first_quadrant_sin(nt, q - r);
  }
}

double grid_cos(int nt, long T) { return grid_sin(nt, T + nt / 4); }

namespace {

// Skew table of eq. (22) for all planes of one shape: B(y', T) =
// round(y' K_T) with K_T the plane's slope of eq. (20), in the plane's own
// family.  A process-wide cache keyed by (nx, ntheta) builds each shape once
// (a batch of plans mostly repeats a few shapes); past kMaxShapes entries
// (at most 2 MB each) the cache starts over (plans keep their tables alive
// by reference).
std::shared_ptr<const std::vector<int16_t>> skew_table(int N, int L) {
  constexpr size_t kMaxShapes = 16;
  static std::mutex mu;
  static std::map<std::pair<int, int>, std::shared_ptr<const std::vector<int16_t>>> cache;
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find({N, L});
    if (it != cache.end()) return it->second;
  }
  auto table = std::make_shared<std::vector<int16_t>>((size_t)L * N);
  for (int T = 0; T < L; T++) {
    const double s = grid_sin(L, T), c = grid_cos(L, T);
    const double K = x_major_plane(L, T) ? s / c : c / s;
    int16_t* row = table->data() + (size_t)T * N;
    for (int y = 0; y < N; y++) row[y] = (int16_t)round_half_away((double)y * K);
  }
  std::lock_guard<std::mutex> lock(mu);
  if (cache.size() >= kMaxShapes) cache.clear();
  cache[{N, L}] = table;
  return table;
}

}  // namespace

int build_tables(const nhp_params& p, HostTables& t) {
  const int N = (int)p.nx, L = (int)p.ntheta, q = L / 4;
  t.beta.assign(L, 0);
  t.psi.assign(L, 0);
  t.family.assign(L, 0);
  t.fwd.assign(L, 0);
  t.edge_len.assign(6 * (size_t)L, 0);
  t.planes_x.clear();
  t.planes_y.clear();

  const double turn_len = 2.0 * kPi * p.turn_radius / (double)L;  // arc of one plane step
  for (int T = 0; T < L; T++) {
    const double s = grid_sin(L, T), c = grid_cos(L, T);
    // eqs. (12)-(13): zeta(x) = round(2x)/2, beta = floor(zeta(R sin)), Psi = zeta - beta
    const double alpha = p.turn_radius * s;
    if (p.half_cell) {
      const long two_zeta = lround(2.0 * alpha);
      const long odd = two_zeta & 1L;
      t.beta[T] = (int32_t)((two_zeta - odd) / 2);
      t.psi[T] = (int32_t)odd;
    } else {
      t.beta[T] = (int32_t)lround(alpha);
      t.psi[T] = 0;
    }
    t.family[T] = x_major_plane(L, T) ? 0 : 1;
    (t.family[T] == 0 ? t.planes_x : t.planes_y).push_back(T);
    // eq. (24) forward sign (the skew of eqs. (20)-(22) is built per shape below)
    t.fwd[T] = t.family[T] == 0 ? (c > 0 ? 1 : -1) : (s > 0 ? 1 : -1);
    // Sec. V.D: straight edges are 1 / max(|cos|, |sin|) long
    const double straight_len = 1.0 / fmax(fabs(c), fabs(s));
    for (int mu = 0; mu < 6; mu++) {
      const double len = (mu == NHP_SF || mu == NHP_SB) ? straight_len : turn_len;
      const long long lq = llround(4.0 * (double)p.gear_q8[mu] * len);  // 1024 * gear / 256
      // every edge must cost at least 1/1024 cell (back-tracking relies on
      // strictly decreasing values) and Lq * 1276 + 128 must fit 32 bits
      if (lq < 1 || (unsigned long long)lq > kMaxLq) return NHP_EINVAL;
      t.edge_len[(size_t)mu * L + T] = (uint32_t)lq;
    }
  }
  // eq. (17)-(18): LEFT curves at (x' + beta_0, y' + beta_3), RIGHT at
  // (x' + beta_2, y' + beta_1), beta_k(T) = beta(T + k N_theta / 4).
  t.turn_off.assign(4 * (size_t)L, 0);
  for (int T = 0; T < L; T++) {
    t.turn_off[0 * L + T] = mod(t.beta[(T + 0 * q) % L], N);
    t.turn_off[1 * L + T] = mod(t.beta[(T + 3 * q) % L], N);
    t.turn_off[2 * L + T] = mod(t.beta[(T + 2 * q) % L], N);
    t.turn_off[3 * L + T] = mod(t.beta[(T + 1 * q) % L], N);
  }
  t.skew16 = skew_table(N, L);
  return NHP_OK;
}

// Footprint sample offsets of plane T, each reduced modulo nx and packed
// dx | (dy << 16).
// Sideways: g = -half_width..half_width along the left normal (-sin, cos),
// from the represented point of eq. (16); lengthwise: g = -rear..front along
// the heading (cos, sin).
void render_taps_host(const nhp_params& p, const HostTables& t, int T, int front, int rear, int half_width,
                      int32_t* side_packed, int32_t* len_packed) {
  const int L = (int)p.ntheta;
  const double sn = grid_sin(L, T), cs = grid_cos(L, T);
  const double hx = p.half_cell ? 0.5 * (double)t.psi[T] : 0.0;
  const double hy = p.half_cell ? 0.5 * (double)t.psi[(T + L / 4) % L] : 0.0;
  int n = 0;
  for (int g = -half_width; g <= half_width; g++, n++) {
    const int dx = mod(lround((double)g * -sn + hx), (int)p.nx);
    const int dy = mod(lround((double)g * cs + hy), (int)p.nx);
    side_packed[n] = (int32_t)((uint32_t)dx | ((uint32_t)dy << 16));
  }
  n = 0;
  for (int g = -rear; g <= front; g++, n++) {
    const int dx = mod(lround((double)g * cs), (int)p.nx);
    const int dy = mod(lround((double)g * sn), (int)p.nx);
    len_packed[n] = (int32_t)((uint32_t)dx | ((uint32_t)dy << 16));
  }
}

}  // namespace nhp
