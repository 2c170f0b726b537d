/*
 * nhp_oracle.c -- plain CPU reference of the kernel-style N-turn planner of
 * Nister, Soundararajan, Wang, Sane, "Nonholonomic Motion Planning as
 * Efficient as Piano Mover's" (arXiv 2306.01301).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this code; the product path never
 * does.  It shares no source, header, table builder or helper with the HIP
 * library: both were written separately from the paper.
 *
 * What it computes, step by step, in the paper's order:
 *   tables     Sec. V.C-D, eqs. (11)-(31): turn offsets beta, half-cell
 *              residual Psi, straight family I, skew K, rounded skew B(y',T),
 *              forward sign J, edge lengths.
 *   render     Sec. VI and Sec. V.C (walls at i=0, j=0): per heading plane a
 *              separable max-dilation of the obstacle image by the vehicle
 *              box, sideways pass then lengthwise pass.
 *   init       Sec. XI step 5 preamble: V = infinity, V(start) = 0.
 *   sweep      Sec. VIII.B: one maneuver kernel, every curve of the
 *              maneuver walked vertex by vertex with the Star-graph
 *              relaxation of Sec. V.A; turns walk two full loops (they are
 *              cyclic), straights one.
 *   cycles     Sec. XVI.A: N cycles of LF, SF, RB, RF, SB, LB.
 *   goal       Sec. IX: best vertex in a window around the goal.
 *   backtrack  Sec. X, eq. (32): reverse Bellman steps back to the start.
 *   soft costs Sec. VI-VII: obstacle codes from the distance to the nearest
 *              hard pixel (a squared-distance table).
 *   sets       Sec. III.A, IX, XII: start sets with costs (also inside a
 *              maneuver in progress) and goal sets with penalties.
 *   reach      App. C, Insert 2: reachability by maneuver count (hard
 *              obstacles only), its goal search and back-tracking.
 *
 * Integer reading of the paper's floating-point costs (the paper is silent on
 * a fixed-point form): values are uint32 in 1/1024 cell, 0xFFFFFFFF is
 * infinity and every addition saturates there.  Obstacle volume cells hold a
 * code kappa in 0..254 (soft; slowness (256 + 4 kappa)/256, i.e. the
 * reciprocal of the highest allowed velocity of Sec. VI) or 255 (hard).
 * The weight of an edge is taken at its source vertex (Sec. VI: the obstacle
 * value multiplies the length of each edge leaving the vertex).
 *
 * Memory layout of every volume: index ((T * N) + j) * N + i, i fastest.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_INF 0xFFFFFFFFu
#define OR_HARD 255
#define OR_PI 3.14159265358979323846

enum { OR_LF = 0, OR_SF = 1, OR_RB = 2, OR_RF = 3, OR_SB = 4, OR_LB = 5 };

enum {
  OR_OK = 0,
  OR_EINVAL = -1,
  OR_ENOMEM = -2,
  OR_ESTART = -4,
  OR_EUNREACH = -5,
  OR_ECAP = -6
};

/* Problem description; mirrored field by field by the Python wrapper. */
typedef struct {
  int32_t nx;        /* N_x = N_y, number of spatial cells per side */
  int32_t nt;        /* N_theta, number of heading planes */
  double R;          /* minimum turn radius in cells */
  int32_t half_cell; /* 1: half-cell representation, eqs. (13)-(16) */
  int32_t nsched;    /* maneuvers per cycle */
  int32_t sched[6];  /* maneuver order within one cycle */
  uint32_t ct[6];    /* transition cost of each maneuver, 1/1024 cell */
  uint32_t gear[6];  /* edge-length multiplier of each maneuver, 1/256 */
} or_problem;

typedef struct {
  uint8_t maneuver;
  uint8_t pad[3];
  uint32_t steps;
  uint32_t from[3]; /* i, j, T */
  uint32_t to[3];
  uint32_t cost; /* transition cost plus the edge sum of this maneuver */
} or_step;

/* ------------------------------------------------------------------ */
/* small arithmetic helpers                                           */
/* ------------------------------------------------------------------ */

static uint32_t sat_add(uint32_t a, uint32_t b) {
  uint64_t s = (uint64_t)a + (uint64_t)b;
  return s >= OR_INF ? OR_INF : (uint32_t)s;
}

static uint32_t umin(uint32_t a, uint32_t b) { return a < b ? a : b; }

static int32_t wrap(int64_t a, int32_t n) {
  int64_t r = a % n;
  return (int32_t)(r < 0 ? r + n : r);
}

static size_t cell_index(const or_problem* p, int32_t i, int32_t j, int32_t T) {
  return ((size_t)T * (size_t)p->nx + (size_t)j) * (size_t)p->nx + (size_t)i;
}

/* ------------------------------------------------------------------ */
/* trigonometry on the heading grid                                   */
/* ------------------------------------------------------------------ */

/* sin(2 pi m / nt) for 0 <= m <= nt/4, with the quadrant end points exact. */
static double quadrant_sin(int32_t nt, int32_t m) {
  if (m == 0) return 0.0;
  if (4 * m == nt) return 1.0;
  return sin(2.0 * OR_PI * (double)m / (double)nt);
}

/* sin(theta(T)), theta(T) = 2 pi T / N_theta (Sec. V.C).  Only the first
 * quadrant is evaluated; the other three follow by the exact symmetries
 * sin(pi - x) = sin(x) and sin(x + pi) = -sin(x), so the table is exactly
 * periodic and exactly mirror-symmetric. */
static double grid_sin(int32_t nt, int64_t T) {
  int32_t q = nt / 4;
  int32_t t = wrap(T, nt);
  int32_t quad = t / q, r = t % q;
  switch (quad) {
    case 0: return quadrant_sin(nt, r);
    case 1: return quadrant_sin(nt, q - r);
    case 2: return -quadrant_sin(nt, r);
    default: return -quadrant_sin(nt, q - r);
  }
}

static double grid_cos(int32_t nt, int64_t T) { return grid_sin(nt, T + nt / 4); }

/* ------------------------------------------------------------------ */
/* tables, eqs. (11)-(31)                                              */
/* ------------------------------------------------------------------ */

typedef struct {
  int32_t* beta;  /* beta(T), eq. (12)-(13), T in [0, nt) */
  int32_t* psi;   /* Psi(T) in half cells (0 or 1), eq. (13) */
  int32_t* I;     /* straight family, eq. (19): 0 when |tan| <= 1 */
  int32_t* J;     /* forward sign, eq. (24) */
  int32_t* Bsk;   /* B(y', T) = round(y' K(T)), eq. (22); [T][y'] */
  uint32_t* Lq;   /* edge length of maneuver mu in plane T, 1/1024 cell; [mu][T] */
} or_tables;

static int32_t straight_family(int32_t nt, int32_t T) {
  /* |tan theta| <= 1 exactly when theta is within pi/4 of 0 or pi.  Decided
   * on the integer heading so that 45 degrees counts as |tan| = 1 in all four
   * diagonal directions. */
  int32_t t = wrap(T, nt / 2);
  return (8 * t <= nt || 8 * t >= 3 * nt) ? 0 : 1;
}

static int tables_build(const or_problem* p, or_tables* tb) {
  int32_t N = p->nx, L = p->nt;
  tb->beta = (int32_t*)malloc(sizeof(int32_t) * L);
  tb->psi = (int32_t*)malloc(sizeof(int32_t) * L);
  tb->I = (int32_t*)malloc(sizeof(int32_t) * L);
  tb->J = (int32_t*)malloc(sizeof(int32_t) * L);
  tb->Bsk = (int32_t*)malloc(sizeof(int32_t) * (size_t)L * N);
  tb->Lq = (uint32_t*)malloc(sizeof(uint32_t) * 6 * (size_t)L);
  if (!tb->beta || !tb->psi || !tb->I || !tb->J || !tb->Bsk || !tb->Lq) return OR_ENOMEM;

  for (int32_t T = 0; T < L; T++) {
    /* alpha(T) = R sin(theta(T)); zeta(x) = round(2x)/2 rounds to the nearest
     * integer or half integer (eq. 12-13).  beta = floor(zeta(alpha)) and
     * Psi = zeta(alpha) - beta, kept here in half cells. */
    double alpha = p->R * grid_sin(L, T);
    if (p->half_cell) {
      long twice = lround(2.0 * alpha); /* 2 zeta(alpha), an integer */
      long fl = (twice - (twice & 1L)) / 2; /* floor(twice / 2) */
      tb->beta[T] = (int32_t)fl;
      tb->psi[T] = (int32_t)(twice & 1L);
    } else {
      /* the plain alternative mentioned after eq. (16): usual rounding, Psi = 0 */
      tb->beta[T] = (int32_t)lround(alpha);
      tb->psi[T] = 0;
    }

    double s = grid_sin(L, T), c = grid_cos(L, T);
    tb->I[T] = straight_family(L, T);
    /* eq. (20): K = tan for the x-major family, cot for the y-major one */
    double K = tb->I[T] == 0 ? s / c : c / s;
    /* eq. (24): forward sign of the sweep coordinate */
    tb->J[T] = tb->I[T] == 0 ? (c > 0 ? 1 : -1) : (s > 0 ? 1 : -1);
    for (int32_t y = 0; y < N; y++) tb->Bsk[(size_t)T * N + y] = (int32_t)lround((double)y * K);

    /* Sec. V.D: a turn edge covers 2 pi R / N_theta, a straight edge
     * 1 / |cos| (x-major) or 1 / |sin| (y-major), i.e. 1 / max(|cos|, |sin|). */
    double turn_len = 2.0 * OR_PI * p->R / (double)L;
    double straight_len = 1.0 / fmax(fabs(c), fabs(s));
    for (int mu = 0; mu < 6; mu++) {
      double len = (mu == OR_SF || mu == OR_SB) ? straight_len : turn_len;
      /* 1024 (Q10) times gear/256 */
      tb->Lq[(size_t)mu * L + T] = (uint32_t)llround(4.0 * (double)p->gear[mu] * len);
    }
  }
  return OR_OK;
}

static void tables_free(or_tables* tb) {
  free(tb->beta);
  free(tb->psi);
  free(tb->I);
  free(tb->J);
  free(tb->Bsk);
  free(tb->Lq);
}

/* beta_k(T) = beta(T + k N_theta / 4), eq. (12) */
static int32_t beta_k(const or_problem* p, const or_tables* tb, int k, int64_t T) {
  return tb->beta[wrap(T + (int64_t)k * (p->nt / 4), p->nt)];
}

/* Turn curve offsets of eq. (17): LEFT uses (beta_0, beta_3), RIGHT uses
 * (beta_2, beta_1). */
static void turn_offset(const or_problem* p, const or_tables* tb, int left, int64_t T, int32_t* ox,
                        int32_t* oy) {
  if (left) {
    *ox = beta_k(p, tb, 0, T);
    *oy = beta_k(p, tb, 3, T);
  } else {
    *ox = beta_k(p, tb, 2, T);
    *oy = beta_k(p, tb, 1, T);
  }
}

static int is_turn(int mu) { return mu == OR_LF || mu == OR_LB || mu == OR_RF || mu == OR_RB; }
static int turn_left(int mu) { return mu == OR_LF || mu == OR_LB; }
/* eqs. (25)-(28): LF and RB step to T+1, RF and LB to T-1 */
static int turn_ascending(int mu) { return mu == OR_LF || mu == OR_RB; }

/* Straight sweeps (eq. 30/31 with the rule after eq. 31): the forward
 * maneuver walks y' upward when J >= 0, the backward one the other way. */
static int straight_ascending(int mu, int32_t J) { return (mu == OR_SF) ? (J > 0) : (J < 0); }

/* Sweep coordinate of step k.  Every straight line starts at y' = 0, which
 * lies in the wall (Sec. V.C), and then runs over the rest of the line. */
static int32_t straight_coord(int32_t N, int asc, int32_t k) { return asc ? k : wrap(N - k, N); }

/* eq. (23): vertex of line x' at sweep coordinate c in plane T */
static void straight_cell(const or_problem* p, const or_tables* tb, int32_t T, int32_t xp, int32_t c,
                          int32_t* i, int32_t* j) {
  int32_t b = tb->Bsk[(size_t)T * p->nx + c];
  if (tb->I[T] == 0) {
    *i = c;
    *j = wrap((int64_t)xp + b, p->nx);
  } else {
    *i = wrap((int64_t)xp + b, p->nx);
    *j = c;
  }
}

/* ------------------------------------------------------------------ */
/* edge weight and node relaxation                                    */
/* ------------------------------------------------------------------ */

/* time to traverse an edge leaving a vertex with obstacle code kappa */
static uint32_t edge_weight(uint32_t Lq, uint8_t kappa) {
  if (kappa == OR_HARD) return OR_INF;
  uint64_t slowness = 256u + 4u * (uint64_t)kappa;
  uint64_t w = ((uint64_t)Lq * slowness + 128u) >> 8;
  return w >= OR_INF ? OR_INF : (uint32_t)w;
}

/* One vertex p of a maneuver's curve, relaxed in the Star graph of Sec. V.A
 * as the sweeps of Sec. VIII.B walk it.  `arrive` is the best value reaching
 * p along the maneuver.  Leaving the maneuver costs nothing, so the
 * transition value of p becomes the smaller of its value before the sweep
 * and `arrive`; the maneuver vertex at p holds the better of continuing
 * (`arrive`) and entering the maneuver at p (the value before the sweep plus
 * ct); the edge leaving p adds its weight for the next vertex along the
 * curve.  Returns that next arriving value.  A hard vertex keeps the value
 * infinity (it is removed from the graph, App. E); its edge is infinite. */
static uint32_t relax_vertex(uint32_t* V, const uint8_t* Bv, size_t p, uint32_t ct, uint32_t Lq, uint32_t arrive) {
  const uint32_t before = V[p];
  const uint32_t in_maneuver = umin(arrive, sat_add(before, ct));
  V[p] = Bv[p] == OR_HARD ? OR_INF : umin(before, arrive);
  return sat_add(in_maneuver, edge_weight(Lq, Bv[p]));
}

/* ------------------------------------------------------------------ */
/* exported: tables                                                   */
/* ------------------------------------------------------------------ */

static int check_problem(const or_problem* p) {
  if (p->nx < 8 || p->nx > 4096) return OR_EINVAL;
  if (p->nt < 8 || p->nt % 8 != 0 || p->nt > 4096) return OR_EINVAL;
  if (!(p->R > 0.0)) return OR_EINVAL;
  if (p->nsched < 1 || p->nsched > 6) return OR_EINVAL;
  for (int k = 0; k < p->nsched; k++)
    if (p->sched[k] < 0 || p->sched[k] > 5) return OR_EINVAL;
  return OR_OK;
}

/* Copies the tables out: beta[nt], psi[nt], I[nt], J[nt], Bsk[nt*nx], Lq[6*nt]. */
int or_tables_export(const or_problem* p, int32_t* beta, int32_t* psi, int32_t* I, int32_t* J,
                     int32_t* Bsk, uint32_t* Lq) {
  int rc = check_problem(p);
  if (rc) return rc;
  or_tables tb;
  rc = tables_build(p, &tb);
  if (rc == OR_OK) {
    memcpy(beta, tb.beta, sizeof(int32_t) * p->nt);
    memcpy(psi, tb.psi, sizeof(int32_t) * p->nt);
    memcpy(I, tb.I, sizeof(int32_t) * p->nt);
    memcpy(J, tb.J, sizeof(int32_t) * p->nt);
    memcpy(Bsk, tb.Bsk, sizeof(int32_t) * (size_t)p->nt * p->nx);
    memcpy(Lq, tb.Lq, sizeof(uint32_t) * 6 * (size_t)p->nt);
  }
  tables_free(&tb);
  return rc;
}

/* ------------------------------------------------------------------ */
/* exported: obstacle rendering (Sec. VI)                             */
/* ------------------------------------------------------------------ */

/* Offsets of the footprint samples in plane T.
 * Sideways samples: g = -s..s along the left normal (-sin, cos); lengthwise
 * samples: g = -r..f along the heading (cos, sin).  With the half-cell
 * representation the sideways samples start from the represented point
 * (i + Psi_0/2... in half cells), eq. (16).  Rounding is half away from zero
 * so that the sample set of -theta is the exact mirror of that of theta. */
static void render_taps(const or_problem* p, const or_tables* tb, int32_t T, int32_t f, int32_t r,
                        int32_t s, int32_t* sdx, int32_t* sdy, int32_t* ldx, int32_t* ldy) {
  double sn = grid_sin(p->nt, T), cs = grid_cos(p->nt, T);
  double hx = p->half_cell ? 0.5 * (double)tb->psi[T] : 0.0;                     /* Psi_0 */
  double hy = p->half_cell ? 0.5 * (double)tb->psi[wrap(T + p->nt / 4, p->nt)] : 0.0; /* Psi_1 */
  for (int32_t g = -s; g <= s; g++) {
    sdx[g + s] = (int32_t)lround((double)g * -sn + hx);
    sdy[g + s] = (int32_t)lround((double)g * cs + hy);
  }
  for (int32_t g = -r; g <= f; g++) {
    ldx[g + r] = (int32_t)lround((double)g * cs);
    ldy[g + r] = (int32_t)lround((double)g * sn);
  }
}

/* Exports the tap offsets of plane T (arrays of 2s+1 and f+r+1 entries). */
int or_render_taps(const or_problem* p, int32_t T, int32_t f, int32_t r, int32_t s, int32_t* sdx,
                   int32_t* sdy, int32_t* ldx, int32_t* ldy) {
  int rc = check_problem(p);
  if (rc) return rc;
  if (f < 0 || r < 0 || s < 0 || T < 0 || T >= p->nt) return OR_EINVAL;
  or_tables tb;
  rc = tables_build(p, &tb);
  if (rc == OR_OK) render_taps(p, &tb, T, f, r, s, sdx, sdy, ldx, ldy);
  tables_free(&tb);
  return rc;
}

/* image: N x N codes, row-major (row j, column i).  B: N_R codes. */
int or_render(const or_problem* p, const uint8_t* image, int32_t f, int32_t r, int32_t s, uint8_t* B) {
  int rc = check_problem(p);
  if (rc) return rc;
  if (f < 0 || r < 0 || s < 0 || f + r + 1 > 4096 || 2 * s + 1 > 4096) return OR_EINVAL;
  int32_t N = p->nx, L = p->nt;
  size_t NN = (size_t)N * N;
  or_tables tb;
  rc = tables_build(p, &tb);
  uint8_t* img = (uint8_t*)malloc(NN);
  if (rc || !img) {
    tables_free(&tb);
    free(img);
    return OR_ENOMEM;
  }
  /* the one-cell hard wall at i = 0 and j = 0 (Sec. V.C), put into the image
   * before dilation so the vehicle box cannot reach through it */
  memcpy(img, image, NN);
  for (int32_t k = 0; k < N; k++) {
    img[k] = OR_HARD;             /* row j = 0 */
    img[(size_t)k * N] = OR_HARD; /* column i = 0 */
  }
  int rcs = OR_OK;
#pragma omp parallel
  {
    uint8_t* side = (uint8_t*)malloc(NN);
    int32_t* sdx = (int32_t*)malloc(sizeof(int32_t) * (2 * s + 1));
    int32_t* sdy = (int32_t*)malloc(sizeof(int32_t) * (2 * s + 1));
    int32_t* ldx = (int32_t*)malloc(sizeof(int32_t) * (f + r + 1));
    int32_t* ldy = (int32_t*)malloc(sizeof(int32_t) * (f + r + 1));
    if (!side || !sdx || !sdy || !ldx || !ldy) {
#pragma omp atomic write
      rcs = OR_ENOMEM;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int32_t T = 0; T < L; T++) {
        render_taps(p, &tb, T, f, r, s, sdx, sdy, ldx, ldy);
        /* sideways max pass */
        for (int32_t j = 0; j < N; j++)
          for (int32_t i = 0; i < N; i++) {
            uint8_t m = 0;
            for (int32_t g = 0; g < 2 * s + 1; g++) {
              uint8_t q = img[(size_t)wrap((int64_t)j + sdy[g], N) * N + wrap((int64_t)i + sdx[g], N)];
              if (q > m) m = q;
            }
            side[(size_t)j * N + i] = m;
          }
        /* lengthwise max pass */
        uint8_t* plane = B + (size_t)T * NN;
        for (int32_t j = 0; j < N; j++)
          for (int32_t i = 0; i < N; i++) {
            uint8_t m = 0;
            for (int32_t g = 0; g < f + r + 1; g++) {
              uint8_t q = side[(size_t)wrap((int64_t)j + ldy[g], N) * N + wrap((int64_t)i + ldx[g], N)];
              if (q > m) m = q;
            }
            plane[(size_t)j * N + i] = m;
          }
        /* the wall cells themselves are always vertices in collision, whatever
         * the footprint offsets */
        for (int32_t k = 0; k < N; k++) {
          plane[k] = OR_HARD;
          plane[(size_t)k * N] = OR_HARD;
        }
      }
    }
    free(side);
    free(sdx);
    free(sdy);
    free(ldx);
    free(ldy);
  }
  free(img);
  tables_free(&tb);
  return rcs;
}

/* ------------------------------------------------------------------ */
/* exported: init, sweeps, cycles                                     */
/* ------------------------------------------------------------------ */

int or_init(const or_problem* p, const uint8_t* B, uint32_t* V, int32_t si, int32_t sj, int32_t st) {
  int rc = check_problem(p);
  if (rc) return rc;
  if (si < 0 || sj < 0 || st < 0 || si >= p->nx || sj >= p->nx || st >= p->nt) return OR_EINVAL;
  size_t NR = (size_t)p->nx * p->nx * p->nt;
  size_t x0 = cell_index(p, si, sj, st);
  if (B[x0] == OR_HARD) return OR_ESTART;
  for (size_t x = 0; x < NR; x++) V[x] = OR_INF;
  V[x0] = 0;
  return OR_OK;
}

static void sweep_turn(const or_problem* p, const or_tables* tb, int mu, const uint8_t* B, uint32_t* V) {
  int32_t N = p->nx, L = p->nt;
  int left = turn_left(mu), asc = turn_ascending(mu);
  uint32_t ct = p->ct[mu], Lq = tb->Lq[(size_t)mu * L]; /* turn length is the same in every plane */
  /* One thread of the paper per curve (x', y').  The curves are disjoint, so
   * they are walked side by side here: carry[x'] is the value v that each
   * curve of the row y' carries. */
#pragma omp parallel
  {
    uint32_t* carry = (uint32_t*)malloc(sizeof(uint32_t) * N);
#pragma omp for schedule(static)
    for (int32_t yp = 0; yp < N; yp++) {
      for (int32_t xp = 0; xp < N; xp++) carry[xp] = OR_INF;
      /* two full loops around the cyclic theta axis (Sec. VIII.B) */
      for (int32_t t = 0; t < 2 * L; t++) {
        int32_t T = asc ? (t % L) : (L - 1 - (t % L));
        int32_t ox, oy;
        turn_offset(p, tb, left, T, &ox, &oy); /* eq. (17)-(18) */
        int32_t j = wrap((int64_t)yp + oy, N);
        for (int32_t xp = 0; xp < N; xp++) {
          int32_t i = wrap((int64_t)xp + ox, N);
          carry[xp] = relax_vertex(V, B, cell_index(p, i, j, T), ct, Lq, carry[xp]);
        }
      }
    }
    free(carry);
  }
}

static void sweep_straight(const or_problem* p, const or_tables* tb, int mu, const uint8_t* B,
                           uint32_t* V) {
  int32_t N = p->nx, L = p->nt;
  uint32_t ct = p->ct[mu];
#pragma omp parallel
  {
    uint32_t* carry = (uint32_t*)malloc(sizeof(uint32_t) * N);
#pragma omp for schedule(static)
    for (int32_t T = 0; T < L; T++) {
      int asc = straight_ascending(mu, tb->J[T]);
      uint32_t Lq = tb->Lq[(size_t)mu * L + T];
      /* one thread of the paper per line x'; one pass (Sec. VIII.B) */
      for (int32_t xp = 0; xp < N; xp++) carry[xp] = OR_INF;
      for (int32_t k = 0; k < N; k++) {
        int32_t c = straight_coord(N, asc, k);
        for (int32_t xp = 0; xp < N; xp++) {
          int32_t i, j;
          straight_cell(p, tb, T, xp, c, &i, &j);
          carry[xp] = relax_vertex(V, B, cell_index(p, i, j, T), ct, Lq, carry[xp]);
        }
      }
    }
    free(carry);
  }
}

int or_sweep(const or_problem* p, int32_t mu, const uint8_t* B, uint32_t* V) {
  int rc = check_problem(p);
  if (rc) return rc;
  if (mu < 0 || mu > 5) return OR_EINVAL;
  or_tables tb;
  rc = tables_build(p, &tb);
  if (rc == OR_OK) {
    if (is_turn(mu))
      sweep_turn(p, &tb, mu, B, V);
    else
      sweep_straight(p, &tb, mu, B, V);
  }
  tables_free(&tb);
  return rc;
}

/* N maneuver cycles over the schedule (Sec. XVI.A). */
int or_cycles(const or_problem* p, const uint8_t* B, uint32_t* V, int32_t n_cycles) {
  int rc = check_problem(p);
  if (rc) return rc;
  if (n_cycles < 0) return OR_EINVAL;
  or_tables tb;
  rc = tables_build(p, &tb);
  if (rc == OR_OK) {
    for (int32_t n = 0; n < n_cycles; n++)
      for (int32_t k = 0; k < p->nsched; k++) {
        int mu = p->sched[k];
        if (is_turn(mu))
          sweep_turn(p, &tb, mu, B, V);
        else
          sweep_straight(p, &tb, mu, B, V);
      }
  }
  tables_free(&tb);
  return rc;
}

/* ------------------------------------------------------------------ */
/* exported: goal search (Sec. IX)                                    */
/* ------------------------------------------------------------------ */

/* Among the vertices within max-norm distance d of the goal (each coordinate
 * taken modulo its dimension), skipping vertices in collision and
 * unreached ones, minimise V + w_xy (|dx| + |dy|) + w_t |dT|; ties go to the
 * smaller (|dx|+|dy|+|dT|, dT, dy, dx), so the goal itself wins a tie. */
int or_goal_search(const or_problem* p, const uint8_t* B, const uint32_t* V, int32_t gi, int32_t gj,
                   int32_t gt, int32_t d, uint32_t w_xy, uint32_t w_t, int32_t* best, uint32_t* score) {
  int rc = check_problem(p);
  if (rc) return rc;
  if (d < 0 || gi < 0 || gj < 0 || gt < 0 || gi >= p->nx || gj >= p->nx || gt >= p->nt) return OR_EINVAL;
  int found = 0;
  uint32_t bs = OR_INF;
  int32_t bm = 0, bt = 0, by = 0, bx = 0;
  for (int32_t dt = -d; dt <= d; dt++)
    for (int32_t dy = -d; dy <= d; dy++)
      for (int32_t dx = -d; dx <= d; dx++) {
        int32_t i = wrap((int64_t)gi + dx, p->nx), j = wrap((int64_t)gj + dy, p->nx);
        int32_t T = wrap((int64_t)gt + dt, p->nt);
        size_t x = cell_index(p, i, j, T);
        if (B[x] == OR_HARD || V[x] == OR_INF) continue;
        uint64_t pen = (uint64_t)w_xy * (uint64_t)(abs(dx) + abs(dy)) + (uint64_t)w_t * (uint64_t)abs(dt);
        uint32_t sc = sat_add(V[x], pen >= OR_INF ? OR_INF : (uint32_t)pen);
        int32_t m = abs(dx) + abs(dy) + abs(dt);
        int better = !found || sc < bs ||
                     (sc == bs && (m < bm || (m == bm && (dt < bt || (dt == bt && (dy < by || (dy == by && dx < bx)))))));
        if (better) {
          found = 1;
          bs = sc;
          bm = m;
          bt = dt;
          by = dy;
          bx = dx;
          best[0] = i;
          best[1] = j;
          best[2] = T;
        }
      }
  if (!found) return OR_EUNREACH;
  *score = bs;
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* exported: back-tracking (Sec. X, eq. 32)                           */
/* ------------------------------------------------------------------ */

/* The k-th vertex before (i, j, T) on the curve of maneuver mu through it,
 * in that maneuver's direction of travel.  Returns 0 when the curve has no
 * such vertex (a straight line reaches back only to its start in the wall). */
static int predecessor(const or_problem* p, const or_tables* tb, int mu, int32_t i, int32_t j, int32_t T,
                       int32_t k, int32_t* pi, int32_t* pj, int32_t* pT) {
  int32_t N = p->nx, L = p->nt;
  if (is_turn(mu)) {
    if (k >= L) return 0;
    int left = turn_left(mu);
    int32_t ox, oy, qx, qy;
    turn_offset(p, tb, left, T, &ox, &oy);
    int32_t xp = wrap((int64_t)i - ox, N), yp = wrap((int64_t)j - oy, N); /* inverse of eq. (18) */
    int32_t Tk = wrap(turn_ascending(mu) ? (int64_t)T - k : (int64_t)T + k, L);
    turn_offset(p, tb, left, Tk, &qx, &qy);
    *pi = wrap((int64_t)xp + qx, N);
    *pj = wrap((int64_t)yp + qy, N);
    *pT = Tk;
    return 1;
  }
  int asc = straight_ascending(mu, tb->J[T]);
  int32_t c = tb->I[T] == 0 ? i : j;
  int32_t other = tb->I[T] == 0 ? j : i;
  int32_t xp = wrap((int64_t)other - tb->Bsk[(size_t)T * N + c], N); /* eq. (29) */
  int32_t step = asc ? c : wrap(N - c, N);                           /* position in the sweep */
  if (k > step) return 0;
  straight_cell(p, tb, T, xp, straight_coord(N, asc, step - k), pi, pj);
  *pT = T;
  return 1;
}

/* Walks back from vertex `cur` to the start.  For every scheduled maneuver
 * every vertex p_k up the curve through the current vertex is a candidate
 * with value V(p_k) + ct + (sum of the k edges from p_k to the current
 * vertex); the smallest (value, schedule position, k) wins and becomes the
 * current vertex.  Steps come out goal first and are then reversed. */
int or_backtrack(const or_problem* p, const uint8_t* B, const uint32_t* V, int32_t si, int32_t sj,
                 int32_t st, const int32_t* goal, or_step* steps, int32_t cap, int32_t* n_steps) {
  int rc = check_problem(p);
  if (rc) return rc;
  int32_t N = p->nx, L = p->nt;
  or_tables tb;
  rc = tables_build(p, &tb);
  if (rc) {
    tables_free(&tb);
    return rc;
  }
  int32_t ci = goal[0], cj = goal[1], cT = goal[2];
  int32_t n = 0;
  int32_t limit = 1 << 20;
  rc = OR_OK;
  while (!(ci == si && cj == sj && cT == st)) {
    if (V[cell_index(p, ci, cj, cT)] == OR_INF || n >= limit) {
      rc = OR_EUNREACH;
      break;
    }
    uint32_t bc = OR_INF, bcost = 0;
    int32_t bk = 0, bi = 0, bj = 0, bT = 0, bmu = -1;
    int32_t maxk = N > L ? N : L;
    for (int32_t pos = 0; pos < p->nsched; pos++) {
      int mu = p->sched[pos];
      uint32_t E = 0;
      for (int32_t k = 1; k <= maxk; k++) {
        int32_t qi, qj, qT;
        if (!predecessor(p, &tb, mu, ci, cj, cT, k, &qi, &qj, &qT)) break;
        size_t q = cell_index(p, qi, qj, qT);
        E = sat_add(E, edge_weight(tb.Lq[(size_t)mu * L + qT], B[q]));
        if (E == OR_INF) break; /* a hard vertex ends the curve */
        uint32_t cand = sat_add(sat_add(V[q], p->ct[mu]), E);
        /* candidates arrive in increasing (position, k) order, so a strict
         * comparison keeps the smallest (value, position, k) */
        if (cand < bc) {
          bc = cand;
          bk = k;
          bmu = mu;
          bi = qi;
          bj = qj;
          bT = qT;
          bcost = sat_add(p->ct[mu], E);
        }
      }
    }
    if (bmu < 0 || bc == OR_INF) {
      rc = OR_EUNREACH;
      break;
    }
    if (n < cap) {
      or_step* sp = &steps[n];
      memset(sp, 0, sizeof(*sp));
      sp->maneuver = (uint8_t)bmu;
      sp->steps = (uint32_t)bk;
      sp->from[0] = (uint32_t)bi;
      sp->from[1] = (uint32_t)bj;
      sp->from[2] = (uint32_t)bT;
      sp->to[0] = (uint32_t)ci;
      sp->to[1] = (uint32_t)cj;
      sp->to[2] = (uint32_t)cT;
      sp->cost = bcost;
    }
    n++;
    ci = bi;
    cj = bj;
    cT = bT;
  }
  tables_free(&tb);
  *n_steps = n;
  if (rc) return rc;
  if (n > cap) return OR_ECAP;
  for (int32_t a = 0, b = n - 1; a < b; a++, b--) { /* start -> goal order */
    or_step t = steps[a];
    steps[a] = steps[b];
    steps[b] = t;
  }
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* exported: start sets and goal sets (Sec. III.A, IX, XII)           */
/* ------------------------------------------------------------------ */

/* A start: a pose with a cost, either at rest (maneuver < 0: the vehicle
 * may begin any maneuver there, paying its transition cost) or inside a
 * maneuver already in progress (Sec. XII: that maneuver continues without a
 * transition cost).  The second kind seeds every pose the maneuver reaches
 * from the start pose with cost + the edge sum so far, up to the first
 * vertex in collision (one loop for turns, to the end of the line for
 * straights). */
typedef struct {
  int32_t i, j, T;
  uint32_t cost;
  int32_t maneuver;
} or_start;

typedef struct {
  size_t x;      /* pose index */
  uint32_t value;
  int32_t start; /* index of the start that seeded it */
  int32_t k;     /* edges from the start pose along its maneuver */
} or_seed;

/* The k-th vertex after (i, j, T) on the curve of maneuver mu, in its
 * direction of travel; 0 when the curve has no such vertex. */
static int successor(const or_problem* p, const or_tables* tb, int mu, int32_t i, int32_t j, int32_t T, int32_t k,
                     int32_t* qi, int32_t* qj, int32_t* qT) {
  int32_t N = p->nx, L = p->nt;
  if (is_turn(mu)) {
    if (k >= L) return 0;
    int left = turn_left(mu);
    int32_t ox, oy, rx, ry;
    turn_offset(p, tb, left, T, &ox, &oy);
    int32_t xp = wrap((int64_t)i - ox, N), yp = wrap((int64_t)j - oy, N);
    int32_t Tk = wrap(turn_ascending(mu) ? (int64_t)T + k : (int64_t)T - k, L);
    turn_offset(p, tb, left, Tk, &rx, &ry);
    *qi = wrap((int64_t)xp + rx, N);
    *qj = wrap((int64_t)yp + ry, N);
    *qT = Tk;
    return 1;
  }
  int asc = straight_ascending(mu, tb->J[T]);
  int32_t c = tb->I[T] == 0 ? i : j;
  int32_t other = tb->I[T] == 0 ? j : i;
  int32_t xp = wrap((int64_t)other - tb->Bsk[(size_t)T * N + c], N);
  int32_t step = asc ? c : wrap(N - c, N);
  if (step + k > N - 1) return 0;
  straight_cell(p, tb, T, xp, straight_coord(N, asc, step + k), qi, qj);
  *qT = T;
  return 1;
}

/* Seeds of a start set, in start order and, per start, in k order.
 * Returns the count (at most cap), or a negative status. */
static int64_t make_seeds(const or_problem* p, const or_tables* tb, const uint8_t* B, const or_start* st, int32_t n,
                          or_seed* seeds, int64_t cap) {
  int64_t m = 0;
  for (int32_t s = 0; s < n; s++) {
    if (st[s].i < 0 || st[s].j < 0 || st[s].T < 0 || st[s].i >= p->nx || st[s].j >= p->nx || st[s].T >= p->nt ||
        st[s].maneuver > 5)
      return OR_EINVAL;
    size_t x0 = cell_index(p, st[s].i, st[s].j, st[s].T);
    if (B[x0] == OR_HARD) return OR_ESTART;
    if (m >= cap) return OR_ECAP;
    seeds[m++] = (or_seed){x0, st[s].cost, s, 0};
    int mu = st[s].maneuver;
    if (mu < 0) continue;
    uint32_t E = 0;
    int32_t ci = st[s].i, cj = st[s].j, cT = st[s].T;
    for (int32_t k = 1;; k++) {
      int32_t qi, qj, qT;
      E = sat_add(E, edge_weight(tb->Lq[(size_t)mu * p->nt + cT], B[cell_index(p, ci, cj, cT)]));
      if (E == OR_INF) break;
      if (!successor(p, tb, mu, st[s].i, st[s].j, st[s].T, k, &qi, &qj, &qT)) break;
      size_t q = cell_index(p, qi, qj, qT);
      if (B[q] == OR_HARD) break;
      if (m >= cap) return OR_ECAP;
      seeds[m++] = (or_seed){q, sat_add(st[s].cost, E), s, k};
      ci = qi;
      cj = qj;
      cT = qT;
    }
  }
  return m;
}

/* V = infinity, then every seed lowers its pose to its value. */
int or_init_set(const or_problem* p, const uint8_t* B, uint32_t* V, const or_start* st, int32_t n) {
  int rc = check_problem(p);
  if (rc) return rc;
  if (n < 1) return OR_EINVAL;
  or_tables tb;
  rc = tables_build(p, &tb);
  int64_t cap = (int64_t)n * ((p->nx > p->nt ? p->nx : p->nt) + 1);
  or_seed* seeds = (or_seed*)malloc(sizeof(or_seed) * (size_t)cap);
  if (rc == OR_OK && !seeds) rc = OR_ENOMEM;
  if (rc == OR_OK) {
    int64_t m = make_seeds(p, &tb, B, st, n, seeds, cap);
    if (m < 0) {
      rc = (int)m;
    } else {
      size_t NR = (size_t)p->nx * p->nx * p->nt;
      for (size_t x = 0; x < NR; x++) V[x] = OR_INF;
      for (int64_t e = 0; e < m; e++) V[seeds[e].x] = umin(V[seeds[e].x], seeds[e].value);
    }
  }
  free(seeds);
  tables_free(&tb);
  return rc;
}

/* Goal set with penalties (a reward expressed as its shortfall from the
 * largest reward, Sec. IX): the goal minimising V + penalty, skipping goals
 * in collision or unreached; ties go to the earlier goal. */
int or_goal_set(const or_problem* p, const uint8_t* B, const uint32_t* V, const int32_t* goals,
                const uint32_t* penalty, int32_t n, int32_t* best_k, uint32_t* score) {
  int rc = check_problem(p);
  if (rc) return rc;
  int found = 0;
  uint32_t bs = OR_INF;
  for (int32_t k = 0; k < n; k++) {
    int32_t i = goals[3 * k], j = goals[3 * k + 1], T = goals[3 * k + 2];
    if (i < 0 || j < 0 || T < 0 || i >= p->nx || j >= p->nx || T >= p->nt) return OR_EINVAL;
    size_t x = cell_index(p, i, j, T);
    if (B[x] == OR_HARD || V[x] == OR_INF) continue;
    uint32_t sc = sat_add(V[x], penalty[k]);
    if (!found || sc < bs) {
      found = 1;
      bs = sc;
      *best_k = k;
    }
  }
  if (!found) return OR_EUNREACH;
  *score = bs;
  return OR_OK;
}

/* Back-tracking to a start set: the walk of or_backtrack, ending at the
 * first pose that is a seed whose value equals V there (first seed in seed
 * order).  A seed inside an in-progress maneuver adds that maneuver's
 * steps from the start pose (cost: the edge sum, no transition). */
int or_backtrack_set(const or_problem* p, const uint8_t* B, const uint32_t* V, const or_start* st, int32_t n_st,
                     const int32_t* goal, or_step* steps, int32_t cap, int32_t* n_steps) {
  int rc = check_problem(p);
  if (rc) return rc;
  int32_t N = p->nx, L = p->nt;
  or_tables tb;
  rc = tables_build(p, &tb);
  int64_t scap = (int64_t)n_st * ((N > L ? N : L) + 1);
  or_seed* seeds = (or_seed*)malloc(sizeof(or_seed) * (size_t)scap);
  int64_t m = 0;
  if (rc == OR_OK && !seeds) rc = OR_ENOMEM;
  if (rc == OR_OK) {
    m = make_seeds(p, &tb, B, st, n_st, seeds, scap);
    if (m < 0) rc = (int)m;
  }
  int32_t ci = goal[0], cj = goal[1], cT = goal[2];
  int32_t n = 0;
  int32_t limit = 1 << 20;
  int64_t hit = -1;
  while (rc == OR_OK) {
    size_t cx = cell_index(p, ci, cj, cT);
    for (int64_t e = 0; e < m && hit < 0; e++)
      if (seeds[e].x == cx && seeds[e].value == V[cx]) hit = e;
    if (hit >= 0) break;
    if (V[cx] == OR_INF || n >= limit) {
      rc = OR_EUNREACH;
      break;
    }
    uint32_t bc = OR_INF, bcost = 0;
    int32_t bk = 0, bi = 0, bj = 0, bT = 0, bmu = -1;
    int32_t maxk = N > L ? N : L;
    for (int32_t pos = 0; pos < p->nsched; pos++) {
      int mu = p->sched[pos];
      uint32_t E = 0;
      for (int32_t k = 1; k <= maxk; k++) {
        int32_t qi, qj, qT;
        if (!predecessor(p, &tb, mu, ci, cj, cT, k, &qi, &qj, &qT)) break;
        size_t q = cell_index(p, qi, qj, qT);
        E = sat_add(E, edge_weight(tb.Lq[(size_t)mu * L + qT], B[q]));
        if (E == OR_INF) break;
        uint32_t cand = sat_add(sat_add(V[q], p->ct[mu]), E);
        if (cand < bc) {
          bc = cand;
          bk = k;
          bmu = mu;
          bi = qi;
          bj = qj;
          bT = qT;
          bcost = sat_add(p->ct[mu], E);
        }
      }
    }
    if (bmu < 0 || bc == OR_INF) {
      rc = OR_EUNREACH;
      break;
    }
    if (n < cap) {
      or_step* sp = &steps[n];
      memset(sp, 0, sizeof(*sp));
      sp->maneuver = (uint8_t)bmu;
      sp->steps = (uint32_t)bk;
      sp->from[0] = (uint32_t)bi;
      sp->from[1] = (uint32_t)bj;
      sp->from[2] = (uint32_t)bT;
      sp->to[0] = (uint32_t)ci;
      sp->to[1] = (uint32_t)cj;
      sp->to[2] = (uint32_t)cT;
      sp->cost = bcost;
    }
    n++;
    ci = bi;
    cj = bj;
    cT = bT;
  }
  if (rc == OR_OK && seeds[hit].k > 0) { /* the maneuver already in progress */
    const or_start* s0 = &st[seeds[hit].start];
    if (n < cap) {
      or_step* sp = &steps[n];
      memset(sp, 0, sizeof(*sp));
      sp->maneuver = (uint8_t)s0->maneuver;
      sp->steps = (uint32_t)seeds[hit].k;
      sp->from[0] = (uint32_t)s0->i;
      sp->from[1] = (uint32_t)s0->j;
      sp->from[2] = (uint32_t)s0->T;
      sp->to[0] = (uint32_t)ci;
      sp->to[1] = (uint32_t)cj;
      sp->to[2] = (uint32_t)cT;
      sp->cost = seeds[hit].value - s0->cost;
    }
    n++;
  }
  free(seeds);
  tables_free(&tb);
  *n_steps = n;
  if (rc) return rc;
  if (n > cap) return OR_ECAP;
  for (int32_t a = 0, b = n - 1; a < b; a++, b--) {
    or_step t = steps[a];
    steps[a] = steps[b];
    steps[b] = t;
  }
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* exported: soft obstacle costs from a distance transform (Sec. VI-VII) */
/* ------------------------------------------------------------------ */

/* The reciprocal of the highest allowed velocity is a function of the
 * distance to the nearest hard obstacle (Sec. VI).  Here the function is a
 * table over the squared Euclidean distance in cells: a free pixel gets
 * table[min(d^2, len - 1)], a hard pixel (code 255) stays 255; with no hard
 * pixel at all, d^2 counts as unbounded (the last entry).  d^2 is the plain
 * minimum over hard pixels of dx^2 + dy^2, evaluated through the identity
 * min over (i', j') = min over i' of ((i - i')^2 + min over j' (j - j')^2),
 * the inner minimum per column first. */
int or_soft_costs(const uint8_t* image, int32_t n, const uint8_t* table, int32_t len, uint8_t* out) {
  if (n < 1 || len < 1) return OR_EINVAL;
  const int64_t far = (int64_t)1 << 40;
  int64_t* g = (int64_t*)malloc(sizeof(int64_t) * (size_t)n * n); /* g[j][i]: (j - nearest hard row in column i)^2 */
  if (!g) return OR_ENOMEM;
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < n; i++)
    for (int32_t j = 0; j < n; j++) {
      int64_t best = far;
      for (int32_t jj = 0; jj < n; jj++)
        if (image[(size_t)jj * n + i] == OR_HARD) {
          int64_t d = (int64_t)(j - jj) * (j - jj);
          if (d < best) best = d;
        }
      g[(size_t)j * n + i] = best;
    }
#pragma omp parallel for schedule(static)
  for (int32_t j = 0; j < n; j++)
    for (int32_t i = 0; i < n; i++) {
      size_t x = (size_t)j * n + i;
      if (image[x] == OR_HARD) {
        out[x] = OR_HARD;
        continue;
      }
      int64_t best = far;
      for (int32_t ii = 0; ii < n; ii++) {
        int64_t d = (int64_t)(i - ii) * (i - ii) + g[(size_t)j * n + ii];
        if (d < best) best = d;
      }
      out[x] = table[best < len - 1 ? best : len - 1];
    }
  free(g);
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* exported: reachability with maneuver counting (App. C)             */
/* ------------------------------------------------------------------ */

/* App. C replaces the costs by the number of maneuvers: edges inside a
 * maneuver cost nothing, every transition costs one, and only hard
 * obstacles remain (any code below OR_HARD counts as free).  A vertex then
 * needs one bit per maneuver count, "reachable with at most m maneuvers".
 * The paper stores the bit inverted (0 = reachable) so that its sweep is an
 * AND with the previous volume followed by an OR with the obstacle bit; here
 * the same logic is written with 1 = reachable:
 *   along a curve:  r = (r_carried OR R_m(X)) AND free(X);  out(X) = r
 * and every maneuver of a cycle starts from the same R_m (the volumes of the
 * maneuver vertices are separate), after which R_{m+1} is the union of the
 * maneuvers' outputs.  Turns close their circle (two loops), straights start
 * at the wall, as in the cost sweeps.  The result is stored as a level per
 * vertex: the smallest m with the vertex in R_m (255 when none up to n). */

static void reach_turn(const or_problem* p, const or_tables* tb, int mu, const uint8_t* B, const uint8_t* R,
                       uint8_t* out) {
  int32_t N = p->nx, L = p->nt;
  int left = turn_left(mu), asc = turn_ascending(mu);
#pragma omp parallel
  {
    uint8_t* carry = (uint8_t*)malloc((size_t)N);
#pragma omp for schedule(static)
    for (int32_t yp = 0; yp < N; yp++) {
      memset(carry, 0, (size_t)N);
      for (int32_t t = 0; t < 2 * L; t++) {
        int32_t T = asc ? (t % L) : (L - 1 - (t % L));
        int32_t ox, oy;
        turn_offset(p, tb, left, T, &ox, &oy);
        int32_t j = wrap((int64_t)yp + oy, N);
        for (int32_t xp = 0; xp < N; xp++) {
          size_t x = cell_index(p, wrap((int64_t)xp + ox, N), j, T);
          uint8_t r = (uint8_t)((carry[xp] | R[x]) & (B[x] != OR_HARD));
          out[x] |= r;
          carry[xp] = r;
        }
      }
    }
    free(carry);
  }
}

static void reach_straight(const or_problem* p, const or_tables* tb, int mu, const uint8_t* B, const uint8_t* R,
                           uint8_t* out) {
  int32_t N = p->nx, L = p->nt;
#pragma omp parallel
  {
    uint8_t* carry = (uint8_t*)malloc((size_t)N);
#pragma omp for schedule(static)
    for (int32_t T = 0; T < L; T++) {
      int asc = straight_ascending(mu, tb->J[T]);
      memset(carry, 0, (size_t)N);
      for (int32_t k = 0; k < N; k++) {
        int32_t c = straight_coord(N, asc, k);
        for (int32_t xp = 0; xp < N; xp++) {
          int32_t i, j;
          straight_cell(p, tb, T, xp, c, &i, &j);
          size_t x = cell_index(p, i, j, T);
          uint8_t r = (uint8_t)((carry[xp] | R[x]) & (B[x] != OR_HARD));
          out[x] |= r;
          carry[xp] = r;
        }
      }
    }
    free(carry);
  }
}

/* level: N_R bytes out.  Start must be free (OR_ESTART otherwise); 0 <=
 * n_cycles <= 254. */
int or_reach(const or_problem* p, const uint8_t* B, int32_t si, int32_t sj, int32_t st, int32_t n_cycles,
             uint8_t* level) {
  int rc = check_problem(p);
  if (rc) return rc;
  if (n_cycles < 0 || n_cycles > 254) return OR_EINVAL;
  if (si < 0 || sj < 0 || st < 0 || si >= p->nx || sj >= p->nx || st >= p->nt) return OR_EINVAL;
  size_t NR = (size_t)p->nx * p->nx * p->nt, x0 = cell_index(p, si, sj, st);
  if (B[x0] == OR_HARD) return OR_ESTART;
  or_tables tb;
  rc = tables_build(p, &tb);
  uint8_t* R = (uint8_t*)calloc(NR, 1);
  uint8_t* next = (uint8_t*)calloc(NR, 1);
  if (rc == OR_OK && (!R || !next)) rc = OR_ENOMEM;
  if (rc == OR_OK) {
    memset(level, 255, NR);
    R[x0] = 1;
    level[x0] = 0;
    for (int32_t m = 0; m < n_cycles; m++) {
      memset(next, 0, NR);
      for (int32_t k = 0; k < p->nsched; k++) {
        int mu = p->sched[k];
        if (is_turn(mu))
          reach_turn(p, &tb, mu, B, R, next);
        else
          reach_straight(p, &tb, mu, B, R, next);
      }
      for (size_t x = 0; x < NR; x++)
        if (next[x] && level[x] == 255) level[x] = (uint8_t)(m + 1);
      uint8_t* t = R;
      R = next;
      next = t;
    }
  }
  free(R);
  free(next);
  tables_free(&tb);
  return rc;
}

/* Goal search on levels: among the vertices within max-norm distance d of
 * the goal (coordinates modulo their dimension) with a level, the smallest
 * (level, |dx|+|dy|+|dT|, dT, dy, dx). */
int or_reach_goal(const or_problem* p, const uint8_t* level, int32_t gi, int32_t gj, int32_t gt, int32_t d,
                  int32_t* best, int32_t* best_level) {
  int rc = check_problem(p);
  if (rc) return rc;
  if (d < 0 || gi < 0 || gj < 0 || gt < 0 || gi >= p->nx || gj >= p->nx || gt >= p->nt) return OR_EINVAL;
  int found = 0;
  int32_t bl = 0, bm = 0, bt = 0, by = 0, bx = 0;
  for (int32_t dt = -d; dt <= d; dt++)
    for (int32_t dy = -d; dy <= d; dy++)
      for (int32_t dx = -d; dx <= d; dx++) {
        int32_t i = wrap((int64_t)gi + dx, p->nx), j = wrap((int64_t)gj + dy, p->nx);
        int32_t T = wrap((int64_t)gt + dt, p->nt);
        int32_t l = level[cell_index(p, i, j, T)];
        if (l == 255) continue;
        int32_t m = abs(dx) + abs(dy) + abs(dt);
        int better = !found || l < bl ||
                     (l == bl && (m < bm || (m == bm && (dt < bt || (dt == bt && (dy < by || (dy == by && dx < bx)))))));
        if (better) {
          found = 1;
          bl = l;
          bm = m;
          bt = dt;
          by = dy;
          bx = dx;
          best[0] = i;
          best[1] = j;
          best[2] = T;
        }
      }
  if (!found) return OR_EUNREACH;
  *best_level = bl;
  return OR_OK;
}

/* Back-tracking on levels: from a vertex of level m >= 1, the first
 * scheduled maneuver (in schedule order) with a vertex p_k, k steps up its
 * curve through free vertices, of level m - 1, nearest first; that vertex
 * becomes the current one.  Every step is one maneuver (cost 1).  Steps come
 * out start -> goal. */
int or_reach_backtrack(const or_problem* p, const uint8_t* B, const uint8_t* level, const int32_t* goal,
                       or_step* steps, int32_t cap, int32_t* n_steps) {
  int rc = check_problem(p);
  if (rc) return rc;
  int32_t N = p->nx, L = p->nt;
  or_tables tb;
  rc = tables_build(p, &tb);
  if (rc) {
    tables_free(&tb);
    return rc;
  }
  int32_t ci = goal[0], cj = goal[1], cT = goal[2];
  int32_t n = 0;
  int32_t m = level[cell_index(p, ci, cj, cT)];
  if (m == 255) rc = OR_EUNREACH;
  int32_t maxk = N > L ? N : L;
  while (rc == OR_OK && m > 0) {
    int32_t bk = 0, bi = 0, bj = 0, bT = 0, bmu = -1;
    for (int32_t pos = 0; pos < p->nsched && bmu < 0; pos++) {
      int mu = p->sched[pos];
      for (int32_t k = 1; k <= maxk; k++) {
        int32_t qi, qj, qT;
        if (!predecessor(p, &tb, mu, ci, cj, cT, k, &qi, &qj, &qT)) break;
        size_t q = cell_index(p, qi, qj, qT);
        if (B[q] == OR_HARD) break; /* a hard vertex ends the curve */
        if (level[q] == m - 1) {
          bk = k;
          bmu = mu;
          bi = qi;
          bj = qj;
          bT = qT;
          break;
        }
      }
    }
    if (bmu < 0) {
      rc = OR_EUNREACH; /* cannot happen for levels made by or_reach */
      break;
    }
    if (n < cap) {
      or_step* sp = &steps[n];
      memset(sp, 0, sizeof(*sp));
      sp->maneuver = (uint8_t)bmu;
      sp->steps = (uint32_t)bk;
      sp->from[0] = (uint32_t)bi;
      sp->from[1] = (uint32_t)bj;
      sp->from[2] = (uint32_t)bT;
      sp->to[0] = (uint32_t)ci;
      sp->to[1] = (uint32_t)cj;
      sp->to[2] = (uint32_t)cT;
      sp->cost = 1;
    }
    n++;
    ci = bi;
    cj = bj;
    cT = bT;
    m--;
  }
  tables_free(&tb);
  *n_steps = n;
  if (rc) return rc;
  if (n > cap) return OR_ECAP;
  for (int32_t a = 0, b = n - 1; a < b; a++, b--) {
    or_step t = steps[a];
    steps[a] = steps[b];
    steps[b] = t;
  }
  return OR_OK;
}

/* Number of host threads the oracle uses; returns the count in effect. */
int or_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}
