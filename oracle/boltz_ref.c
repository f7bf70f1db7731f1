/*
 * boltz_ref.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY; see the
 * header).  Every loop below follows the paper's statement of the method in
 * the order the paper gives it; nothing is blocked, fused or reordered.
 *
 * Sections of the paper followed here:
 *   Sec. 2  Eqs. definition, MaxwellDist, devIntColl   deviational form
 *   Sec. 2  Eqs. densita..sforzi                       moments (re-derived in V0 units)
 *   Sec. 2  Eq. bcMax and the zero-net-flux condition  diffuse walls
 *   Sec. 3  Eq. streaming2D                            first-order upwind streaming
 *   Sec. 3  Eqs. coll8Dim, monteCarloInt               MC collision integral
 *   Sec. 3  Eq. collision_step                         explicit (Jacobi) update
 *   Alg. 3                                             in-place sequential update (option)
 *   Sec. 3  Eqs. rinorm_a, correzione                  conservation correction
 *   Sec. 5.1                                           units, driven cavity, CFL
 * The readings taken where the paper is silent or garbled are listed in the
 * repository's design notes; the ones that shape a formula are repeated at
 * the formula.
 */
#include "boltz_ref.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define INV_SQRT_PI 0.56418958354775628694807945156077
#define PI_OVER_4 0.78539816339744830961566084581988
#define TWO_PI 6.28318530717958647692528676655901
#define FIELD_BITS 12 /* bits of a Philox word that select one node index */

enum { WALL_LEFT = 0, WALL_RIGHT = 1, WALL_BOTTOM = 2, WALL_TOP = 3 };

struct boltz_ref_ctx {
  boltz_ref_problem p;
  int n[3];
  double a[3];
  int nv, ncells;
  double dvel[3];
  double inv_cell[3]; /* n / (2 a): maps x + a to a cell coordinate */
  int stretched;      /* cells in geometric progression (Sec. 5.1)        */
  double* edge[3];    /* stretched grids: cell edges e_0 = -a .. e_n = a    */
  double* v[3];
  double* om[3];
  double Om[3];
  uint64_t* T[3]; /* T[k][i] = T_i for i in [1, n); T[k][0] = 0 */
  double* pphi[3];  /* realised per-axis Maxwellian law (T_{i+1} - T_i) 2^-12 */
  int sstretched;   /* spatial cells in geometric progression (Sec. 5.1) */
  double* wx;       /* widths of the nx spatial cells along x            */
  double* wy;       /* ... and of the ny cells along y                   */
  double* punif[3]; /* realised per-axis uniform law of floor(f n / 2^12)     */
  double beta;      /* weight of the uniform component, mix16 / 16           */
  double dx, dy, dt, K, W, qfac;
  char err[256];
};

static char g_create_err[256];

static void set_err(char* buf, const char* msg) {
  strncpy(buf, msg, 255);
  buf[255] = 0;
}

void boltz_ref_set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

int boltz_ref_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

const char* boltz_ref_last_error(const boltz_ref_ctx* ctx) {
  return ctx ? ctx->err : g_create_err;
}

/* ---------------------------------------------------------------- setup -- */

void boltz_ref_destroy(boltz_ref_ctx* c) {
  if (!c) return;
  for (int k = 0; k < 3; ++k) {
    free(c->v[k]);
    free(c->om[k]);
    free(c->T[k]);
    free(c->pphi[k]);
    free(c->punif[k]);
    free(c->edge[k]);
  }
  free(c->wx);
  free(c->wy);
  free(c);
}

int boltz_ref_create(const boltz_ref_problem* p, boltz_ref_ctx** out) {
  if (!p || !out) {
    set_err(g_create_err, "null argument");
    return BOLTZ_REF_EINVAL;
  }
  *out = NULL;
  int min_cells = (p->bc == BOLTZ_REF_BC_CAVITY) ? 2 : 1;
  if (p->nx < min_cells || p->ny < min_cells || p->nx > 100000 || p->ny > 100000) {
    set_err(g_create_err, "nx, ny out of range (cavity needs >= 2)");
    return BOLTZ_REF_EINVAL;
  }
  for (int k = 0; k < 3; ++k) {
    if (p->nv[k] < 1 || p->nv[k] > 255 || !(p->vmax[k] > 0.0)) {
      set_err(g_create_err, "velocity grid out of range (1 <= nv <= 255, vmax > 0)");
      return BOLTZ_REF_EINVAL;
    }
  }
  if (!(p->delta > 0.0) || !(p->eps > 0.0) || (p->order != 1 && p->order != 2) ||
      (p->bc != BOLTZ_REF_BC_CAVITY && p->bc != BOLTZ_REF_BC_PERIODIC) || p->n_pairs < 0 ||
      p->n_pairs >= (int64_t)1 << 31 || p->sample_group < 0 || p->mix16 > 16 ||
      (!(p->dt > 0.0) && !(p->cfl > 0.0))) {
    set_err(g_create_err, "invalid scalar parameter");
    return BOLTZ_REF_EINVAL;
  }
  /* rv: 0 or 1 = uniform velocity cells; 0 < rv < 1 = cells stretched in
   * the progression ratio rv, smallest at the origin (Sec. 5.1), which needs
   * an even cell count per axis */
  const int stretched = (p->rv != 0.0 && p->rv != 1.0);
  if (stretched && (!(p->rv > 0.0 && p->rv < 1.0) || (p->nv[0] & 1) || (p->nv[1] & 1) || (p->nv[2] & 1))) {
    set_err(g_create_err, "stretched velocity grid needs 0 < rv < 1 and an even cell count per axis");
    return BOLTZ_REF_EINVAL;
  }
  /* rx, ry: 0 or 1 = uniform spatial cells; 0 < r < 1 = stretched (Sec.
   * 5.1), with the first-order scheme of Eq. streaming2D only */
  const int sx_str = (p->rx != 0.0 && p->rx != 1.0), sy_str = (p->ry != 0.0 && p->ry != 1.0);
  if ((sx_str && !(p->rx > 0.0 && p->rx < 1.0)) || (sy_str && !(p->ry > 0.0 && p->ry < 1.0)) ||
      ((sx_str || sy_str) && p->order != 1)) {
    set_err(g_create_err, "stretched spatial cells need 0 < rx, ry < 1 and first-order streaming");
    return BOLTZ_REF_EINVAL;
  }
  boltz_ref_ctx* c = (boltz_ref_ctx*)calloc(1, sizeof(*c));
  if (!c) {
    set_err(g_create_err, "out of memory");
    return BOLTZ_REF_ENOMEM;
  }
  c->p = *p;
  c->nv = 1;
  for (int k = 0; k < 3; ++k) {
    int n = p->nv[k];
    double a = p->vmax[k];
    c->n[k] = n;
    c->a[k] = a;
    c->nv *= n;
    c->v[k] = (double*)malloc(sizeof(double) * n);
    c->om[k] = (double*)malloc(sizeof(double) * n);
    c->T[k] = (uint64_t*)malloc(sizeof(uint64_t) * n);
    c->pphi[k] = (double*)malloc(sizeof(double) * n);
    c->punif[k] = (double*)malloc(sizeof(double) * n);
    if (!c->v[k] || !c->om[k] || !c->T[k] || !c->pphi[k] || !c->punif[k]) {
      boltz_ref_destroy(c);
      set_err(g_create_err, "out of memory");
      return BOLTZ_REF_ENOMEM;
    }
    /* Sec. 3: h is constant in each velocity cell with the node at the cell
     * centre; uniform cells on [-a, a].  The node formula is exactly
     * antisymmetric in floating point. */
    c->dvel[k] = (2.0 * a) / n;
    c->inv_cell[k] = (double)n / (2.0 * a);
    double om_sum = 0.0;
    if (!stretched) {
      for (int i = 0; i < n; ++i) {
        double vi = ((double)(2 * i + 1 - n) * a) / n;
        c->v[k][i] = vi;
        /* per-axis midpoint weight of Phi0: omega = dv exp(-v^2)/sqrt(pi) */
        c->om[k][i] = (c->dvel[k] * exp(-(vi * vi))) * INV_SQRT_PI;
        om_sum += c->om[k][i];
      }
    } else {
      /* Sec. 5.1: cell lengths stretched in the progression ratio rv, the
       * smallest at the origin: on each half axis the i-th cell from the
       * origin is w0 rv^-i long, i = 0 .. m-1 (m = n/2), and the lengths add
       * up to a; the outermost edge is set to a exactly.  Nodes at the cell
       * centres, the negative half the exact mirror of the positive one. */
      const int m = n / 2;
      double* e = (double*)malloc(sizeof(double) * (n + 1));
      double* E = (double*)malloc(sizeof(double) * (m + 1));
      c->edge[k] = e;
      if (!e || !E) {
        free(E);
        boltz_ref_destroy(c);
        set_err(g_create_err, "out of memory");
        return BOLTZ_REF_ENOMEM;
      }
      double sum = 0.0, t = 1.0;
      for (int i = 0; i < m; ++i) {
        sum += t;
        t /= p->rv;
      }
      const double w0 = a / sum;
      E[0] = 0.0;
      t = 1.0;
      for (int i = 0; i < m; ++i) {
        E[i + 1] = E[i] + w0 * t;
        t /= p->rv;
      }
      E[m] = a;
      for (int i = 0; i <= m; ++i) {
        e[m + i] = E[i];
        e[m - i] = -E[i];
      }
      for (int i = 0; i < m; ++i) {
        const double vi = 0.5 * (E[i] + E[i + 1]);
        c->v[k][m + i] = vi;
        c->v[k][m - 1 - i] = -vi;
      }
      free(E);
      for (int i = 0; i < n; ++i) {
        const double vi = c->v[k][i];
        c->om[k][i] = ((e[i + 1] - e[i]) * exp(-(vi * vi))) * INV_SQRT_PI;
        om_sum += c->om[k][i];
      }
    }
    c->Om[k] = om_sum;
    /* cumulative thresholds of the per-axis node law, on 12-bit fields */
    double s = 0.0;
    c->T[k][0] = 0;
    for (int i = 0; i < n; ++i) {
      if (i > 0) c->T[k][i] = (uint64_t)nearbyint(ldexp(s / om_sum, FIELD_BITS));
      s += c->om[k][i];
    }
    /* realised probabilities of the two per-axis laws on a field f in
     * [0, 2^12): node i of the Maxwellian law for f in [T_i, T_{i+1}); node i
     * of the uniform law for floor(f n / 2^12) = i, i.e.
     * f in [ceil(i 2^12/n), ceil((i+1) 2^12/n)) */
    for (int i = 0; i < n; ++i) {
      uint64_t hi = (i + 1 < n) ? c->T[k][i + 1] : ((uint64_t)1 << FIELD_BITS);
      c->pphi[k][i] = ldexp((double)(hi - c->T[k][i]), -FIELD_BITS);
      uint64_t lo_u = (((uint64_t)i << FIELD_BITS) + (uint64_t)n - 1) / (uint64_t)n;
      uint64_t hi_u = (((uint64_t)(i + 1) << FIELD_BITS) + (uint64_t)n - 1) / (uint64_t)n;
      c->punif[k][i] = ldexp((double)(hi_u - lo_u), -FIELD_BITS);
    }
  }
  /* Eq. coll8Dim read as an importance-sampling estimate is unbiased only if
   * every node the integrand reaches has a positive probability of being
   * drawn.  The Maxwellian law on 12-bit fields gives probability zero to
   * the far-tail nodes of wide grids (T_{i+1} = T_i); without the uniform
   * component those nodes would never be drawn and their loss terms would
   * be dropped, so the pure Maxwellian law (mix16 = 0) is refused there. */
  if (p->mix16 == 0 && !(p->flags & BOLTZ_REF_CONTINUOUS)) {
    for (int k = 0; k < 3; ++k)
      for (int i = 0; i < c->n[k]; ++i)
        if (!(c->pphi[k][i] > 0.0)) {
          boltz_ref_destroy(c);
          set_err(g_create_err,
                  "mix16 = 0: the Maxwellian node law gives probability zero to tail nodes of this "
                  "velocity grid (biased estimate); use mix16 > 0");
          return BOLTZ_REF_EINVAL;
        }
  }
  c->stretched = stretched;
  c->beta = p->mix16 / 16.0;
  c->ncells = p->nx * p->ny;
  c->dx = 1.0 / p->nx;
  c->dy = 1.0 / p->ny;
  /* Sec. 5.1: spatial cell lengths in geometric progression.  Along x the
   * cell at distance d (in cells) from the nearer side wall is w0 rx^-d long,
   * along y the cell d cells below the lid w0 ry^-d; the lengths add up to
   * the cavity side 1.  Uniform cells: all 1/n. */
  c->sstretched = sx_str || sy_str;
  c->wx = (double*)malloc(sizeof(double) * p->nx);
  c->wy = (double*)malloc(sizeof(double) * p->ny);
  {
    double sum = 0.0;
    for (int i = 0; i < p->nx; ++i) {
      int d = i < p->nx - 1 - i ? i : p->nx - 1 - i;
      c->wx[i] = sx_str ? pow(p->rx, -d) : 1.0;
      sum += c->wx[i];
    }
    for (int i = 0; i < p->nx; ++i) c->wx[i] /= sum;
    sum = 0.0;
    for (int i = 0; i < p->ny; ++i) {
      c->wy[i] = sy_str ? pow(p->ry, -(p->ny - 1 - i)) : 1.0;
      sum += c->wy[i];
    }
    for (int i = 0; i < p->ny; ++i) c->wy[i] /= sum;
  }
  double mwx = c->wx[0], mwy = c->wy[0];
  for (int i = 0; i < p->nx; ++i) mwx = c->wx[i] < mwx ? c->wx[i] : mwx;
  for (int i = 0; i < p->ny; ++i) mwy = c->wy[i] < mwy ? c->wy[i] : mwy;
  if (!c->sstretched) {
    mwx = c->dx;
    mwy = c->dy;
  }
  double vmx = fabs(c->v[0][0]), vmy = fabs(c->v[1][0]);
  if (p->dt > 0.0) {
    c->dt = p->dt;
  } else {
    /* Sec. 5.1: the largest Courant number over nodes, cells and axes
     * equals cfl */
    double rx = vmx / mwx, ry = vmy / mwy;
    c->dt = p->cfl / (rx > ry ? rx : ry);
  }
  double cx = vmx * c->dt / mwx, cy = vmy * c->dt / mwy;
  int stable = (p->order == 1) ? (cx + cy <= 1.0 + 1e-12) : (cx <= 1.0 + 1e-12 && cy <= 1.0 + 1e-12);
  if (!stable && !(p->flags & BOLTZ_REF_ALLOW_UNSTABLE)) {
    boltz_ref_destroy(c);
    set_err(g_create_err, "time step violates the Courant limit of the streaming scheme");
    return BOLTZ_REF_EINVAL;
  }
  /* Collision constant K = pi n0 sigma^2 from lambda0 = mu0/p0 sqrt(2 R T0)
   * with the hard-sphere viscosity (Chapman-Cowling, 1.016034 correction):
   * K = (5/16) sqrt(2 pi) 1.016034 delta. */
  c->K = 0.3125 * sqrt(TWO_PI) * 1.016034 * p->delta;
  c->W = (c->Om[0] * c->Om[1]) * c->Om[2];
  c->qfac = (p->n_pairs > 0) ? (c->dt * c->K) / (double)p->n_pairs : 0.0;
  *out = c;
  return BOLTZ_REF_OK;
}

int boltz_ref_info(const boltz_ref_ctx* c, double* out) {
  if (!c || !out) return BOLTZ_REF_EINVAL;
  out[BOLTZ_REF_INFO_DT] = c->dt;
  out[BOLTZ_REF_INFO_K] = c->K;
  out[BOLTZ_REF_INFO_W] = c->W;
  out[BOLTZ_REF_INFO_QFAC] = c->qfac;
  out[BOLTZ_REF_INFO_DX] = c->dx;
  out[BOLTZ_REF_INFO_DY] = c->dy;
  out[BOLTZ_REF_INFO_NCELLS] = c->ncells;
  out[BOLTZ_REF_INFO_NV] = c->nv;
  return BOLTZ_REF_OK;
}

int boltz_ref_cell_widths(const boltz_ref_ctx* c, int axis, double* widths) {
  if (!c || axis < 0 || axis > 1 || !widths) return BOLTZ_REF_EINVAL;
  const int n = axis == 0 ? c->p.nx : c->p.ny;
  for (int i = 0; i < n; ++i) widths[i] = axis == 0 ? c->wx[i] : c->wy[i];
  return BOLTZ_REF_OK;
}

int boltz_ref_axis_edges(const boltz_ref_ctx* c, int axis, double* edges) {
  if (!c || axis < 0 || axis > 2 || !edges) return BOLTZ_REF_EINVAL;
  const int n = c->n[axis];
  for (int i = 0; i <= n; ++i)
    edges[i] = c->stretched ? c->edge[axis][i] : -c->a[axis] + i * c->dvel[axis];
  return BOLTZ_REF_OK;
}

int boltz_ref_axis(const boltz_ref_ctx* c, int axis, double* v, double* omega, uint64_t* thr) {
  if (!c || axis < 0 || axis > 2) return BOLTZ_REF_EINVAL;
  for (int i = 0; i < c->n[axis]; ++i) {
    if (v) v[i] = c->v[axis][i];
    if (omega) omega[i] = c->om[axis][i];
    if (thr && i > 0) thr[i - 1] = c->T[axis][i];
  }
  return BOLTZ_REF_OK;
}

/* -------------------------------------------------------- node helpers -- */

static void node_idx(const boltz_ref_ctx* c, int j, int* jx, int* jy, int* jz) {
  *jz = j % c->n[2];
  *jy = (j / c->n[2]) % c->n[1];
  *jx = j / (c->n[2] * c->n[1]);
}

static int node_of(const boltz_ref_ctx* c, int jx, int jy, int jz) {
  return (jx * c->n[1] + jy) * c->n[2] + jz;
}

static double node_w(const boltz_ref_ctx* c, int jx, int jy, int jz) {
  return (c->om[0][jx] * c->om[1][jy]) * c->om[2][jz];
}

static double node_w_flat(const boltz_ref_ctx* c, int j) {
  int jx, jy, jz;
  node_idx(c, j, &jx, &jy, &jz);
  return node_w(c, jx, jy, jz);
}

/* ------------------------------------------------------------- Philox -- */

/* Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw (SC'11):
 * ten rounds of two 32x32->64 multiplies with a Weyl-sequence key schedule. */
void boltz_ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x0 = y0;
    x1 = y1;
    x2 = y2;
    x3 = y3;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

/* ------------------------------------------------------- direction map -- */

/* cos and sin of 2 pi u for u in (0, 1): reduce to an octant exactly
 * (8u is exact for u = (r + 1/2) 2^-16), fold to [0, pi/4], then Taylor
 * polynomials in z^2 of degree 13 (sin) and 12 (cos): truncation below
 * 4e-13 on [0, pi/4]. */
void boltz_ref_cos_sin_2pi(double u, double* cs, double* sn) {
  double t = u * 8.0;
  double o = floor(t);
  double f = t - o;
  int oct = ((int)o) & 7;
  double z = ((oct & 1) ? (1.0 - f) : f) * PI_OVER_4;
  double z2 = z * z;
  double ps = 1.0 / 6227020800.0;
  ps = -1.0 / 39916800.0 + z2 * ps;
  ps = 1.0 / 362880.0 + z2 * ps;
  ps = -1.0 / 5040.0 + z2 * ps;
  ps = 1.0 / 120.0 + z2 * ps;
  ps = -1.0 / 6.0 + z2 * ps;
  ps = 1.0 + z2 * ps;
  double S = z * ps;
  double pc = 1.0 / 479001600.0;
  pc = -1.0 / 3628800.0 + z2 * pc;
  pc = 1.0 / 40320.0 + z2 * pc;
  pc = -1.0 / 720.0 + z2 * pc;
  pc = 1.0 / 24.0 + z2 * pc;
  pc = -1.0 / 2.0 + z2 * pc;
  double C = 1.0 + z2 * pc;
  switch (oct) {
    case 0: *cs = C; *sn = S; break;
    case 1: *cs = S; *sn = C; break;
    case 2: *cs = -S; *sn = C; break;
    case 3: *cs = -C; *sn = S; break;
    case 4: *cs = -C; *sn = -S; break;
    case 5: *cs = -S; *sn = -C; break;
    case 6: *cs = S; *sn = -C; break;
    default: *cs = C; *sn = -S; break;
  }
}

/* ------------------------------------------------------------ -ln u -- */

/* -ln u, u in (0, 1]: u = 2^e m with m in [sqrt(1/2), sqrt(2)) (exact, from
 * the bits), ln m = ln(1 + t) with t = m - 1 (exact) by its alternating
 * series t - t^2/2 + ... to 40 terms (|t|^40 / 40 < 2e-17), Horner from the
 * last term; -ln u = -(e ln 2 + ln m). */
static const double kLn2 = 0.6931471805599453094172321;
double boltz_ref_neg_ln(double u) {
  uint64_t bits;
  memcpy(&bits, &u, sizeof(bits));
  int e = (int)((bits >> 52) & 0x7FF) - 1023;
  uint64_t mb = (bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull;
  double m;
  memcpy(&m, &mb, sizeof(m));
  if (m > 1.4142135623730951) {
    m = m * 0.5;
    e += 1;
  }
  double t = m - 1.0;
  double p = 0.0;
  for (int n = 40; n >= 1; --n) {
    const double cn = ((n & 1) ? 1.0 : -1.0) / (double)n;
    p = cn + t * p;
  }
  return -((double)e * kLn2 + t * p);
}

/* --------------------------------------------------------- pair sample -- */

typedef struct {
  int kept;
  int a, b, as, bs;
  double q;
  uint32_t r[4];
  double vel[12]; /* v_a, v_b, v*, v1* (continuous) */
} pair_t;

/* Inverse CDF of the per-axis node law on a 12-bit field f: the number of
 * thresholds <= f. */
static int axis_draw(const boltz_ref_ctx* c, int k, uint32_t f) {
  int idx = 0;
  for (int i = 1; i < c->n[k]; ++i)
    if ((uint64_t)f >= c->T[k][i]) idx++;
  return idx;
}

/* Uniform node law on a 12-bit field: floor(f n / 2^12). */
static int axis_uniform(const boltz_ref_ctx* c, int k, uint32_t f) {
  return (int)(((uint64_t)f * (uint64_t)c->n[k]) >> FIELD_BITS);
}

int boltz_ref_axis_draw(const boltz_ref_ctx* c, int axis, uint32_t f) {
  if (!c || axis < 0 || axis > 2 || f >= (1u << FIELD_BITS)) return -1;
  return axis_draw(c, axis, f);
}

/* Cell of a velocity component, or -1 outside the box: uniform cells by
 * floor((x + a) n / 2a); stretched cells by counting the interior edges at
 * or below x (a component on an edge belongs to the upper cell, as with the
 * floor), outside when x < e_0 or x >= e_n. */
static int axis_cell(const boltz_ref_ctx* c, int k, double x) {
  if (c->stretched) {
    const double* e = c->edge[k];
    const int n = c->n[k];
    if (!(x >= e[0] && x < e[n])) return -1;
    int cnt = 0;
    for (int i = 1; i < n; ++i)
      if (x >= e[i]) cnt++;
    return cnt;
  }
  double t = floor((x + c->a[k]) * c->inv_cell[k]);
  if (!(t >= 0.0 && t < (double)c->n[k])) return -1;
  return (int)t;
}

/* w_a / p~_a for node (i, j, k): the midpoint weight of Phi0 over the
 * probability of drawing the node from the mixture (1 - beta) p_Phi0 + beta
 * p_uniform (Eq. coll8Dim as an importance-sampling estimate). */
static double node_ratio(const boltz_ref_ctx* c, int i, int j, int k) {
  double w = (c->om[0][i] * c->om[1][j]) * c->om[2][k];
  double pm = (c->pphi[0][i] * c->pphi[1][j]) * c->pphi[2][k];
  double pu = (c->punif[0][i] * c->punif[1][j]) * c->punif[2][k];
  return w / ((1.0 - c->beta) * pm + c->beta * pu);
}

/* One Monte Carlo collision sample (Sec. 3, Eqs. coll8Dim / monteCarloInt)
 * from one Philox4x32-10 block r0..r3 with counter (m, group, step, cavity):
 *   r0 = [a_x:12][a_y:12][choice_a:4][choice_b:4]
 *   r1 = [a_z:12][b_x:12][phi_hi:8]    r2 = [b_y:12][b_z:12][phi_lo:8]
 *   r3 = u for k_z.
 * Each node comes from the discrete Maxwellian law (choice >= mix16) or the
 * uniform law (choice < mix16) of its 12-bit fields; k is uniform on the unit
 * sphere, k_z = 2 u - 1 with u = (r3 + 1/2) 2^-32, azimuth 2 pi (phi + 1/2)
 * 2^-16; post-collision velocities v* = v_a + (v_r.k) k, v1* = v_b - (v_r.k) k
 * with v_r = v_b - v_a (the sign of the sampling-kernel listing, which
 * conserves energy); weight q = dt K |v_r.k| (w_a/p~_a)(w_b/p~_b) / N_t, the
 * importance-sampling estimate of Eq. coll8Dim for the mixture density
 * p~ = (1 - beta) p_Maxwell + beta p_uniform.  Pairs whose post-collision
 * velocity leaves the box are discarded (they still count in N_t). */
static void sample_pair_continuous(const boltz_ref_ctx* c, uint32_t group, uint32_t step, uint32_t m,
                                   pair_t* out);

static void sample_pair(const boltz_ref_ctx* c, uint32_t group, uint32_t step, uint32_t m,
                        pair_t* out) {
  if (c->p.flags & BOLTZ_REF_CONTINUOUS) {
    sample_pair_continuous(c, group, step, m, out);
    return;
  }
  const uint32_t key[2] = {(uint32_t)c->p.seed, (uint32_t)(c->p.seed >> 32)};
  const uint32_t ctr[4] = {m, group, step, c->p.cavity_id};
  uint32_t* r = out->r;
  boltz_ref_philox4x32_10(ctr, key, r);
  const uint32_t fa[3] = {r[0] >> 20, (r[0] >> 8) & 0xFFFu, r[1] >> 20};
  const uint32_t fb[3] = {(r[1] >> 8) & 0xFFFu, r[2] >> 20, (r[2] >> 8) & 0xFFFu};
  const int unif_a = (int)((r[0] >> 4) & 15u) < (int)c->p.mix16;
  const int unif_b = (int)(r[0] & 15u) < (int)c->p.mix16;
  int ia[3], ib[3];
  for (int k = 0; k < 3; ++k) {
    ia[k] = unif_a ? axis_uniform(c, k, fa[k]) : axis_draw(c, k, fa[k]);
    ib[k] = unif_b ? axis_uniform(c, k, fb[k]) : axis_draw(c, k, fb[k]);
  }
  const uint32_t phi = ((r[1] & 0xFFu) << 8) | (r[2] & 0xFFu);
  double u6 = ((double)r[3] + 0.5) * 0x1p-32;
  double u7 = ((double)phi + 0.5) * 0x1p-16;
  double kz = 2.0 * u6 - 1.0;
  double s = sqrt((1.0 - kz) * (1.0 + kz));
  double cp, sp;
  boltz_ref_cos_sin_2pi(u7, &cp, &sp);
  double kx = s * cp, ky = s * sp;
  double vax = c->v[0][ia[0]], vay = c->v[1][ia[1]], vaz = c->v[2][ia[2]];
  double vbx = c->v[0][ib[0]], vby = c->v[1][ib[1]], vbz = c->v[2][ib[2]];
  double vrx = vbx - vax, vry = vby - vay, vrz = vbz - vaz;
  double alpha = (vrx * kx + vry * ky) + vrz * kz;
  double ddx = alpha * kx, ddy = alpha * ky, ddz = alpha * kz;
  int sx = axis_cell(c, 0, vax + ddx), sy = axis_cell(c, 1, vay + ddy), sz = axis_cell(c, 2, vaz + ddz);
  int tx = axis_cell(c, 0, vbx - ddx), ty = axis_cell(c, 1, vby - ddy), tz = axis_cell(c, 2, vbz - ddz);
  out->a = node_of(c, ia[0], ia[1], ia[2]);
  out->b = node_of(c, ib[0], ib[1], ib[2]);
  const double vel[12] = {vax, vay, vaz, vbx, vby, vbz, vax + ddx, vay + ddy, vaz + ddz,
                          vbx - ddx, vby - ddy, vbz - ddz};
  memcpy(out->vel, vel, sizeof(vel));
  out->kept = (sx >= 0 && sy >= 0 && sz >= 0 && tx >= 0 && ty >= 0 && tz >= 0);
  if (out->kept) {
    out->as = node_of(c, sx, sy, sz);
    out->bs = node_of(c, tx, ty, tz);
    out->q = ((c->qfac * fabs(alpha)) * node_ratio(c, ia[0], ia[1], ia[2])) *
             node_ratio(c, ib[0], ib[1], ib[2]);
  } else {
    out->as = -1;
    out->bs = -1;
    out->q = 0.0;
  }
}

/* The continuous variant (problem flag BOLTZ_REF_CONTINUOUS; the sampling
 * kernel of Sec. 4 as printed): v and v1 are drawn from the Maxwellian Phi0
 * (each component normal with variance 1/2) by the Box-Muller method, k as
 * above, and every velocity is binned to the cell that contains it.  Two
 * Philox4x32-10 blocks per sample: A with counter (m, group, step, cavity),
 * B with (m, group | 2^31, step, cavity).  With U(w) = (w + 1) 2^-32 (in
 * (0, 1]) for radii and U'(w) = (w + 1/2) 2^-32 for angles:
 *   (v_x, v_y) = sqrt(-ln U(A0)) (cos, sin)(2 pi U'(A1)),
 *   (v_z, v1_x) from (A2, A3), (v1_y, v1_z) from (B0, B1),
 *   k_z = 2 U'(B2) - 1, azimuth 2 pi U'(B3).
 * h is taken in the cells a = cell(v), b = cell(v1); the weight is
 * q = dt K |v_r.k| / N_t (Phi0 is the sampling density itself).  A pair
 * with any of the four velocities outside the box is discarded (it counts
 * in N_t); a and b are then -1 when v or v1 is outside. */
static void sample_pair_continuous(const boltz_ref_ctx* c, uint32_t group, uint32_t step, uint32_t m,
                                   pair_t* out) {
  const uint32_t key[2] = {(uint32_t)c->p.seed, (uint32_t)(c->p.seed >> 32)};
  const uint32_t ca[4] = {m, group, step, c->p.cavity_id};
  const uint32_t cb[4] = {m, group | 0x80000000u, step, c->p.cavity_id};
  uint32_t A[4], B[4];
  boltz_ref_philox4x32_10(ca, key, A);
  boltz_ref_philox4x32_10(cb, key, B);
  memcpy(out->r, A, sizeof(A));
  double nrm[6];
  const uint32_t rad[3] = {A[0], A[2], B[0]}, ang[3] = {A[1], A[3], B[1]};
  for (int i = 0; i < 3; ++i) {
    const double r = sqrt(boltz_ref_neg_ln(((double)rad[i] + 1.0) * 0x1p-32));
    double cs, sn;
    boltz_ref_cos_sin_2pi(((double)ang[i] + 0.5) * 0x1p-32, &cs, &sn);
    nrm[2 * i] = r * cs;
    nrm[2 * i + 1] = r * sn;
  }
  const double vax = nrm[0], vay = nrm[1], vaz = nrm[2], vbx = nrm[3], vby = nrm[4], vbz = nrm[5];
  const double kz = 2.0 * (((double)B[2] + 0.5) * 0x1p-32) - 1.0;
  const double s = sqrt((1.0 - kz) * (1.0 + kz));
  double cp, sp;
  boltz_ref_cos_sin_2pi(((double)B[3] + 0.5) * 0x1p-32, &cp, &sp);
  const double kx = s * cp, ky = s * sp;
  const double vrx = vbx - vax, vry = vby - vay, vrz = vbz - vaz;
  const double alpha = (vrx * kx + vry * ky) + vrz * kz;
  const double ddx = alpha * kx, ddy = alpha * ky, ddz = alpha * kz;
  const int ax = axis_cell(c, 0, vax), ay = axis_cell(c, 1, vay), az = axis_cell(c, 2, vaz);
  const int bx = axis_cell(c, 0, vbx), by = axis_cell(c, 1, vby), bz = axis_cell(c, 2, vbz);
  const int sx = axis_cell(c, 0, vax + ddx), sy = axis_cell(c, 1, vay + ddy), sz = axis_cell(c, 2, vaz + ddz);
  const int tx = axis_cell(c, 0, vbx - ddx), ty = axis_cell(c, 1, vby - ddy), tz = axis_cell(c, 2, vbz - ddz);
  const double vel[12] = {vax, vay, vaz, vbx, vby, vbz, vax + ddx, vay + ddy, vaz + ddz,
                          vbx - ddx, vby - ddy, vbz - ddz};
  memcpy(out->vel, vel, sizeof(vel));
  const int in_a = ax >= 0 && ay >= 0 && az >= 0, in_b = bx >= 0 && by >= 0 && bz >= 0;
  out->a = in_a ? node_of(c, ax, ay, az) : -1;
  out->b = in_b ? node_of(c, bx, by, bz) : -1;
  out->kept = in_a && in_b && sx >= 0 && sy >= 0 && sz >= 0 && tx >= 0 && ty >= 0 && tz >= 0;
  if (out->kept) {
    out->as = node_of(c, sx, sy, sz);
    out->bs = node_of(c, tx, ty, tz);
    out->q = c->qfac * fabs(alpha);
  } else {
    out->as = -1;
    out->bs = -1;
    out->q = 0.0;
  }
}

static uint32_t group_of(const boltz_ref_ctx* c, int64_t cell) {
  return (c->p.sample_group == 0) ? 0u : (uint32_t)(cell / c->p.sample_group);
}

int boltz_ref_debug_pairs(const boltz_ref_ctx* c, int64_t cell, int64_t step, int64_t m0,
                          int64_t count, int32_t* idx4, double* q, uint32_t* words, double* vel) {
  if (!c || cell < 0 || cell >= c->ncells || m0 < 0 || count < 0 ||
      m0 + count > ((int64_t)1 << 31) || !idx4 || !q)
    return BOLTZ_REF_EINVAL;
  uint32_t g = group_of(c, cell);
  for (int64_t i = 0; i < count; ++i) {
    pair_t pr;
    sample_pair(c, g, (uint32_t)step, (uint32_t)(m0 + i), &pr);
    idx4[4 * i + 0] = pr.a;
    idx4[4 * i + 1] = pr.b;
    idx4[4 * i + 2] = pr.as;
    idx4[4 * i + 3] = pr.bs;
    q[i] = pr.q;
    if (words) memcpy(words + 4 * i, pr.r, 4 * sizeof(uint32_t));
    if (vel) memcpy(vel + 12 * i, pr.vel, 12 * sizeof(double));
  }
  return BOLTZ_REF_OK;
}

/* --------------------------------------------------------------- walls -- */

/* Temperature ratio of the face `pos` of a wall (the bottom wall may carry
 * a per-face profile). */
static double wall_tau(const boltz_ref_walls* w, int wall, int pos) {
  switch (wall) {
    case WALL_LEFT: return w->tau_left;
    case WALL_RIGHT: return w->tau_right;
    case WALL_BOTTOM: return w->tau_bottom_x ? w->tau_bottom_x[pos] : w->tau_bottom;
    default: return w->tau_top;
  }
}

/* Phi_w(v) / Phi0(v) for a wall Maxwellian of velocity (U, 0, 0) and
 * temperature ratio tau (Eq. bcMax with the wall Maxwellian). */
static double wall_ratio(double vx, double vy, double vz, double U, double tau) {
  double v2 = (vx * vx + vy * vy) + vz * vz;
  double ux = vx - U;
  double c2 = (ux * ux + vy * vy) + vz * vz;
  return pow(tau, -1.5) * exp(v2 - c2 / tau);
}

/* Wall density n_w of one boundary face from the zero-net-mass-flux
 * condition of Sec. 2, written with discrete sums over the velocity nodes so
 * that the streaming step passes zero net mass through the face:
 *   n_w = sum_{out} |v_n| w_j (1 + eps hhat_j) / sum_{in} |v_n| w_j R_j,
 * R = Phi_w / Phi0.  hhat is the scheme's own gas-side face value (adjacent
 * cell for order 1; the Beam-Warming face value h_a + (1-C)(h_a - h_a')/2 for
 * order 2).  The incoming sum runs over the mirror images of the outgoing
 * nodes in the same order, so a wall at rest facing h = 0 gives n_w = 1
 * exactly. */
static double face_density(const boltz_ref_ctx* c, const double* src, int wall, int pos,
                           const boltz_ref_walls* walls, int order) {
  const int nx = c->p.nx, ny = c->p.ny;
  int nax = (wall == WALL_LEFT || wall == WALL_RIGHT) ? 0 : 1;
  int sgn = (wall == WALL_LEFT || wall == WALL_BOTTOM) ? 1 : -1;
  int ca, cb;
  switch (wall) {
    case WALL_LEFT: ca = pos * nx + 0; cb = pos * nx + 1; break;
    case WALL_RIGHT: ca = pos * nx + nx - 1; cb = pos * nx + nx - 2; break;
    case WALL_BOTTOM: ca = 0 * nx + pos; cb = 1 * nx + pos; break;
    default: ca = (ny - 1) * nx + pos; cb = (ny - 2) * nx + pos; break;
  }
  double dl = (nax == 0) ? c->dx : c->dy;
  double U = (wall == WALL_TOP) ? walls->lid_u : 0.0;
  double tau = wall_tau(walls, wall, pos);
  double phi_out = 0.0, dens = 0.0;
  for (int j = 0; j < c->nv; ++j) {
    int jx, jy, jz;
    node_idx(c, j, &jx, &jy, &jz);
    double vn = (nax == 0) ? c->v[0][jx] : c->v[1][jy];
    if (!(sgn * vn < 0.0)) continue; /* outgoing nodes only */
    double an = fabs(vn);
    double hh = src[(size_t)ca * c->nv + j];
    if (order == 2) {
      double C = an * c->dt / dl;
      hh = hh + 0.5 * (1.0 - C) * (hh - src[(size_t)cb * c->nv + j]);
    }
    double w = node_w(c, jx, jy, jz);
    phi_out += (an * w) * (1.0 + c->p.eps * hh);
    int mx = jx, my = jy;
    if (nax == 0) mx = c->n[0] - 1 - jx; else my = c->n[1] - 1 - jy;
    double R = wall_ratio(c->v[0][mx], c->v[1][my], c->v[2][jz], U, tau);
    dens += (an * node_w(c, mx, my, jz)) * R;
  }
  return phi_out / dens;
}

/* Re-emitted deviation h_w = (n_w Phi_w/Phi0 - 1)/eps (Eq. bcMax) of face
 * `pos` of a wall. */
static double ghost_value(const boltz_ref_ctx* c, int wall, int pos, double nw, int j,
                          const boltz_ref_walls* walls) {
  int jx, jy, jz;
  node_idx(c, j, &jx, &jy, &jz);
  double U = (wall == WALL_TOP) ? walls->lid_u : 0.0;
  double R = wall_ratio(c->v[0][jx], c->v[1][jy], c->v[2][jz], U, wall_tau(walls, wall, pos));
  return (nw * R - 1.0) / c->p.eps;
}

/* ----------------------------------------------------------- streaming -- */

static int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

/* Beam-Warming update of one node along one axis (second-order upwind, flux
 * form with face value h_i + (1-C)(h_i - h_{i-s})/2). */
static double bw_update(double h0, double h1, double h2, double C) {
  return h0 - C * (h0 - h1) - 0.5 * C * (1.0 - C) * ((h0 - 2.0 * h1) + h2);
}

/* x-sweep of order 2 over all rows: hx = BW_x(h), ghosts from the x walls. */
static void sweep_x(const boltz_ref_ctx* c, const double* h, double* hx, const double* nw_left,
                    const double* nw_right, const boltz_ref_walls* walls) {
  const int nx = c->p.nx, ny = c->p.ny, nv = c->nv;
  const int periodic = (c->p.bc == BOLTZ_REF_BC_PERIODIC);
#pragma omp parallel for schedule(static)
  for (int cell = 0; cell < nx * ny; ++cell) {
    int ix = cell % nx, iy = cell / nx;
    for (int j = 0; j < nv; ++j) {
      int jx, jy, jz;
      node_idx(c, j, &jx, &jy, &jz);
      double vx = c->v[0][jx];
      double h0 = h[(size_t)cell * nv + j];
      if (vx == 0.0) {
        hx[(size_t)cell * nv + j] = h0;
        continue;
      }
      int s = vx > 0.0 ? 1 : -1;
      double C = fabs(vx) * c->dt / c->dx;
      double hn[2];
      for (int d = 1; d <= 2; ++d) {
        int i = ix - d * s;
        if (i >= 0 && i < nx) hn[d - 1] = h[((size_t)iy * nx + i) * nv + j];
        else if (periodic) hn[d - 1] = h[((size_t)iy * nx + wrap(i, nx)) * nv + j];
        else if (i < 0) hn[d - 1] = ghost_value(c, WALL_LEFT, iy, nw_left[iy], j, walls);
        else hn[d - 1] = ghost_value(c, WALL_RIGHT, iy, nw_right[iy], j, walls);
      }
      hx[(size_t)cell * nv + j] = bw_update(h0, hn[0], hn[1], C);
    }
  }
}

/* y-sweep of order 2: hs = BW_y(hx), ghosts from the y walls. */
static void sweep_y(const boltz_ref_ctx* c, const double* hx, double* hs, const double* nw_bottom,
                    const double* nw_top, const boltz_ref_walls* walls) {
  const int nx = c->p.nx, ny = c->p.ny, nv = c->nv;
  const int periodic = (c->p.bc == BOLTZ_REF_BC_PERIODIC);
#pragma omp parallel for schedule(static)
  for (int cell = 0; cell < nx * ny; ++cell) {
    int ix = cell % nx, iy = cell / nx;
    for (int j = 0; j < nv; ++j) {
      int jx, jy, jz;
      node_idx(c, j, &jx, &jy, &jz);
      double vy = c->v[1][jy];
      double h0 = hx[(size_t)cell * nv + j];
      if (vy == 0.0) {
        hs[(size_t)cell * nv + j] = h0;
        continue;
      }
      int s = vy > 0.0 ? 1 : -1;
      double C = fabs(vy) * c->dt / c->dy;
      double hn[2];
      for (int d = 1; d <= 2; ++d) {
        int i = iy - d * s;
        if (i >= 0 && i < ny) hn[d - 1] = hx[((size_t)i * nx + ix) * nv + j];
        else if (periodic) hn[d - 1] = hx[((size_t)wrap(i, ny) * nx + ix) * nv + j];
        else if (i < 0) hn[d - 1] = ghost_value(c, WALL_BOTTOM, ix, nw_bottom[ix], j, walls);
        else hn[d - 1] = ghost_value(c, WALL_TOP, ix, nw_top[ix], j, walls);
      }
      hs[(size_t)cell * nv + j] = bw_update(h0, hn[0], hn[1], C);
    }
  }
}

/* First-order unsplit upwind step, Eq. streaming2D with the upwind side
 * chosen by the sign of each velocity component. */
static void stream_order1(const boltz_ref_ctx* c, const double* h, double* hs, const double* nw,
                          const boltz_ref_walls* walls) {
  const int nx = c->p.nx, ny = c->p.ny, nv = c->nv;
  const int periodic = (c->p.bc == BOLTZ_REF_BC_PERIODIC);
  const double* nwl = nw;
  const double* nwr = nw + ny;
  const double* nwb = nw + 2 * ny;
  const double* nwt = nw + 2 * ny + nx;
#pragma omp parallel for schedule(static)
  for (int cell = 0; cell < nx * ny; ++cell) {
    int ix = cell % nx, iy = cell / nx;
    for (int j = 0; j < nv; ++j) {
      int jx, jy, jz;
      node_idx(c, j, &jx, &jy, &jz);
      double vx = c->v[0][jx], vy = c->v[1][jy];
      double h0 = h[(size_t)cell * nv + j];
      /* Courant numbers of this cell: its own lengths (the upwind
       * finite-volume form, conservative on stretched cells) */
      double Cx = fabs(vx) * c->dt / (c->sstretched ? c->wx[ix] : c->dx);
      double Cy = fabs(vy) * c->dt / (c->sstretched ? c->wy[iy] : c->dy);
      double hxn = h0, hyn = h0;
      if (vx != 0.0) {
        int i = ix - (vx > 0.0 ? 1 : -1);
        if (i >= 0 && i < nx) hxn = h[((size_t)iy * nx + i) * nv + j];
        else if (periodic) hxn = h[((size_t)iy * nx + wrap(i, nx)) * nv + j];
        else if (i < 0) hxn = ghost_value(c, WALL_LEFT, iy, nwl[iy], j, walls);
        else hxn = ghost_value(c, WALL_RIGHT, iy, nwr[iy], j, walls);
      }
      if (vy != 0.0) {
        int i = iy - (vy > 0.0 ? 1 : -1);
        if (i >= 0 && i < ny) hyn = h[((size_t)i * nx + ix) * nv + j];
        else if (periodic) hyn = h[((size_t)wrap(i, ny) * nx + ix) * nv + j];
        else if (i < 0) hyn = ghost_value(c, WALL_BOTTOM, ix, nwb[ix], j, walls);
        else hyn = ghost_value(c, WALL_TOP, ix, nwt[ix], j, walls);
      }
      hs[(size_t)cell * nv + j] = ((1.0 - Cx) - Cy) * h0 + Cx * hxn + Cy * hyn;
    }
  }
}

/* n_w of every face exactly as the streaming step uses them; for order 2 the
 * y-wall faces are computed from the x-swept state (passed as hx). */
static void all_wall_densities(const boltz_ref_ctx* c, const double* h, const double* hx,
                               const boltz_ref_walls* walls, double* nw, int which) {
  const int nx = c->p.nx, ny = c->p.ny, order = c->p.order;
  /* which: 1 = x walls, 2 = y walls, 3 = both */
  if (which & 1)
    for (int iy = 0; iy < ny; ++iy) {
      nw[iy] = face_density(c, h, WALL_LEFT, iy, walls, order);
      nw[ny + iy] = face_density(c, h, WALL_RIGHT, iy, walls, order);
    }
  if (which & 2) {
    const double* src = (order == 2) ? hx : h;
    for (int ix = 0; ix < nx; ++ix) {
      nw[2 * ny + ix] = face_density(c, src, WALL_BOTTOM, ix, walls, order);
      nw[2 * ny + nx + ix] = face_density(c, src, WALL_TOP, ix, walls, order);
    }
  }
}

int boltz_ref_wall_density(const boltz_ref_ctx* c, const double* h, const boltz_ref_walls* walls,
                           double* nw) {
  if (!c || !h || !walls || !nw || c->p.bc != BOLTZ_REF_BC_CAVITY) return BOLTZ_REF_EINVAL;
  const int nx = c->p.nx, ny = c->p.ny;
  all_wall_densities(c, h, NULL, walls, nw, 1);
  if (c->p.order == 2) {
    double* hx = (double*)malloc(sizeof(double) * (size_t)c->ncells * c->nv);
    if (!hx) return BOLTZ_REF_ENOMEM;
    sweep_x(c, h, hx, nw, nw + ny, walls);
    all_wall_densities(c, h, hx, walls, nw, 2);
    free(hx);
  } else {
    all_wall_densities(c, h, NULL, walls, nw, 2);
  }
  (void)nx;
  return BOLTZ_REF_OK;
}

int boltz_ref_stream(const boltz_ref_ctx* c, const double* h_in, double* h_out,
                     const boltz_ref_walls* walls) {
  if (!c || !h_in || !h_out || h_in == h_out) return BOLTZ_REF_EINVAL;
  const int cavity = (c->p.bc == BOLTZ_REF_BC_CAVITY);
  if (cavity && !walls) return BOLTZ_REF_EINVAL;
  const int nx = c->p.nx, ny = c->p.ny;
  double* nw = (double*)calloc((size_t)2 * (nx + ny), sizeof(double));
  if (!nw) return BOLTZ_REF_ENOMEM;
  if (c->p.order == 1) {
    if (cavity) all_wall_densities(c, h_in, NULL, walls, nw, 3);
    stream_order1(c, h_in, h_out, nw, walls);
  } else {
    double* hx = (double*)malloc(sizeof(double) * (size_t)c->ncells * c->nv);
    if (!hx) {
      free(nw);
      return BOLTZ_REF_ENOMEM;
    }
    if (cavity) all_wall_densities(c, h_in, NULL, walls, nw, 1);
    sweep_x(c, h_in, hx, nw, nw + ny, walls);
    if (cavity) all_wall_densities(c, h_in, hx, walls, nw, 2);
    sweep_y(c, hx, h_out, nw + 2 * ny, nw + 2 * ny + nx, walls);
    free(hx);
  }
  free(nw);
  return BOLTZ_REF_OK;
}

/* ----------------------------------------------------------- collision -- */

/* Cholesky solve of the 5x5 symmetric positive definite system M x = r. */
static int solve5(double M[5][5], const double r[5], double x[5]) {
  double L[5][5] = {{0}};
  for (int i = 0; i < 5; ++i) {
    for (int j = 0; j <= i; ++j) {
      double s = M[i][j];
      for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
      if (i == j) {
        if (!(s > 0.0)) return -1;
        L[i][i] = sqrt(s);
      } else {
        L[i][j] = s / L[j][j];
      }
    }
  }
  double y[5];
  for (int i = 0; i < 5; ++i) {
    double s = r[i];
    for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
    y[i] = s / L[i][i];
  }
  for (int i = 4; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < 5; ++k) s -= L[k][i] * x[k];
    x[i] = s / L[i][i];
  }
  return 0;
}

/* Collision of one cell: hs (copy of the cell's post-stream h), work
 * arrays dn, hc of nv doubles; writes the cell's output to ho. */
static int collide_cell(const boltz_ref_ctx* c, int64_t cell, int64_t step, uint32_t flags,
                        const double* hs, double* dn, double* hc, double* ho, double* dN_out,
                        double* defect) {
  const int nv = c->nv;
  const double eps = c->p.eps;
  const int64_t nt = c->p.n_pairs;
  int status = BOLTZ_REF_OK;
  memset(dn, 0, sizeof(double) * nv);
  uint32_t g = group_of(c, cell);
  if (c->p.flags & BOLTZ_REF_SEQUENTIAL) {
    /* Alg. 3: the samples update h in place in the order m = 0, 1, ...;
     * each reads the current h at its nodes a and b, then adds its four
     * increments, at a*, b*, a and b in this order, each to the current
     * value (where two of the nodes coincide both increments land). */
    memcpy(hc, hs, sizeof(double) * nv);
    for (int64_t m = 0; m < nt; ++m) {
      pair_t pr;
      sample_pair(c, g, (uint32_t)step, (uint32_t)m, &pr);
      if (!pr.kept) continue;
      double ha = hc[pr.a], hb = hc[pr.b];
      double gg = (ha + hb) + (eps * ha) * hb;
      double qg = pr.q * gg;
      hc[pr.as] += qg / node_w_flat(c, pr.as);
      hc[pr.bs] += qg / node_w_flat(c, pr.bs);
      hc[pr.a] -= qg / node_w_flat(c, pr.a);
      hc[pr.b] -= qg / node_w_flat(c, pr.b);
    }
    /* the change of the number of particles per node, as in the Jacobi
     * form: Delta N_j = dV_j Phi0_j (h^c_j - h^s_j) */
    for (int j = 0; j < nv; ++j) dn[j] = node_w_flat(c, j) * (hc[j] - hs[j]);
  } else {
    /* Eq. monteCarloInt evaluated at the post-stream h (Eq. collision_step):
     * every sample reads the same h (Jacobi form). */
    for (int64_t m = 0; m < nt; ++m) {
      pair_t pr;
      sample_pair(c, g, (uint32_t)step, (uint32_t)m, &pr);
      if (!pr.kept) continue;
      double ha = hs[pr.a], hb = hs[pr.b];
      double gg = (ha + hb) + (eps * ha) * hb;
      double qg = pr.q * gg;
      dn[pr.as] += qg;
      dn[pr.bs] += qg;
      dn[pr.a] -= qg;
      dn[pr.b] -= qg;
    }
    /* Eq. collision_step: h^c_j = h^s_j + Delta N_j / (dV_j Phi0_j) */
    for (int j = 0; j < nv; ++j) hc[j] = hs[j] + dn[j] / node_w_flat(c, j);
  }
  if (flags & BOLTZ_REF_NO_CORRECTION) {
    memcpy(ho, hc, sizeof(double) * nv);
  } else {
    /* Eqs. rinorm_a / correzione: F^{n+1} = F^c (1 + A + B.v + C v^2)
     * with the moments of psi = (1, v, v^2) of F^{n+1} equal to those of
     * the post-stream F^s.  Linear system M x = r,
     *   M_kl = sum_j w_j F^c_j psi_k psi_l,
     *   r_k  = sum_j w_j psi_k (F^s_j - F^c_j) = -eps sum_j psi_k dN_j. */
    double M[5][5] = {{0}}, rr[5] = {0}, x[5];
    for (int j = 0; j < nv; ++j) {
      int jx, jy, jz;
      node_idx(c, j, &jx, &jy, &jz);
      double vx = c->v[0][jx], vy = c->v[1][jy], vz = c->v[2][jz];
      double psi[5] = {1.0, vx, vy, vz, (vx * vx + vy * vy) + vz * vz};
      double wF = node_w(c, jx, jy, jz) * (1.0 + eps * hc[j]);
      for (int k = 0; k < 5; ++k) {
        for (int l = 0; l < 5; ++l) M[k][l] += wF * psi[k] * psi[l];
        rr[k] += -eps * psi[k] * dn[j];
      }
    }
    if (solve5(M, rr, x) != 0) {
      status = BOLTZ_REF_ENUMERIC;
      for (int k = 0; k < 5; ++k) x[k] = 0.0;
    }
    for (int j = 0; j < nv; ++j) {
      int jx, jy, jz;
      node_idx(c, j, &jx, &jy, &jz);
      double vx = c->v[0][jx], vy = c->v[1][jy], vz = c->v[2][jz];
      double xpsi = x[0] + x[1] * vx + x[2] * vy + x[3] * vz + x[4] * ((vx * vx + vy * vy) + vz * vz);
      ho[j] = hc[j] + (1.0 + eps * hc[j]) * xpsi / eps;
    }
  }
  if (dN_out) memcpy(dN_out, dn, sizeof(double) * nv);
  if (defect) {
    double d[5] = {0};
    for (int j = 0; j < nv; ++j) {
      int jx, jy, jz;
      node_idx(c, j, &jx, &jy, &jz);
      double vx = c->v[0][jx], vy = c->v[1][jy], vz = c->v[2][jz];
      double psi[5] = {1.0, vx, vy, vz, (vx * vx + vy * vy) + vz * vz};
      double diff = eps * (ho[j] - hs[j]) * node_w(c, jx, jy, jz);
      for (int k = 0; k < 5; ++k) d[k] += psi[k] * diff;
    }
    memcpy(defect, d, sizeof(d));
  }
  return status;
}

/* cells == NULL: all cells of full arrays; otherwise the listed cells, with
 * h_s / h_out holding only those cells (count * nv, compact). */
static int collide_list(const boltz_ref_ctx* c, const double* h_s, double* h_out, int64_t step,
                        uint32_t flags, const int64_t* cells, int64_t count, double* dN_out,
                        double* defect) {
  const int nv = c->nv;
  int status = BOLTZ_REF_OK;
#pragma omp parallel
  {
    double* hs = (double*)malloc(sizeof(double) * nv);
    double* dn = (double*)malloc(sizeof(double) * nv);
    double* hc = (double*)malloc(sizeof(double) * nv);
#pragma omp for schedule(dynamic, 1)
    for (int64_t i = 0; i < count; ++i) {
      int64_t cell = cells ? cells[i] : i;
      memcpy(hs, h_s + (size_t)i * nv, sizeof(double) * nv);
      int st = collide_cell(c, cell, step, flags, hs, dn, hc, h_out + (size_t)i * nv,
                            dN_out ? dN_out + (size_t)cell * nv : NULL,
                            defect ? defect + (size_t)cell * 5 : NULL);
      if (st != BOLTZ_REF_OK) {
#pragma omp atomic write
        status = st;
      }
    }
    free(hs);
    free(dn);
    free(hc);
  }
  return status;
}

int boltz_ref_collide(const boltz_ref_ctx* c, const double* h_s, double* h_out, int64_t step,
                      uint32_t flags, double* dN_out, double* defect) {
  if (!c || !h_s || !h_out) return BOLTZ_REF_EINVAL;
  return collide_list(c, h_s, h_out, step, flags, NULL, c->ncells, dN_out, defect);
}

int boltz_ref_collide_cells(const boltz_ref_ctx* c, const double* h_s, double* h_out, int64_t step,
                            uint32_t flags, const int64_t* cells, int64_t count) {
  if (!c || !h_s || !h_out || !cells || count < 0) return BOLTZ_REF_EINVAL;
  for (int64_t i = 0; i < count; ++i)
    if (cells[i] < 0 || cells[i] >= c->ncells) return BOLTZ_REF_EINVAL;
  return collide_list(c, h_s, h_out, step, flags, cells, count, NULL, NULL);
}

/* ------------------------------------------------------------- moments -- */

int boltz_ref_moments(const boltz_ref_ctx* c, const double* h, const boltz_ref_walls* walls,
                      double* mom, double* lid_shear) {
  if (!c || !h || !mom) return BOLTZ_REF_EINVAL;
  const int nv = c->nv;
  const double eps = c->p.eps;
#pragma omp parallel for schedule(static)
  for (int cell = 0; cell < c->ncells; ++cell) {
    /* midpoint sums of Eqs. densita..sforzi */
    double rho = 0, U[3] = {0, 0, 0}, E = 0, P[6] = {0, 0, 0, 0, 0, 0};
    for (int j = 0; j < nv; ++j) {
      int jx, jy, jz;
      node_idx(c, j, &jx, &jy, &jz);
      double v[3] = {c->v[0][jx], c->v[1][jy], c->v[2][jz]};
      double wh = node_w(c, jx, jy, jz) * h[(size_t)cell * nv + j];
      rho += wh;
      for (int k = 0; k < 3; ++k) U[k] += wh * v[k];
      E += wh * ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
      P[0] += wh * v[0] * v[0];
      P[1] += wh * v[0] * v[1];
      P[2] += wh * v[0] * v[2];
      P[3] += wh * v[1] * v[1];
      P[4] += wh * v[1] * v[2];
      P[5] += wh * v[2] * v[2];
    }
    /* In units of V0 = sqrt(2 R T0): n/n0 = 1 + eps rho, u = U/(1 + eps rho),
     * theta = ((2/3) E - rho)/(1 + eps rho) - (2/3) eps |u|^2,
     * Pi_ij = 2 P_ij - 2 eps (1 + eps rho) u_i u_j. */
    double n = 1.0 + eps * rho;
    double u[3] = {U[0] / n, U[1] / n, U[2] / n};
    double uu = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
    double* o = mom + (size_t)cell * 11;
    o[0] = rho;
    o[1] = u[0];
    o[2] = u[1];
    o[3] = u[2];
    o[4] = ((2.0 / 3.0) * E - rho) / n - (2.0 / 3.0) * eps * uu;
    const int pi_k[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    for (int k = 0; k < 6; ++k) o[5 + k] = 2.0 * P[k] - 2.0 * eps * n * u[pi_k[k][0]] * u[pi_k[k][1]];
  }
  if (lid_shear) {
    if (c->p.bc != BOLTZ_REF_BC_CAVITY || !walls) return BOLTZ_REF_EINVAL;
    /* Lid shear D: the x-y stress on the lid face, built from the gas-side
     * values of the top cells (v_y > 0) and the wall emission (v_y < 0, with
     * n_w from the first-order face values); D = -(1/nx) sum Pi_xy so that
     * D > 0 for a lid moving in +x. */
    const int nx = c->p.nx, ny = c->p.ny;
    double total = 0.0;
    for (int ix = 0; ix < nx; ++ix) {
      int cell = (ny - 1) * nx + ix;
      double nw = face_density(c, h, WALL_TOP, ix, walls, 1);
      double pxy = 0.0;
      for (int j = 0; j < nv; ++j) {
        int jx, jy, jz;
        node_idx(c, j, &jx, &jy, &jz);
        double vx = c->v[0][jx], vy = c->v[1][jy];
        double hh = (vy > 0.0) ? h[(size_t)cell * nv + j]
                               : (vy < 0.0 ? ghost_value(c, WALL_TOP, ix, nw, j, walls) : 0.0);
        pxy += node_w(c, jx, jy, jz) * vx * vy * hh;
      }
      /* stretched cells: the faces weighted by their lengths (the mean
       * over the lid) */
      total += c->sstretched ? c->wx[ix] * (2.0 * pxy) : 2.0 * pxy;
    }
    *lid_shear = c->sstretched ? -total : -total / nx;
  }
  return BOLTZ_REF_OK;
}

/* ------------------------------------------------------------- adjoint -- */
/* Reverse-mode derivatives of the discrete step above (the paper has no
 * adjoint: every function below is the transpose of the linearisation of
 * the forward function it names, taken piece by piece).  Wall parameters
 * theta are indexed in grad[] as
 *   0 lid_u, 1 tau_left, 2 tau_right, 3 tau_top, 4 + ix: tau of bottom face ix
 * (for a uniform bottom wall the sum of the last nx entries is the
 * derivative with respect to tau_bottom).  Pinned against centred finite
 * differences of the forward functions (tests/test_oracle_adjoint.py). */

enum { GRAD_LID_U = 0, GRAD_TAU_LEFT = 1, GRAD_TAU_RIGHT = 2, GRAD_TAU_TOP = 3, GRAD_TAU_BOTTOM0 = 4 };

static int tau_index(int wall, int pos) {
  switch (wall) {
    case WALL_LEFT: return GRAD_TAU_LEFT;
    case WALL_RIGHT: return GRAD_TAU_RIGHT;
    case WALL_BOTTOM: return GRAD_TAU_BOTTOM0 + pos;
    default: return GRAD_TAU_TOP;
  }
}

/* dR/dU and dR/dtau of R = tau^-3/2 exp(|v|^2 - |v - U e_x|^2 / tau). */
static void wall_ratio_grad(double vx, double vy, double vz, double U, double tau, double* dU,
                            double* dtau) {
  double R = wall_ratio(vx, vy, vz, U, tau);
  double ux = vx - U;
  double c2 = (ux * ux + vy * vy) + vz * vz;
  *dU = R * 2.0 * ux / tau;
  *dtau = R * (c2 / (tau * tau) - 1.5 / tau);
}

/* Adjoint of ghost_value: lam is the adjoint of h_w = (n_w R_j - 1)/eps of
 * node j at face (wall, pos).  Adds the wall-parameter part to grad and
 * returns the adjoint of n_w. */
static double ghost_value_adj(const boltz_ref_ctx* c, int wall, int pos, double nw, int j,
                              const boltz_ref_walls* walls, double lam, double* grad) {
  int jx, jy, jz;
  node_idx(c, j, &jx, &jy, &jz);
  double U = (wall == WALL_TOP) ? walls->lid_u : 0.0;
  double tau = wall_tau(walls, wall, pos);
  double vx = c->v[0][jx], vy = c->v[1][jy], vz = c->v[2][jz];
  double R = wall_ratio(vx, vy, vz, U, tau);
  double dU, dtau;
  wall_ratio_grad(vx, vy, vz, U, tau, &dU, &dtau);
  if (grad) {
    if (wall == WALL_TOP) grad[GRAD_LID_U] += lam * nw * dU / c->p.eps;
    grad[tau_index(wall, pos)] += lam * nw * dtau / c->p.eps;
  }
  return lam * R / c->p.eps;
}

/* Adjoint of face_density: lam_nw is the adjoint of n_w of face (wall, pos)
 * computed from src; adds the adjoint of src to lam_src and the
 * wall-parameter part to grad. */
static void face_density_adj(const boltz_ref_ctx* c, const double* src, int wall, int pos,
                             const boltz_ref_walls* walls, int order, double lam_nw, double* lam_src,
                             double* grad) {
  const int nx = c->p.nx, ny = c->p.ny, nv = c->nv;
  int nax = (wall == WALL_LEFT || wall == WALL_RIGHT) ? 0 : 1;
  int sgn = (wall == WALL_LEFT || wall == WALL_BOTTOM) ? 1 : -1;
  int ca, cb;
  switch (wall) {
    case WALL_LEFT: ca = pos * nx + 0; cb = pos * nx + 1; break;
    case WALL_RIGHT: ca = pos * nx + nx - 1; cb = pos * nx + nx - 2; break;
    case WALL_BOTTOM: ca = 0 * nx + pos; cb = 1 * nx + pos; break;
    default: ca = (ny - 1) * nx + pos; cb = (ny - 2) * nx + pos; break;
  }
  double dl = (nax == 0) ? c->dx : c->dy;
  double U = (wall == WALL_TOP) ? walls->lid_u : 0.0;
  double tau = wall_tau(walls, wall, pos);
  /* forward sums: n_w = phi_out / dens */
  double phi_out = 0.0, dens = 0.0;
  for (int j = 0; j < nv; ++j) {
    int jx, jy, jz;
    node_idx(c, j, &jx, &jy, &jz);
    double vn = (nax == 0) ? c->v[0][jx] : c->v[1][jy];
    if (!(sgn * vn < 0.0)) continue;
    double an = fabs(vn);
    double hh = src[(size_t)ca * nv + j];
    if (order == 2) {
      double C = an * c->dt / dl;
      hh = hh + 0.5 * (1.0 - C) * (hh - src[(size_t)cb * nv + j]);
    }
    phi_out += (an * node_w(c, jx, jy, jz)) * (1.0 + c->p.eps * hh);
    int mx = jx, my = jy;
    if (nax == 0) mx = c->n[0] - 1 - jx; else my = c->n[1] - 1 - jy;
    dens += (an * node_w(c, mx, my, jz)) * wall_ratio(c->v[0][mx], c->v[1][my], c->v[2][jz], U, tau);
  }
  double nw = phi_out / dens;
  for (int j = 0; j < nv; ++j) {
    int jx, jy, jz;
    node_idx(c, j, &jx, &jy, &jz);
    double vn = (nax == 0) ? c->v[0][jx] : c->v[1][jy];
    if (!(sgn * vn < 0.0)) continue;
    double an = fabs(vn);
    /* d n_w / d hhat_j = eps |v_n| w_j / dens */
    double lam_hh = lam_nw * c->p.eps * an * node_w(c, jx, jy, jz) / dens;
    if (order == 2) {
      double C = an * c->dt / dl;
      lam_src[(size_t)ca * nv + j] += lam_hh * (1.0 + 0.5 * (1.0 - C));
      lam_src[(size_t)cb * nv + j] -= lam_hh * 0.5 * (1.0 - C);
    } else {
      lam_src[(size_t)ca * nv + j] += lam_hh;
    }
    if (grad) {
      /* d n_w / d R_m = -n_w |v_n| w_m / dens at the mirror node m */
      int mx = jx, my = jy;
      if (nax == 0) mx = c->n[0] - 1 - jx; else my = c->n[1] - 1 - jy;
      double lam_R = -lam_nw * nw * an * node_w(c, mx, my, jz) / dens;
      double dU, dtau;
      wall_ratio_grad(c->v[0][mx], c->v[1][my], c->v[2][jz], U, tau, &dU, &dtau);
      if (wall == WALL_TOP) grad[GRAD_LID_U] += lam_R * dU;
      grad[tau_index(wall, pos)] += lam_R * dtau;
    }
  }
}

/* Coefficients of the Beam-Warming update: bw_update(h0, h1, h2, C) =
 * a0 h0 + a1 h1 + a2 h2. */
static void bw_coefs(double C, double* a) {
  double c2 = 0.5 * C * (1.0 - C);
  a[0] = (1.0 - C) - c2;
  a[1] = C + 2.0 * c2;
  a[2] = -c2;
}

/* Adjoint of one order-2 sweep along axis `ax` (0: x, 1: y): lam_out is the
 * adjoint of out = BW_ax(in); adds the adjoint of `in` to lam_in and that of
 * the face densities of the walls crossed to lam_nw (face order of
 * boltz_ref_wall_density); wall-parameter parts go to grad. */
static void sweep_adj(const boltz_ref_ctx* c, int ax, const double* lam_out, double* lam_in,
                      const double* nw, double* lam_nw, const boltz_ref_walls* walls, double* grad) {
  const int nx = c->p.nx, ny = c->p.ny, nv = c->nv;
  const int periodic = (c->p.bc == BOLTZ_REF_BC_PERIODIC);
  for (int cell = 0; cell < nx * ny; ++cell) {
    int ix = cell % nx, iy = cell / nx;
    for (int j = 0; j < nv; ++j) {
      int jx, jy, jz;
      node_idx(c, j, &jx, &jy, &jz);
      double v = (ax == 0) ? c->v[0][jx] : c->v[1][jy];
      double lam = lam_out[(size_t)cell * nv + j];
      if (v == 0.0) {
        lam_in[(size_t)cell * nv + j] += lam;
        continue;
      }
      int s = v > 0.0 ? 1 : -1;
      double a[3];
      bw_coefs(fabs(v) * c->dt / ((ax == 0) ? c->dx : c->dy), a);
      lam_in[(size_t)cell * nv + j] += a[0] * lam;
      for (int d = 1; d <= 2; ++d) {
        int i = ((ax == 0) ? ix : iy) - d * s, n = (ax == 0) ? nx : ny;
        double l = a[d] * lam;
        if (i >= 0 && i < n) {
          int nb = (ax == 0) ? iy * nx + i : i * nx + ix;
          lam_in[(size_t)nb * nv + j] += l;
        } else if (periodic) {
          int nb = (ax == 0) ? iy * nx + wrap(i, nx) : wrap(i, ny) * nx + ix;
          lam_in[(size_t)nb * nv + j] += l;
        } else {
          int wall, pos, f;
          if (ax == 0) {
            wall = i < 0 ? WALL_LEFT : WALL_RIGHT;
            pos = iy;
            f = (wall == WALL_LEFT ? 0 : ny) + iy;
          } else {
            wall = i < 0 ? WALL_BOTTOM : WALL_TOP;
            pos = ix;
            f = 2 * ny + (wall == WALL_BOTTOM ? 0 : nx) + ix;
          }
          lam_nw[f] += ghost_value_adj(c, wall, pos, nw[f], j, walls, l, grad);
        }
      }
    }
  }
}

/* Adjoint of the first-order unsplit step (stream_order1). */
static void order1_adj(const boltz_ref_ctx* c, const double* lam_out, double* lam_in, const double* nw,
                       double* lam_nw, const boltz_ref_walls* walls, double* grad) {
  const int nx = c->p.nx, ny = c->p.ny, nv = c->nv;
  const int periodic = (c->p.bc == BOLTZ_REF_BC_PERIODIC);
  for (int cell = 0; cell < nx * ny; ++cell) {
    int ix = cell % nx, iy = cell / nx;
    for (int j = 0; j < nv; ++j) {
      int jx, jy, jz;
      node_idx(c, j, &jx, &jy, &jz);
      double vx = c->v[0][jx], vy = c->v[1][jy];
      double Cx = fabs(vx) * c->dt / c->dx, Cy = fabs(vy) * c->dt / c->dy;
      double lam = lam_out[(size_t)cell * nv + j];
      lam_in[(size_t)cell * nv + j] += ((1.0 - Cx) - Cy) * lam;
      for (int ax = 0; ax < 2; ++ax) {
        double v = ax == 0 ? vx : vy;
        if (v == 0.0) continue;
        double l = (ax == 0 ? Cx : Cy) * lam;
        int n = ax == 0 ? nx : ny;
        int i = (ax == 0 ? ix : iy) - (v > 0.0 ? 1 : -1);
        if (i >= 0 && i < n) {
          int nb = ax == 0 ? iy * nx + i : i * nx + ix;
          lam_in[(size_t)nb * nv + j] += l;
        } else if (periodic) {
          int nb = ax == 0 ? iy * nx + wrap(i, nx) : wrap(i, ny) * nx + ix;
          lam_in[(size_t)nb * nv + j] += l;
        } else {
          int wall, pos, f;
          if (ax == 0) {
            wall = i < 0 ? WALL_LEFT : WALL_RIGHT;
            pos = iy;
            f = (wall == WALL_LEFT ? 0 : ny) + iy;
          } else {
            wall = i < 0 ? WALL_BOTTOM : WALL_TOP;
            pos = ix;
            f = 2 * ny + (wall == WALL_BOTTOM ? 0 : nx) + ix;
          }
          lam_nw[f] += ghost_value_adj(c, wall, pos, nw[f], j, walls, l, grad);
        }
      }
    }
  }
}

int boltz_ref_stream_adjoint(const boltz_ref_ctx* c, const double* h_in, const double* lam_out,
                             double* lam_in, double* grad, const boltz_ref_walls* walls) {
  if (!c || !h_in || !lam_out || !lam_in) return BOLTZ_REF_EINVAL;
  /* the adjoint follows uniform spatial cells only */
  if (c->sstretched) return BOLTZ_REF_EINVAL;
  const int cavity = (c->p.bc == BOLTZ_REF_BC_CAVITY);
  if (cavity && !walls) return BOLTZ_REF_EINVAL;
  const int nx = c->p.nx, ny = c->p.ny;
  const size_t n = (size_t)c->ncells * c->nv;
  const int nf = 2 * (nx + ny);
  double* nw = (double*)calloc((size_t)nf, sizeof(double));
  double* lam_nw = (double*)calloc((size_t)nf, sizeof(double));
  double* hx = (double*)malloc(sizeof(double) * n);
  double* lam_hx = (double*)calloc(n, sizeof(double));
  if (!nw || !lam_nw || !hx || !lam_hx) {
    free(nw); free(lam_nw); free(hx); free(lam_hx);
    return BOLTZ_REF_ENOMEM;
  }
  memset(lam_in, 0, sizeof(double) * n);
  if (c->p.order == 1) {
    if (cavity) all_wall_densities(c, h_in, NULL, walls, nw, 3);
    order1_adj(c, lam_out, lam_in, nw, lam_nw, walls, grad);
    if (cavity) {
      for (int iy = 0; iy < ny; ++iy) {
        face_density_adj(c, h_in, WALL_LEFT, iy, walls, 1, lam_nw[iy], lam_in, grad);
        face_density_adj(c, h_in, WALL_RIGHT, iy, walls, 1, lam_nw[ny + iy], lam_in, grad);
      }
      for (int ix = 0; ix < nx; ++ix) {
        face_density_adj(c, h_in, WALL_BOTTOM, ix, walls, 1, lam_nw[2 * ny + ix], lam_in, grad);
        face_density_adj(c, h_in, WALL_TOP, ix, walls, 1, lam_nw[2 * ny + nx + ix], lam_in, grad);
      }
    }
  } else {
    /* forward intermediates: x faces from h, the x-swept state, y faces */
    if (cavity) all_wall_densities(c, h_in, NULL, walls, nw, 1);
    sweep_x(c, h_in, hx, nw, nw + ny, walls);
    if (cavity) all_wall_densities(c, h_in, hx, walls, nw, 2);
    /* y sweep, then the y faces (which read the x-swept state) */
    sweep_adj(c, 1, lam_out, lam_hx, nw, lam_nw, walls, grad);
    if (cavity)
      for (int ix = 0; ix < nx; ++ix) {
        face_density_adj(c, hx, WALL_BOTTOM, ix, walls, 2, lam_nw[2 * ny + ix], lam_hx, grad);
        face_density_adj(c, hx, WALL_TOP, ix, walls, 2, lam_nw[2 * ny + nx + ix], lam_hx, grad);
      }
    /* x sweep, then the x faces */
    sweep_adj(c, 0, lam_hx, lam_in, nw, lam_nw, walls, grad);
    if (cavity)
      for (int iy = 0; iy < ny; ++iy) {
        face_density_adj(c, h_in, WALL_LEFT, iy, walls, 2, lam_nw[iy], lam_in, grad);
        face_density_adj(c, h_in, WALL_RIGHT, iy, walls, 2, lam_nw[ny + iy], lam_in, grad);
      }
  }
  free(nw); free(lam_nw); free(hx); free(lam_hx);
  return BOLTZ_REF_OK;
}

/* Adjoint of the collision of one cell (see collide_cell): lam_o is the
 * adjoint of the cell's output, lam_hs receives that of its post-stream h. */
static void collide_cell_adj(const boltz_ref_ctx* c, int64_t cell, int64_t step, uint32_t flags,
                             const double* hs, const double* lam_o, double* lam_hs, double* dn,
                             double* hc, double* lam_dn) {
  const int nv = c->nv;
  const double eps = c->p.eps;
  const int64_t nt = c->p.n_pairs;
  uint32_t g = group_of(c, cell);
  /* forward: Monte Carlo increments and h^c */
  memset(dn, 0, sizeof(double) * nv);
  for (int64_t m = 0; m < nt; ++m) {
    pair_t pr;
    sample_pair(c, g, (uint32_t)step, (uint32_t)m, &pr);
    if (!pr.kept) continue;
    double ha = hs[pr.a], hb = hs[pr.b];
    double qg = pr.q * ((ha + hb) + (eps * ha) * hb);
    dn[pr.as] += qg;
    dn[pr.bs] += qg;
    dn[pr.a] -= qg;
    dn[pr.b] -= qg;
  }
  for (int j = 0; j < nv; ++j) {
    int jx, jy, jz;
    node_idx(c, j, &jx, &jy, &jz);
    hc[j] = hs[j] + dn[j] / node_w(c, jx, jy, jz);
  }
  /* forward correction: M x = r; adjoint: y = M^-1 z with z = dJ/dx */
  double x[5] = {0, 0, 0, 0, 0}, y[5] = {0, 0, 0, 0, 0};
  int corrected = 0;
  if (!(flags & BOLTZ_REF_NO_CORRECTION)) {
    double M[5][5] = {{0}}, rr[5] = {0}, z[5] = {0};
    for (int j = 0; j < nv; ++j) {
      int jx, jy, jz;
      node_idx(c, j, &jx, &jy, &jz);
      double vx = c->v[0][jx], vy = c->v[1][jy], vz = c->v[2][jz];
      double psi[5] = {1.0, vx, vy, vz, (vx * vx + vy * vy) + vz * vz};
      double wF = node_w(c, jx, jy, jz) * (1.0 + eps * hc[j]);
      for (int k = 0; k < 5; ++k) {
        for (int l = 0; l < 5; ++l) M[k][l] += wF * psi[k] * psi[l];
        rr[k] += -eps * psi[k] * dn[j];
        /* h_out = h^c + (1 + eps h^c)(x . psi)/eps: dJ/dx_k */
        z[k] += lam_o[j] * (1.0 + eps * hc[j]) * psi[k] / eps;
      }
    }
    if (solve5(M, rr, x) == 0 && solve5(M, z, y) == 0) corrected = 1;
    else for (int k = 0; k < 5; ++k) x[k] = y[k] = 0.0;
  }
  for (int j = 0; j < nv; ++j) {
    int jx, jy, jz;
    node_idx(c, j, &jx, &jy, &jz);
    double w = node_w(c, jx, jy, jz);
    double lam_hc = lam_o[j];
    lam_dn[j] = 0.0;
    if (corrected) {
      double vx = c->v[0][jx], vy = c->v[1][jy], vz = c->v[2][jz];
      double psi[5] = {1.0, vx, vy, vz, (vx * vx + vy * vy) + vz * vz};
      double xpsi = 0.0, ypsi = 0.0;
      for (int k = 0; k < 5; ++k) {
        xpsi += x[k] * psi[k];
        ypsi += y[k] * psi[k];
      }
      /* direct term, and M_kl = sum w (1 + eps h^c) psi_k psi_l (dJ/dM = -y x^T) */
      lam_hc = lam_o[j] * (1.0 + xpsi) - eps * w * ypsi * xpsi;
      /* r_k = -eps sum psi_k dN_j */
      lam_dn[j] = -eps * ypsi;
    }
    /* h^c = h^s + dN / w */
    lam_hs[j] = lam_hc;
    lam_dn[j] += lam_hc / w;
  }
  /* Monte Carlo increments: dN_t += +-q g(h_a, h_b) */
  for (int64_t m = 0; m < nt; ++m) {
    pair_t pr;
    sample_pair(c, g, (uint32_t)step, (uint32_t)m, &pr);
    if (!pr.kept) continue;
    double G = pr.q * ((lam_dn[pr.as] + lam_dn[pr.bs]) - (lam_dn[pr.a] + lam_dn[pr.b]));
    lam_hs[pr.a] += G * (1.0 + eps * hs[pr.b]);
    lam_hs[pr.b] += G * (1.0 + eps * hs[pr.a]);
  }
}

int boltz_ref_collide_adjoint(const boltz_ref_ctx* c, const double* h_s, const double* lam_out,
                              double* lam_s, int64_t step, uint32_t flags) {
  if (!c || !h_s || !lam_out || !lam_s) return BOLTZ_REF_EINVAL;
  /* the adjoint follows the Jacobi form of Eq. collision_step only */
  if (c->p.flags & BOLTZ_REF_SEQUENTIAL) return BOLTZ_REF_EINVAL;
  const int nv = c->nv;
#pragma omp parallel
  {
    double* dn = (double*)malloc(sizeof(double) * nv);
    double* hc = (double*)malloc(sizeof(double) * nv);
    double* ld = (double*)malloc(sizeof(double) * nv);
#pragma omp for schedule(dynamic, 1)
    for (int64_t cell = 0; cell < c->ncells; ++cell)
      collide_cell_adj(c, cell, step, flags, h_s + (size_t)cell * nv, lam_out + (size_t)cell * nv,
                       lam_s + (size_t)cell * nv, dn, hc, ld);
    free(dn);
    free(hc);
    free(ld);
  }
  return BOLTZ_REF_OK;
}

int boltz_ref_step_adjoint(const boltz_ref_ctx* c, const double* h_in, const double* lam_out,
                           double* lam_in, double* grad, const boltz_ref_walls* walls, int64_t step) {
  if (!c || !h_in || !lam_out || !lam_in || lam_out == lam_in) return BOLTZ_REF_EINVAL;
  /* the adjoint follows uniform spatial cells only */
  if (c->sstretched) return BOLTZ_REF_EINVAL;
  if (c->p.flags & BOLTZ_REF_SEQUENTIAL) return BOLTZ_REF_EINVAL;
  const size_t n = (size_t)c->ncells * c->nv;
  double* hs = (double*)malloc(sizeof(double) * n);
  double* lam_s = (double*)malloc(sizeof(double) * n);
  if (!hs || !lam_s) {
    free(hs);
    free(lam_s);
    return BOLTZ_REF_ENOMEM;
  }
  int rc = boltz_ref_stream(c, h_in, hs, walls);
  if (rc == BOLTZ_REF_OK) rc = boltz_ref_collide_adjoint(c, hs, lam_out, lam_s, step, 0u);
  if (rc == BOLTZ_REF_OK) rc = boltz_ref_stream_adjoint(c, h_in, lam_s, lam_in, grad, walls);
  free(hs);
  free(lam_s);
  return rc;
}

int boltz_ref_lid_shear_adjoint(const boltz_ref_ctx* c, const double* h, const boltz_ref_walls* walls,
                                double weight, double* lam, double* grad) {
  if (!c || !h || !walls || !lam || c->p.bc != BOLTZ_REF_BC_CAVITY) return BOLTZ_REF_EINVAL;
  /* the adjoint follows uniform spatial cells only */
  if (c->sstretched) return BOLTZ_REF_EINVAL;
  const int nx = c->p.nx, ny = c->p.ny, nv = c->nv;
  /* D = -(1/nx) sum_ix 2 sum_j w_j v_x v_y hhat_j (see boltz_ref_moments) */
  for (int ix = 0; ix < nx; ++ix) {
    int cell = (ny - 1) * nx + ix;
    double nw = face_density(c, h, WALL_TOP, ix, walls, 1);
    double lam_nw = 0.0;
    for (int j = 0; j < nv; ++j) {
      int jx, jy, jz;
      node_idx(c, j, &jx, &jy, &jz);
      double vx = c->v[0][jx], vy = c->v[1][jy];
      double coef = weight * (-2.0 / nx) * node_w(c, jx, jy, jz) * vx * vy;
      if (vy > 0.0) lam[(size_t)cell * nv + j] += coef;
      else if (vy < 0.0) lam_nw += ghost_value_adj(c, WALL_TOP, ix, nw, j, walls, coef, grad);
    }
    face_density_adj(c, h, WALL_TOP, ix, walls, 1, lam_nw, lam, grad);
  }
  return BOLTZ_REF_OK;
}

/* ---------------------------------------------------------------- step -- */

int boltz_ref_step(const boltz_ref_ctx* c, const double* h_in, double* h_out,
                   const boltz_ref_walls* walls, int64_t step) {
  if (!c || !h_in || !h_out || h_in == h_out) return BOLTZ_REF_EINVAL;
  int rc = boltz_ref_stream(c, h_in, h_out, walls);
  if (rc != BOLTZ_REF_OK) return rc;
  return boltz_ref_collide(c, h_out, h_out, step, 0u, NULL, NULL);
}
