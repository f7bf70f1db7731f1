/*
 * boltz_ref.h -- plain FP64 CPU oracle for one time-split step of the
 * semi-regular Boltzmann solver of Frezzotti, Ghiroldi and Gibelli
 * ("Solving the Boltzmann Equation on GPUs").
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP
 * implementation; it is never part of the product path.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header, table or constant generator with the HIP
 * library: every quantity below is recomputed here from its definition.
 *
 * Units (paper Sec. 2 and Sec. 5.1): n0 = 1, V0 = sqrt(2 R T0) = 1, the
 * cavity is the unit square [0,1]^2 with the lid at y = 1 moving in +x.
 * The unknown is the deviational part h of f = Phi0 (1 + eps h)
 * (Eq. definition), stored cell-major: h[cell][j], cell = iy*nx + ix,
 * j = (jx*ny_v + jy)*nz_v + jz.
 *
 * Parity status of each function is recorded in its comment; functions
 * marked "parity unpinned" have no independent pin.
 */
#ifndef BOLTZ_REF_H
#define BOLTZ_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  BOLTZ_REF_OK = 0,
  BOLTZ_REF_EINVAL = -1,
  BOLTZ_REF_ENOMEM = -2,
  BOLTZ_REF_ENUMERIC = -4,
};

enum { BOLTZ_REF_BC_CAVITY = 0, BOLTZ_REF_BC_PERIODIC = 1 };

/* problem flags */
/* BOLTZ_REF_CONTINUOUS: the pre-collision velocities are drawn from the
 * continuous Maxwellian by the Box-Muller method and binned to their cells
 * (the sampling kernel of Sec. 4), instead of the node law.
 * BOLTZ_REF_SEQUENTIAL: the collision updates h in place, sample after
 * sample (Alg. 3), instead of evaluating every sample at the post-stream h
 * (Eq. collision_step). */
enum { BOLTZ_REF_ALLOW_UNSTABLE = 1u, BOLTZ_REF_CONTINUOUS = 4u, BOLTZ_REF_SEQUENTIAL = 8u };
/* collide flags */
enum { BOLTZ_REF_NO_CORRECTION = 1u };

typedef struct boltz_ref_problem {
  int32_t nx, ny;        /* spatial cells on the unit square                */
  int32_t nv[3];         /* velocity cells per axis                         */
  double vmax[3];        /* velocity box half width per axis (units of V0)  */
  double delta;          /* rarefaction parameter L / lambda0               */
  double eps;            /* deviation scale of Eq. definition (> 0)         */
  double cfl;            /* Courant number used when dt <= 0                */
  double dt;             /* explicit time step; <= 0 means derive from cfl  */
  int32_t order;         /* streaming order: 1 (Eq. streaming2D) or 2       */
  int32_t bc;            /* BOLTZ_REF_BC_CAVITY or BOLTZ_REF_BC_PERIODIC    */
  int64_t n_pairs;       /* N_t: Monte Carlo pairs per cell per step        */
  int64_t sample_group;  /* G: cells sharing one pair stream (0 = all)      */
  uint64_t seed;         /* Philox key                                      */
  uint32_t cavity_id;    /* fourth Philox counter word                      */
  uint32_t flags;        /* BOLTZ_REF_ALLOW_UNSTABLE | BOLTZ_REF_CONTINUOUS */
                         /* | BOLTZ_REF_SEQUENTIAL                          */
  uint32_t mix16;        /* uniform share of the pair law, in 1/16 (0..16); */
                         /* 0 only on grids where every node has a positive */
                         /* Maxwellian-law probability (else EINVAL)        */
  double rv;             /* 0 or 1: uniform velocity cells; 0 < rv < 1:     */
                         /* cells stretched in the progression ratio rv,    */
                         /* smallest at the origin (Sec. 5.1; even counts)  */
  double rx, ry;         /* 0 or 1: uniform spatial cells; 0 < r < 1:       */
                         /* cells stretched in the progression ratio r,     */
                         /* smallest at the side walls (x) and at the lid   */
                         /* (y) (Sec. 5.1); first-order streaming only      */
} boltz_ref_problem;

typedef struct boltz_ref_walls {
  double lid_u;          /* x velocity of the top wall (y = 1)              */
  double tau_left, tau_right, tau_bottom, tau_top;  /* T_w / T0            */
  const double* tau_bottom_x;  /* NULL, or nx per-face T_w / T0 of the     */
                               /* bottom wall (replaces tau_bottom)         */
} boltz_ref_walls;

typedef struct boltz_ref_ctx boltz_ref_ctx;

/* Derived constants reported by boltz_ref_info (in this order). */
enum {
  BOLTZ_REF_INFO_DT = 0, BOLTZ_REF_INFO_K, BOLTZ_REF_INFO_W, BOLTZ_REF_INFO_QFAC,
  BOLTZ_REF_INFO_DX, BOLTZ_REF_INFO_DY, BOLTZ_REF_INFO_NCELLS, BOLTZ_REF_INFO_NV,
  BOLTZ_REF_INFO_COUNT
};

int boltz_ref_create(const boltz_ref_problem* p, boltz_ref_ctx** out);
void boltz_ref_destroy(boltz_ref_ctx* ctx);
const char* boltz_ref_last_error(const boltz_ref_ctx* ctx);
int boltz_ref_info(const boltz_ref_ctx* ctx, double* out /* BOLTZ_REF_INFO_COUNT */);
void boltz_ref_set_threads(int nthreads);
int boltz_ref_get_threads(void);

/* Velocity grid of one axis: node values, weights omega, cumulative
 * thresholds T_1..T_{n-1} of the node law on 12-bit fields (T in [0, 4096]). */
int boltz_ref_axis(const boltz_ref_ctx* ctx, int axis, double* v, double* omega,
                   uint64_t* thresholds /* n-1 entries */);

/* Cell edges of one axis (n + 1 values from -a to a): uniform cells, or
 * the stretched cells of Sec. 5.1. */
/* Widths of the nx (axis 0) or ny (axis 1) spatial cells. */
int boltz_ref_cell_widths(const boltz_ref_ctx* ctx, int axis, double* widths);
int boltz_ref_axis_edges(const boltz_ref_ctx* ctx, int axis, double* edges);

/* Inverse CDF of the per-axis node law on a 12-bit field f:
 * #{i in [1, n) : f >= T_i} (-1 for f >= 4096). */
int boltz_ref_axis_draw(const boltz_ref_ctx* ctx, int axis, uint32_t f);

/* Philox4x32-10 (Salmon et al., SC'11).  Pinned by published known-answer
 * vectors and by the Philox4x64 instance of the same round structure. */
void boltz_ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* cos(2 pi u), sin(2 pi u) by the octant reduction + Taylor polynomials that
 * define the direction map of the pair sampler. */
void boltz_ref_cos_sin_2pi(double u, double* c, double* s);

/* -ln u for u in (0, 1], from the binary exponent and a 40-term series of
 * ln(1 + t), |t| <= sqrt(2) - 1, in a fixed order of IEEE adds and
 * multiplies. */
double boltz_ref_neg_ln(double u);

/* Pair sampler for (cell, step, m0 .. m0+count-1): node indices
 * (a, b, a*, b*) with -1 for a*, b* when the pair is discarded, the weight q
 * (0 when discarded), optionally the four Philox words per pair and the
 * continuous velocities v_a, v_b, v*, v1* (12 doubles per pair). */
int boltz_ref_debug_pairs(const boltz_ref_ctx* ctx, int64_t cell, int64_t step,
                          int64_t m0, int64_t count, int32_t* idx4, double* q,
                          uint32_t* words /* count*4 or NULL */,
                          double* vel /* count*12 or NULL */);

/* Wall densities n_w per boundary face, in the order
 * left[ny], right[ny], bottom[nx], top[nx], exactly as used by one streaming
 * step of h (periodic problems return EINVAL). */
int boltz_ref_wall_density(const boltz_ref_ctx* ctx, const double* h,
                           const boltz_ref_walls* walls, double* nw);

int boltz_ref_stream(const boltz_ref_ctx* ctx, const double* h_in, double* h_out,
                     const boltz_ref_walls* walls);

/* Collision (MC gain/loss + conservation correction).  h_s and h_out may
 * alias.  dN (ncells*nv, optional) receives the raw Monte Carlo increments
 * Delta N; defect (ncells*5, optional) receives sum_j w_j psi_k (F^out - F^s). */
int boltz_ref_collide(const boltz_ref_ctx* ctx, const double* h_s, double* h_out,
                      int64_t step, uint32_t flags, double* dN, double* defect);

/* The same collision for the listed cells only; h_s and h_out hold just
 * those cells (count * nv values, in list order). */
int boltz_ref_collide_cells(const boltz_ref_ctx* ctx, const double* h_s, double* h_out,
                            int64_t step, uint32_t flags, const int64_t* cells, int64_t count);

/* Per-cell moments rho, u_x, u_y, u_z, theta, Pi_xx, Pi_xy, Pi_xz, Pi_yy,
 * Pi_yz, Pi_zz (11 per cell) and the lid shear D (cavity only, optional). */
int boltz_ref_moments(const boltz_ref_ctx* ctx, const double* h,
                      const boltz_ref_walls* walls, double* mom, double* lid_shear);

int boltz_ref_step(const boltz_ref_ctx* ctx, const double* h_in, double* h_out,
                   const boltz_ref_walls* walls, int64_t step);

/* ------------------------------------------------------------ adjoint --
 * Reverse-mode derivatives of the functions above (their transposed
 * linearisations), FP64.  Wall parameters in grad[] (cavity problems,
 * 4 + nx entries, accumulated): lid_u, tau_left, tau_right, tau_top, then
 * the temperature of every bottom face.  Pinned against centred finite
 * differences of the forward functions. */

/* lam_in = (d stream / d h_in)^T lam_out; grad += (d stream / d theta)^T lam_out. */
int boltz_ref_stream_adjoint(const boltz_ref_ctx* ctx, const double* h_in, const double* lam_out,
                             double* lam_in, double* grad, const boltz_ref_walls* walls);

/* lam_s = (d collide / d h_s)^T lam_out for fixed samples (flags as in
 * boltz_ref_collide). */
int boltz_ref_collide_adjoint(const boltz_ref_ctx* ctx, const double* h_s, const double* lam_out,
                              double* lam_s, int64_t step, uint32_t flags);

/* Adjoint of boltz_ref_step (forward recomputed from h_in). */
int boltz_ref_step_adjoint(const boltz_ref_ctx* ctx, const double* h_in, const double* lam_out,
                           double* lam_in, double* grad, const boltz_ref_walls* walls, int64_t step);

/* lam += weight dD/dh and grad += weight dD/dtheta for the lid shear D of
 * boltz_ref_moments. */
int boltz_ref_lid_shear_adjoint(const boltz_ref_ctx* ctx, const double* h, const boltz_ref_walls* walls,
                                double weight, double* lam, double* grad);

#ifdef __cplusplus
}
#endif
#endif
