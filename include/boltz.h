/*
 * boltz.h -- C ABI of the MI355X (gfx950) implementation of one time-split
 * step of the semi-regular Boltzmann solver of Frezzotti, Ghiroldi and
 * Gibelli, "Solving the Boltzmann Equation on GPUs" (arXiv:1005.5405).
 *
 * One step advances the deviational distribution h of f = Phi0 (1 + eps h)
 * (Sec. 2, Eq. definition) on a 2D spatial x 3D velocity grid:
 *   S1  diffuse Maxwell walls with zero net mass flux   (Sec. 2, Eq. bcMax)
 *   S2  free streaming, first-order upwind (Sec. 3, Eq. streaming2D) or its
 *       second-order Beam-Warming counterpart (dimension split x then y)
 *   S3  Monte Carlo sampling of velocity-node pairs and directions
 *       (Sec. 3, Eqs. coll8Dim, monteCarloInt)
 *   S4  gain/loss scatter and the explicit update (Sec. 3, Eq. collision_step)
 *   S5  conservation correction (Sec. 3, Eqs. rinorm_a, correzione)
 *   S6  macroscopic moments (Sec. 2, Eqs. densita..sforzi) and lid shear
 *
 * Units (Sec. 5.1): n0 = 1, V0 = sqrt(2 R T0) = 1, cavity = unit square,
 * lid at y = 1 moving in +x, time unit L/V0, delta = L/lambda0.
 *
 * Layout of every distribution buffer: FP32, cell-major,
 *   h[cell * nv + j],  cell = iy * nx + ix,  j = (jx * nv_y + jy) * nv_z + jz,
 * velocity node of axis k: v_i = (2 i + 1 - nv_k) * vmax_k / nv_k (uniform
 * cells), or the centre of the i-th stretched cell (boltz_problem.rv).
 *
 * Conventions of every call below:
 *   - Buffers named h*, mom, defect, lid_shear are DEVICE pointers owned by
 *     the caller; the library never frees them.  The context owns its own
 *     constant tables and scratch (allocated in boltz_create); the compute
 *     calls allocate nothing.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Compute calls
 *     only enqueue work and return without synchronising; errors detected on
 *     the device (a non-SPD correction matrix, a non-finite value) set bits
 *     of a status word read with boltz_read_status.
 *   - Return value: BOLTZ_OK or a negative boltz_status; the message of the
 *     last failure is returned by boltz_last_error.  No C++ exception
 *     crosses this interface.
 *   - Calls on one context must not overlap on different streams (they
 *     share the context scratch).
 */
#ifndef BOLTZ_H
#define BOLTZ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum boltz_status {
  BOLTZ_OK = 0,
  BOLTZ_EINVAL = -1,       /* invalid argument or problem                    */
  BOLTZ_ENOMEM = -2,       /* device allocation failed                       */
  BOLTZ_EHIP = -3,         /* a HIP runtime call failed                      */
  BOLTZ_ENUMERIC = -4,     /* numerical failure reported by the device       */
  BOLTZ_EUNSUPPORTED = -5  /* valid request the library does not implement  */
} boltz_status;

enum { BOLTZ_BC_CAVITY = 0, BOLTZ_BC_PERIODIC = 1 };

/* boltz_problem.flags */
enum { BOLTZ_ALLOW_UNSTABLE = 1u,    /* accept a dt above the Courant limit  */
       BOLTZ_WITH_ADJOINT = 2u,      /* also allocate the scratch of         */
                                     /* boltz_step_adjoint                   */
       BOLTZ_CONTINUOUS_PAIRS = 4u,  /* draw v, v1 of every pair from the    */
                                     /* continuous Maxwellian (Box-Muller)   */
                                     /* and bin them to cells (Sec. 4's      */
                                     /* sampling kernel) instead of the node */
                                     /* law; see boltz_collide               */
       BOLTZ_SEQUENTIAL_UPDATE = 8u };/* collide in place, sample after      */
                                     /* sample (Alg. 3), instead of the      */
                                     /* Jacobi form; see boltz_collide       */
/* boltz_collide flags */
enum { BOLTZ_NO_CORRECTION = 1u };   /* skip S5 (raw Monte Carlo update)     */
/* device status bits (boltz_read_status) */
enum { BOLTZ_STATUS_NOT_SPD = 1u, BOLTZ_STATUS_NONFINITE = 2u };

/* Problem statement (Sec. 3 discretisation, Sec. 5.1 driven cavity). */
typedef struct boltz_problem {
  int32_t nx, ny;        /* spatial cells on the unit square (cavity: >= 2)  */
  int32_t nv[3];         /* velocity cells per axis, 1..255                  */
  double vmax[3];        /* half width of the velocity box per axis, in V0   */
  double delta;          /* rarefaction parameter L / lambda0 (= 1/Kn)       */
  double eps;            /* deviation scale eps > 0 of Eq. definition        */
  double cfl;            /* largest Courant number when dt <= 0 (Sec. 5.1)   */
  double dt;             /* explicit time step; <= 0: dt from cfl            */
  int32_t order;         /* streaming order: 1 or 2                          */
  int32_t bc;            /* BOLTZ_BC_CAVITY or BOLTZ_BC_PERIODIC             */
  int64_t n_pairs;       /* N_t of Eq. monteCarloInt, pairs per cell per step*/
  int64_t sample_group;  /* G: cells cell/G share a pair stream; 0 = all.    */
                         /* G != 1: the pairs of every group are drawn once */
                         /* per step into a context table (24 B per pair)   */
  uint64_t seed;         /* Philox4x32-10 key (low word, high word)          */
  uint32_t cavity_id;    /* fourth Philox counter word                       */
  uint32_t flags;        /* BOLTZ_ALLOW_UNSTABLE | BOLTZ_WITH_ADJOINT |
                            BOLTZ_CONTINUOUS_PAIRS | BOLTZ_SEQUENTIAL_UPDATE */
  uint32_t mix16;        /* uniform share beta = mix16/16 of the node-pair   */
                         /* law, 0..16.  0 = nodes from the 12-bit discrete  */
                         /* Maxwellian alone: accepted only on grids where   */
                         /* that law gives every node a positive probability */
                         /* (else EINVAL: tail nodes would never be drawn)   */
  double rv;             /* velocity cells: 0 or 1 uniform; 0 < rv < 1      */
                         /* stretched in the progression ratio rv, the      */
                         /* smallest at the origin (Sec. 5.1): on each half */
                         /* axis the i-th cell from the origin is w0 rv^-i  */
                         /* long; needs even nv[k] (else EINVAL)            */
  double rx, ry;         /* spatial cells: 0 or 1 uniform; 0 < r < 1        */
                         /* stretched in the progression ratio r (Sec. 5.1):*/
                         /* along x the cell d cells from the nearer side   */
                         /* wall is w0 rx^-d long, along y the cell d cells */
                         /* below the lid w0 ry^-d (lengths adding up to 1);*/
                         /* streams at order 1 with each cell's own lengths */
                         /* in its Courant numbers, the time step from the  */
                         /* smallest cells, the lid shear D weighted by the */
                         /* face lengths.  Needs order 1; no adjoint and no */
                         /* batches (EINVAL)                                 */
} boltz_problem;

/* Wall state for one call (Sec. 2, Eq. bcMax; Sec. 5.1). */
typedef struct boltz_walls {
  double lid_u;          /* x velocity of the top wall y = 1, in V0          */
  double tau_left, tau_right, tau_bottom, tau_top;  /* T_w / T0, > 0         */
  const double* tau_bottom_x;  /* NULL, or a HOST array of nx values T_w/T0  */
                               /* of the bottom faces (replaces tau_bottom;  */
                               /* read during the call only)                 */
} boltz_walls;

typedef struct boltz_info {
  int64_t ncells;        /* nx * ny                                          */
  int64_t nv;            /* nv[0] * nv[1] * nv[2]                            */
  double dt;             /* time step in use                                 */
  double K;              /* pi n0 sigma^2 = (5/16) sqrt(2 pi) 1.016034 delta */
  double W;              /* discrete mass of Phi0 on the velocity grid       */
  double qfac;           /* dt K / N_t                                       */
  int64_t device_bytes;  /* device memory held by the context                */
  int32_t collide_layout;   /* LDS layout of the collision (BOLTZ_LAYOUT_*) */
  int32_t collide_block;    /* its threads per workgroup (shared samples)   */
  int32_t collide_lds_nodes; /* nodes of the h tile held in LDS             */
  int32_t collide_per_cu;   /* its workgroups resident per CU (occupancy)  */
} boltz_info;

/* LDS layouts of the collision kernel (boltz_info.collide_layout): where the
 * per-cell increments of Eq. monteCarloInt are accumulated.
 *   FIXED   64-bit fixed point for every node next to the full h tile
 *   SPLIT   the same for one half of the nodes per pass over the pairs
 *   CAS     FP32 compare-and-swap
 *   HYBRID  64-bit fixed point for the central x-slabs, FP32 for the rest
 *   PART    64-bit fixed point for every node, the h tile of the central
 *           x-slabs in LDS and the outer slabs read from global memory
 *   SEQUENTIAL  BOLTZ_SEQUENTIAL_UPDATE: the FP32 h tile updated in place,
 *           one wavefront per cell
 * The environment variable BOLTZ_COLLIDE_LAYOUT=hybrid, read by
 * boltz_create, selects HYBRID over PART where both fit. */
enum { BOLTZ_LAYOUT_CAS = 0, BOLTZ_LAYOUT_FIXED = 1, BOLTZ_LAYOUT_SPLIT = 2, BOLTZ_LAYOUT_HYBRID = 3,
       BOLTZ_LAYOUT_PART = 4, BOLTZ_LAYOUT_SEQUENTIAL = 5 };

typedef struct boltz_ctx boltz_ctx;

/* Validate the problem, build the velocity-grid tables (Sec. 3) and the
 * per-axis sampling thresholds, and allocate the context on the current HIP
 * device.  EINVAL: out-of-range sizes, a dt above the Courant limit of the
 * streaming scheme (unless BOLTZ_ALLOW_UNSTABLE), n_pairs >= 2^31.
 * EINVAL also for shared samples (G != 1) with more than 65535 groups or
 * velocity nodes, and for mix16 = 0 on a grid where the Maxwellian node law
 * leaves a node unreachable (checked before any device call).  EUNSUPPORTED: a velocity grid whose two per-cell FP32
 * tiles exceed the 160 KB local data share.  ENOMEM / EHIP: device
 * allocation failed. */
int boltz_create(const boltz_problem* problem, boltz_ctx** out);

void boltz_destroy(boltz_ctx* ctx);

int boltz_query(const boltz_ctx* ctx, boltz_info* out);

/* Message of the last failure on ctx (ctx = NULL: of the last failed
 * boltz_create on this thread).  Valid until the next call on ctx. */
const char* boltz_last_error(const boltz_ctx* ctx);

/* S1 + S2: one free-streaming step h_in -> h_out (Sec. 3, Eq. freestreaming
 * discretised by Eq. streaming2D for order 1, Beam-Warming x then y for
 * order 2), with the diffuse-wall emission of Eq. bcMax whose density n_w
 * makes the discrete mass flux through every boundary face vanish.  h_in and
 * h_out: ncells*nv FP32, must not overlap.  walls: host pointer, required for
 * cavities, ignored (may be NULL) for periodic problems. */
int boltz_stream(boltz_ctx* ctx, const float* h_in, float* h_out, const boltz_walls* walls,
                 void* stream);

/* S3 + S4 + S5: one collision step at fixed position (Sec. 3, Eq. homrel),
 * h_s -> h_out.  N_t pairs per cell: nodes a, b drawn from the mixture
 * (1 - beta) Maxwellian node law + beta uniform node law, a direction
 * uniform on the sphere, from one Philox4x32-10 block with counter
 * (m, group, step, cavity_id) and key seed; each pair carries the
 * importance weight dt K |v_r . k| (w_a/p_a)(w_b/p_b) / N_t of Eq. coll8Dim
 * (w = midpoint weight of Phi0, p = probability of the draw); the Monte Carlo
 * increments of Eq. monteCarloInt are applied in Jacobi form
 * (Eq. collision_step), then the correction of Eq. rinorm_a restores the
 * post-stream mass, momentum and energy (FP64 sums and 5x5 solve).
 * With BOLTZ_CONTINUOUS_PAIRS (problem flag) the pairs follow the sampling
 * kernel of Sec. 4 instead: v and v1 from the continuous Maxwellian by the
 * Box-Muller method (two Philox blocks, counters (m, group, step, cavity)
 * and (m, group | 2^31, step, cavity)), h taken in the cells that contain
 * them, weight dt K |v_r . k| / N_t; a pair with any velocity outside the
 * box is discarded (it still counts in N_t).
 * With BOLTZ_SEQUENTIAL_UPDATE (problem flag; shared samples only, i.e.
 * sample_group != 1, else boltz_create returns EINVAL) the samples update h
 * in place in the order m = 0, 1, ... as in Alg. 3: each reads the current
 * h at a and b and adds its four increments before the next one is read
 * (where two of its nodes coincide, both increments land).  The cell's h is
 * kept in FP32 during the loop (the paper's precision), the correction
 * restores the moments of h_s as above.  Results do not depend on the
 * launch (the order of every node's updates is the sample order).  The
 * samples that share no node are applied together; which of two schedules
 * groups them is chosen per problem at boltz_create (the environment
 * variable BOLTZ_SEQ_SCHEDULE=steps|groups, read there, overrides it).
 * h_s may equal h_out (in place); otherwise they must not overlap.
 * flags: BOLTZ_NO_CORRECTION.  defect: NULL or ncells*5 FP64 device buffer
 * receiving sum_j w_j psi_k (F_out - F_s) of the stored FP32 values. */
int boltz_collide(boltz_ctx* ctx, const float* h_s, float* h_out, int64_t step, uint32_t flags,
                  double* defect, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * collision as boltz_collide, same arguments and results, except that the
 * shared-sample pair records of the step (sample_group != 1) are kept in a
 * file-scope device array of the library instead of the context: 16 MiB per
 * device, i.e. about 699 000 records per step (half that with velocity grids
 * whose collision sorts the records), held until the process ends.  EINVAL
 * beyond that size.  The call allocates nothing and frees nothing.  Every
 * call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (any context, any stream) race and must be serialised by the caller.
 * With BOLTZ_SEQUENTIAL_UPDATE the array also holds the step schedule of
 * the records (12 B per record, 36 B per record in all).
 * With per-cell samples (sample_group == 1) it uses no scratch. */
int boltz_collide_noalloc(boltz_ctx* ctx, const float* h_s, float* h_out, int64_t step, uint32_t flags,
                          double* defect, void* stream);

/* S6: per-cell moments (Sec. 2, Eqs. densita..sforzi, re-derived in units
 * of V0): mom[cell*11 + k] = rho, u_x, u_y, u_z, theta, Pi_xx, Pi_xy, Pi_xz,
 * Pi_yy, Pi_yz, Pi_zz (FP64 device buffer).  lid_shear: NULL or one FP64
 * device value D = -(1/nx) sum over lid faces of Pi_xy, built from the
 * gas-side values of the top cells and the wall emission (Sec. 5.2 defines
 * D as the mean shear stress on the moving wall); cavity only. */
int boltz_moments(boltz_ctx* ctx, const float* h, const boltz_walls* walls, double* mom,
                  double* lid_shear, void* stream);

/* One full time-split step h_in -> h_out: boltz_stream then boltz_collide
 * in place on h_out (Sec. 3).  h_in and h_out must not overlap. */
int boltz_step(boltz_ctx* ctx, const float* h_in, float* h_out, const boltz_walls* walls,
               int64_t step, void* stream);

/* ---- Reverse mode (the paper has no adjoint; these are the transposes of
 * the linearised calls above for fixed Philox samples, used to differentiate
 * a functional of the flow with respect to the initial state and the wall
 * parameters).  Adjoints are FP64 device buffers of ncells*nv values in the
 * layout of h.  grad_walls: NULL or a device FP64 array of 4 + nx entries to
 * which the call ADDS the wall-parameter gradient, in the order
 *   lid_u, tau_left, tau_right, tau_top, tau of bottom face 0 .. nx-1
 * (a uniform bottom wall: the sum of the last nx entries is the derivative
 * with respect to tau_bottom); periodic problems add nothing.  The context
 * scratch used by these calls (BOLTZ_WITH_ADJOINT at boltz_create): 12 bytes
 * per phase-space node.  EUNSUPPORTED: a velocity grid whose h tile, FP32
 * and 64-bit arrays and tables exceed the 160 KB local data share. */

/* Adjoint of boltz_stream (Sec. 3, Eq. streaming2D / the Beam-Warming
 * sweeps, with the wall emission of Eq. bcMax): lam_in = (dh_out/dh_in)^T
 * lam_out, where h_out = boltz_stream(h_in).  h_in: the FP32 state that was
 * streamed.  lam_in must not overlap lam_out.  Order 2 needs the
 * BOLTZ_WITH_ADJOINT scratch. */
int boltz_stream_adjoint(boltz_ctx* ctx, const float* h_in, const double* lam_out, double* lam_in,
                         double* grad_walls, const boltz_walls* walls, void* stream);

/* Adjoint of boltz_collide (Sec. 3, Eqs. monteCarloInt, collision_step,
 * rinorm_a, correzione) at the post-stream state h_s: lam_s =
 * (dh_out/dh_s)^T lam_out.  The collision is recomputed per cell from h_s;
 * the correction's 5x5 system is solved a second time for the transposed
 * right-hand side.  lam_s may equal lam_out (in place).  flags:
 * BOLTZ_NO_CORRECTION. */
int boltz_collide_adjoint(boltz_ctx* ctx, const float* h_s, const double* lam_out, double* lam_s, int64_t step,
                          uint32_t flags, void* stream);

/* Adjoint of boltz_step (h_in -> h_out at `step`): lam_in = (dh_out/dh_in)^T
 * lam_out, and the wall-parameter gradient added to grad_walls.  The
 * post-stream state is recomputed from h_in.  lam_in may equal lam_out (in
 * place); needs the BOLTZ_WITH_ADJOINT scratch (EINVAL otherwise). */
int boltz_step_adjoint(boltz_ctx* ctx, const float* h_in, const double* lam_out, double* lam_in,
                       double* grad_walls, const boltz_walls* walls, int64_t step, void* stream);

/* Adjoint of weight * D, D the lid shear of boltz_moments (Sec. 5.2): ADDS
 * weight * dD/dh to lam (only the top row of cells changes) and
 * weight * dD/dtheta to grad_walls (NULL: not formed).  Cavity only. */
int boltz_lid_shear_adjoint(boltz_ctx* ctx, const float* h, const boltz_walls* walls, double weight, double* lam,
                            double* grad_walls, void* stream);

/* ---- Batches: many independent problems (cavities of different size,
 * velocity grid, Knudsen number, lid velocity and pair count) advanced by
 * one step with one launch per phase: the face densities of every cavity,
 * the streaming of every problem, the shared-sample records of every
 * problem, and one persistent collision launch over a work list of
 * (problem, cell) items sorted by decreasing cost.  Every problem's result
 * is bitwise that of boltz_step on the problem alone.  The step number is a
 * device counter (boltz_batch_set_step; boltz_batch_step advances it), so a
 * captured HIP graph of boltz_batch_step calls replays successive steps.
 * All problems must share the streaming order and have nv[2] % 4 == 0. */
typedef struct boltz_batch boltz_batch;

typedef struct boltz_batch_info {
  int32_t count;         /* problems                                         */
  int32_t collide_block; /* threads per workgroup of the collision of the
                            class with the most pair-cells                   */
  int64_t nodes;         /* phase-space nodes of the whole batch             */
  int64_t pair_cells;    /* sum over problems of cells * n_pairs             */
  int64_t device_bytes;  /* device memory held by the batch                  */
  int32_t classes;       /* classes (problems with one velocity grid)        */
  int32_t stream_tile[2]; /* cells per stream workgroup in x and y           */
  int32_t reserved;
} boltz_batch_info;

/* A class of a batch: its problems with one velocity grid.  Each class's
 * cells are one collision launch per step with settings of their own. */
typedef struct boltz_batch_class {
  int32_t nv[3];          /* the class's velocity grid                       */
  int32_t problems;       /* problems in it                                  */
  int64_t cells;          /* their cells                                     */
  int64_t pair_cells;     /* sum of cells * n_pairs                          */
  int32_t collide_block;  /* threads per workgroup                           */
  int32_t pairs_per_lane; /* shared pair records per thread in flight (2, 4) */
  int32_t spread;         /* workgroups: 0 one per resident slot, 1 two per
                             slot, 2 one per cell                            */
  int32_t grid;           /* the resulting workgroups of the launch          */
  int32_t cells_per_group; /* cells per workgroup, rounded up               */
  int32_t reserved;
  double ms;              /* ms per launch measured by boltz_batch_tune at
                             these settings (0 before tuning)                */
} boltz_batch_class;

/* Create a batch of `count` (1..4096) problems on the current device; each
 * problem is validated as by boltz_create (its error message names it).
 * EINVAL also for mixed streaming orders or nv[2] % 4 != 0. */
int boltz_batch_create(const boltz_problem* problems, int count, boltz_batch** out);

void boltz_batch_destroy(boltz_batch* batch);

int boltz_batch_query(const boltz_batch* batch, boltz_batch_info* out);

const char* boltz_batch_last_error(const boltz_batch* batch);

/* offsets (host, count values): first element of each problem's state in
 * the batch's h buffers (ncells * nv FP32 values each, contiguous). */
int boltz_batch_offsets(const boltz_batch* batch, int64_t* offsets);

/* The context of problem `index` (owned by the batch, valid until
 * boltz_batch_destroy): every single-problem call (moments, adjoints, ...)
 * works on its slice of the batch state.  NULL for an invalid index. */
boltz_ctx* boltz_batch_problem(boltz_batch* batch, int index);

/* Set the device step counter (enqueued on `stream`). */
int boltz_batch_set_step(boltz_batch* batch, int64_t step, void* stream);

/* One step of every problem: h_in -> h_out (device, batch layout, must not
 * overlap) at the device step counter, which is then advanced.  walls: host
 * array of `count` wall states (entries of periodic problems ignored; NULL
 * if there is no cavity).  Enqueues only kernels; while the wall states do
 * not change it can be captured into a HIP graph. */
int boltz_batch_step(boltz_batch* batch, const float* h_in, float* h_out, const boltz_walls* walls,
                     void* stream);

/* Tuning (h_a and h_b are working buffers, both overwritten; the step
 * counter advances).  First the stream tile shape (16 x 8 or 32 x 4 cells),
 * by `steps` whole steps each; then, for every class, every collision
 * setting whose LDS fits (block size 256, 512, 1024 threads x 2 or 4 shared
 * records per thread in flight x the three workgroup spreads), by `steps`
 * launches of the class's collision alone; the fastest of each is kept.
 * The sample group G is part of each problem (it decides which samples a
 * cell uses) and is not tuned.  ms_out (host, 2 values or NULL): ms per
 * whole step before and after.  Synchronises `stream`. */
int boltz_batch_tune(boltz_batch* batch, float* h_a, float* h_b, const boltz_walls* walls, int steps,
                     void* stream, double* ms_out);

/* Use a given collision block size (256, 512 or 1024) for every class whose
 * layout allows it (the partial-tile layout of 24^3-class grids runs 1024
 * threads only); EINVAL if no class can. */
int boltz_batch_set_block(boltz_batch* batch, int block);

/* Settings of class `index` (0 .. classes - 1; EINVAL beyond) into *out. */
int boltz_batch_class_info(const boltz_batch* batch, int index, boltz_batch_class* out);

/* Set one class's collision (block 256/512/1024 where its LDS fits,
 * pairs_per_lane 2 or 4, spread 0..2; EINVAL otherwise). */
int boltz_batch_set_class(boltz_batch* batch, int index, int block, int pairs_per_lane, int spread);

/* Stream tile shape: (16, 8) or (32, 4) cells per workgroup; EINVAL else. */
int boltz_batch_set_stream_tile(boltz_batch* batch, int tx, int ty);

/* Test hook: the pairs the collision kernel draws for (cell, step) and pair
 * indices m0 .. m0+count-1, computed on the device by the kernel's own
 * sampler.  idx4 (host, count*4): a, b, a*, b* (a* = b* = -1 for a discarded
 * pair); q (host, count): weight dt K |v_r . k| (w_a/p_a)(w_b/p_b) / N_t (0 if
 * discarded);
 * words (host, count*4 or NULL): the Philox4x32-10 block.  Synchronous. */
int boltz_debug_pairs(boltz_ctx* ctx, int64_t cell, int64_t step, int64_t m0, int64_t count,
                      int32_t* idx4, double* q, uint32_t* words);

/* Test hook: thresholds T_1..T_{n-1} of the Maxwellian node law of one axis
 * on 12-bit fields (host buffer of nv[axis]-1 uint64 values in [0, 4096]). */
int boltz_axis_thresholds(const boltz_ctx* ctx, int axis, uint64_t* out);

/* Read (and optionally clear) the device status word after synchronising
 * `stream`.  *out: OR of BOLTZ_STATUS_* bits raised since the last clear. */
int boltz_read_status(boltz_ctx* ctx, uint32_t* out, int clear, void* stream);

#ifdef __cplusplus
}
#endif
#endif
