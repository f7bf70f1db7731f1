// kernels.hpp -- HIP kernels of one time-split step (CDNA4 / gfx950).
//
//   wallconst_kernel S1  per wall: table Phi_w / Phi0 of the re-emitted
//                        Maxwellian and the flux sums A_w, D_w (rebuilt only
//                        when the walls change)
//   wall_kernel      S1  per boundary face: the discrete zero-net-flux
//                        density n_w (Sec. 2, Eq. bcMax)
//   stream4_kernel   S2  one HBM pass: (16x8 cells + upwind halo) x 32
//                        velocities per workgroup staged in LDS, four
//                        velocities per thread; order 1 = Eq. streaming2D,
//                        order 2 = Beam-Warming x sweep then y sweep
//   stream_kernel    S2  scalar form for velocity grids with n_z % 4 != 0
//   collide_kernel   S3-S5  (collide.hpp) persistent workgroups walking the
//                        spatial cells: the cell's h tile and its increment
//                        accumulators live in LDS, lanes draw Philox pairs
//                        (or read the shared-sample table), gather h_a, h_b
//                        and scatter gain/loss with LDS atomics (Eqs.
//                        monteCarloInt, collision_step), then FP64 moment
//                        sums, a 5x5 LDL^T solve and the correction of
//                        Eq. rinorm_a, one coalesced store
//   moments_kernel   S6  FP64 moments per cell (Eqs. densita..sforzi) and the
//                        lid-face shear partial sums
#pragma once

#include "device_math.hpp"

namespace boltz {

enum { WALL_LEFT = 0, WALL_RIGHT = 1, WALL_BOTTOM = 2, WALL_TOP = 3 };

// Problem constants and device tables (by value, one kernel argument).
struct Params {
  int nx, ny, nv;
  int n[3];
  int vneg[3], vpos[3];   // per axis: nodes 0 .. vneg - 1 move with v < 0, vpos .. n - 1 with v > 0
  int order, bc;
  int64_t n_pairs, sample_group;
  uint32_t key0, key1, cavity, mix16;
  double beta;            // mix16 / 16
  double dt, dx, dy, eps, inv_eps, qfac;
  double a[3], inv_cell[3];
  const double* vtab;     // [3][kMaxAxis] node velocities
  const double* omtab;    // [3][kMaxAxis] per-axis weights omega
  const double* rwtab;    // [3][kMaxAxis] 1 / omega
  const float4* nqtab;    // [3][kMaxAxis] {omega, p_phi, p_unif, 0} in FP32: weight
                          // and realised Maxwellian / uniform laws of one axis
  const uint8_t* icdf;    // [3][kFieldSize] Maxwellian inverse CDF on 12-bit fields
  const float* cour;      // [2][kMaxAxis] Courant number |v| dt / d{x,y}
  const float* cour2;     // [2][kMaxAxis] C (1 - C) / 2
  double* nw;             // [2 ny + 2 nx] face densities: left, right, bottom, top
  double* ratio;          // [4][nv] Phi_w / Phi0 per wall and node (bottom slot unused)
  double* ratio_b;        // [nx][nv] Phi_w / Phi0 of every bottom face
  const double* tau_b;    // [nx] T_w / T0 of every bottom face
  const double* m0;       // [15] sum_j w_j psi_k psi_l, psi = (1, v, |v|^2), packed k <= l
  const double* zmom;     // [nv_z][8] omega_z v_z^p for p = 0..4 (then zeros)
  double* dpart;          // [nx] lid shear partial sums
  double* wconst;         // [4][2] per wall: A_w, D_w of the face densities
  double* wconst_b;       // [nx][2] A, D of every bottom face
  uint32_t* status;       // device status bits
  // ACC_HYBRID collisions: nodes hyb_lo .. hyb_lo + hyb_n - 1 (whole
  // x-slabs) take 64-bit accumulators, the others FP32; hyb_ovf: one row of
  // nv FP32 values per persistent workgroup for the rare terms beyond the
  // 64-bit range (zero between uses)
  int hyb_lo, hyb_n;
  float* hyb_ovf;
  // stretched velocity cells (Sec. 5.1): post-collision cells by search
  int stretched;
  // pairs from the continuous Maxwellian (Box-Muller), binned to cells
  int continuous;
  // stretched spatial cells (Sec. 5.1; first-order streaming): widths of
  // the x cells and reciprocal widths along x and y, else null
  const double* wx;
  const double* inv_wx;
  const double* inv_wy;
  const double* edgetab;  // [3][kMaxAxis + 1] cell edges -a .. a per axis
};

// One problem of a batch: its constants and tables, the offset of its state
// in the batch's h buffers and its shared-sample records.
struct BatchCav {
  Params P;
  int64_t hoff;    // first element of the problem's h in the batch buffers
  uint2* tidx;     // shared-sample records (G != 1), else null
  float4* tcoef;
  uint2* sidx;     // where the sampler writes them (ACC_SPLIT: before the
  float4* scoef;   // sort by target half; else tidx, tcoef)
  int mode;        // accumulation of the collide increments (ACC_*)
  int pad;
};

// Problem of work unit u of a batched launch: the largest c with
// start[c] <= u, start[0] = 0 (start has count + 1 entries).
__device__ __forceinline__ int find_cav(const int* __restrict__ start, int count, int u) {
  int lo = 0, hi = count;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= u) lo = mid;
    else hi = mid;
  }
  return lo;
}

struct WallArgs {
  double lid_u;
  double tau[4];   // left, right, bottom, top
  double tfac[4];  // tau^-3/2
};

__device__ __forceinline__ void node_decode(int j, int n1, int n2, int& jx, int& jy, int& jz) {
  jz = j % n2;
  const int t = j / n2;
  jy = t % n1;
  jx = t / n1;
}

// Phi_w(v) / Phi0(v) for a wall Maxwellian (U, 0, 0), T_w / T0 = tau.
__device__ __forceinline__ double wall_ratio(double vx, double vy, double vz, double U, double tau,
                                             double tfac) {
  const double v2 = (vx * vx + vy * vy) + vz * vz;
  const double ux = vx - U;
  const double c2 = (ux * ux + vy * vy) + vz * vz;
  return tfac * exp(v2 - c2 / tau);
}

// Re-emitted deviation h_w = (n_w Phi_w/Phi0 - 1)/eps, stored in FP32.
__device__ __forceinline__ float ghost_value(double nw, double R, double inv_eps) {
  return (float)((nw * R - 1.0) * inv_eps);
}

__device__ __forceinline__ int64_t cell_off(const Params& P, int ix, int iy) {
  return ((int64_t)iy * P.nx + ix) * P.nv;
}

// Phi_w / Phi0 of all nodes for face `pos` of a wall (the bottom wall has one
// table per face: it may carry a temperature profile).
__device__ __forceinline__ const double* ratio_row(const Params& P, int wall, int pos) {
  return wall == WALL_BOTTOM ? P.ratio_b + (int64_t)pos * P.nv : P.ratio + (int64_t)wall * P.nv;
}

// A and D of the face densities of face `pos` of a wall.
__device__ __forceinline__ const double* wall_consts(const Params& P, int wall, int pos) {
  return wall == WALL_BOTTOM ? P.wconst_b + 2 * pos : P.wconst + 2 * wall;
}

// ------------------------------------------------------------------- S1 --
// x-swept value (order 2) of node j at (ix, iy), read straight from global
// memory; the same FP32 arithmetic as the stream kernel's x sweep.
__device__ float xswept_value(const Params& P, const float* h, int ix, int iy,
                              int j, int jx, int jy, int jz, double nwl, double nwr) {
  const double vx = P.vtab[jx];
  const float h0 = h[cell_off(P, ix, iy) + j];
  if (vx == 0.0) return h0;
  const int s = vx > 0.0 ? 1 : -1;
  float hn[2];
  for (int d = 1; d <= 2; ++d) {
    const int i = ix - d * s;
    if (i >= 0 && i < P.nx) {
      hn[d - 1] = h[cell_off(P, i, iy) + j];
    } else {
      const int wall = (i < 0) ? WALL_LEFT : WALL_RIGHT;
      hn[d - 1] = ghost_value(i < 0 ? nwl : nwr, P.ratio[(int64_t)wall * P.nv + j], P.inv_eps);
    }
  }
  return bw_update(h0, hn[0], hn[1], P.cour[jx], P.cour2[jx]);
}

// Density n_w of one face.  A = sum_out |v_n| w_j, D = sum over the mirror
// images of the outgoing nodes of |v_n| w R (same order as A, so a wall at
// rest facing h = 0 gives n_w = 1 exactly), B = sum_out |v_n| w_j hhat_j;
// n_w = (A + eps B) / D.  `order` selects the face value: 1 = adjacent cell,
// 2 = Beam-Warming face value, from the x-swept state for y faces.
__device__ double face_density(const Params& P, const float* h, int wall, int pos,
                               int order, double nwl0, double nwl1, double nwr0, double nwr1,
                               double* red) {
  const int nx = P.nx, ny = P.ny, nv = P.nv, n1 = P.n[1], n2 = P.n[2];
  const int nax = (wall <= WALL_RIGHT) ? 0 : 1;
  const int sgn = (wall == WALL_LEFT || wall == WALL_BOTTOM) ? 1 : -1;
  int ax_, ay_, bx_, by_;
  switch (wall) {
    case WALL_LEFT: ax_ = 0; ay_ = pos; bx_ = 1; by_ = pos; break;
    case WALL_RIGHT: ax_ = nx - 1; ay_ = pos; bx_ = nx - 2; by_ = pos; break;
    case WALL_BOTTOM: ax_ = pos; ay_ = 0; bx_ = pos; by_ = 1; break;
    default: ax_ = pos; ay_ = ny - 1; bx_ = pos; by_ = ny - 2; break;
  }
  const double dl = nax ? P.dy : P.dx;
  const bool ysw = (order == 2) && (nax == 1);
  double s[3] = {0.0, 0.0, 0.0};
  // four nodes per thread and pass, so that their loads are in flight together
  constexpr int U = 4;
  const int step = blockDim.x;
  NodeWalk walk(threadIdx.x, step, n1, n2);
  for (int j0 = threadIdx.x; j0 < nv; j0 += U * step) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u * step;
      const int jx = walk.jx, jy = walk.jy, jz = walk.jz;
      walk.next();
      if (j >= nv) continue;
      const double vn = nax ? P.vtab[kMaxAxis + jy] : P.vtab[jx];
      if (!(sgn * vn < 0.0)) continue;
      const double an = fabs(vn);
      const double w = (P.omtab[jx] * P.omtab[kMaxAxis + jy]) * P.omtab[2 * kMaxAxis + jz];
      int mx = jx, my = jy;
      if (nax == 0) mx = P.n[0] - 1 - jx; else my = n1 - 1 - jy;
      const double R = ratio_row(P, wall, pos)[(mx * n1 + my) * n2 + jz];
      double ha, hb = 0.0;
      if (ysw) {
        ha = xswept_value(P, h, ax_, ay_, j, jx, jy, jz, nwl0, nwr0);
        hb = xswept_value(P, h, bx_, by_, j, jx, jy, jz, nwl1, nwr1);
      } else {
        ha = h[cell_off(P, ax_, ay_) + j];
        if (order == 2) hb = h[cell_off(P, bx_, by_) + j];
      }
      double hh = ha;
      if (order == 2) {
        const double C = an * P.dt / dl;
        hh = ha + 0.5 * (1.0 - C) * (ha - hb);
      }
      const double aw = an * w;
      s[0] += aw;
      s[1] += aw * R;
      s[2] += aw * hh;
    }
  }
  block_sum<3>(s, red);
  return (s[0] + P.eps * s[2]) / s[1];
}

// One workgroup per wall (left, right, top) and per bottom face: the table
// Phi_w / Phi0 of every node (FP64; only the lid moves, with velocity lid_u
// along x), then A = sum_out |v_n| w_j and D = sum over the mirror images of
// the outgoing nodes of |v_n| w R, reduced in one pass with the same tree so
// that a wall at rest (R = 1) gives D = A bitwise.  Launched only when the
// wall state changes.
constexpr int kWallConstBlock = 1024;

// Blocks first, first + 1, ... of the full set (0 left, 1 right, 2 top, 3 +
// i bottom face i): a change of the lid alone rebuilds block 2 only.
__global__ __launch_bounds__(kWallConstBlock) void wallconst_kernel(Params P, WallArgs W, int first) {
  __shared__ double red[2 * (kWallConstBlock / 64)];
  const int b = (int)blockIdx.x + first;
  const int wall = b == 0 ? WALL_LEFT : (b == 1 ? WALL_RIGHT : (b == 2 ? WALL_TOP : WALL_BOTTOM));
  const int pos = b < 3 ? 0 : b - 3;
  const int nv = P.nv, n1 = P.n[1], n2 = P.n[2];
  const double Uw = (wall == WALL_TOP) ? W.lid_u : 0.0;
  const double tau = wall == WALL_BOTTOM ? P.tau_b[pos] : W.tau[wall];
  const double tfac = wall == WALL_BOTTOM ? pow(tau, -1.5) : W.tfac[wall];
  double* R = const_cast<double*>(ratio_row(P, wall, pos));
  for (int j = threadIdx.x; j < nv; j += blockDim.x) {
    int jx, jy, jz;
    node_decode(j, n1, n2, jx, jy, jz);
    R[j] = wall_ratio(P.vtab[jx], P.vtab[kMaxAxis + jy], P.vtab[2 * kMaxAxis + jz], Uw, tau, tfac);
  }
  __syncthreads();
  const int nax = (wall <= WALL_RIGHT) ? 0 : 1;
  const int sgn = (wall == WALL_LEFT || wall == WALL_BOTTOM) ? 1 : -1;
  double s[2] = {0.0, 0.0};
  for (int j = threadIdx.x; j < nv; j += blockDim.x) {
    int jx, jy, jz;
    node_decode(j, n1, n2, jx, jy, jz);
    const double vn = nax ? P.vtab[kMaxAxis + jy] : P.vtab[jx];
    if (!(sgn * vn < 0.0)) continue;
    const double aw = fabs(vn) * ((P.omtab[jx] * P.omtab[kMaxAxis + jy]) * P.omtab[2 * kMaxAxis + jz]);
    int mx = jx, my = jy;
    if (nax == 0) mx = P.n[0] - 1 - jx; else my = n1 - 1 - jy;
    s[0] += aw;
    s[1] += aw * R[(mx * n1 + my) * n2 + jz];
  }
  block_sum<2>(s, red);
  if (threadIdx.x == 0) {
    double* k = const_cast<double*>(wall_consts(P, wall, pos));
    k[0] = s[0];
    k[1] = s[1];
  }
}

// B of one face: sum over the outgoing nodes of |v_n| w_j hhat_j (hhat as in
// face_density).  The outgoing nodes (a range of the normal axis) are
// numbered t = 0, 1, ... in velocity order; this thread takes t = j0, j0 +
// step, ..., U nodes per pass with every load of a pass issued before it
// is used.  A y face of order 2 away from the corner columns reads the three
// cells of each x sweep directly (no ghost value is needed there).
template <int U>
__device__ double face_b(const Params& P, const float* h, int wall, int pos, int order,
                         double nwl0, double nwl1, double nwr0, double nwr1, int j0, int step) {
  const int nx = P.nx, ny = P.ny, nv = P.nv, n1 = P.n[1], n2 = P.n[2];
  const int nax = (wall <= WALL_RIGHT) ? 0 : 1;
  const int sgn = (wall == WALL_LEFT || wall == WALL_BOTTOM) ? 1 : -1;
  int ax_, ay_, bx_, by_;
  switch (wall) {
    case WALL_LEFT: ax_ = 0; ay_ = pos; bx_ = 1; by_ = pos; break;
    case WALL_RIGHT: ax_ = nx - 1; ay_ = pos; bx_ = nx - 2; by_ = pos; break;
    case WALL_BOTTOM: ax_ = pos; ay_ = 0; bx_ = pos; by_ = 1; break;
    default: ax_ = pos; ay_ = ny - 1; bx_ = pos; by_ = ny - 2; break;
  }
  const double dl = nax ? P.dy : P.dx;
  const bool ysw = (order == 2) && (nax == 1);
  const bool corner = ysw && (pos < 2 || pos >= nx - 2);
  const float* ca = h + cell_off(P, ax_, ay_);
  const float* cb = h + cell_off(P, bx_, by_);
  // outgoing along the normal: v < 0 at the left / bottom wall, v > 0 at
  // the right / top wall
  const int i0 = sgn > 0 ? 0 : P.vpos[nax], i1 = sgn > 0 ? P.vneg[nax] : P.n[nax];
  // the outgoing nodes as a (c0, c1, n2) box: c0 = x nodes, c1 = y nodes
  const int c0 = nax ? P.n[0] : i1 - i0, c1 = nax ? i1 - i0 : n1;
  const int nt = c0 * c1 * n2;
  double b = 0.0;
  if (nt <= 0) return b;
  NodeWalk walk(j0, step, c1, n2);
  for (int tb = j0; tb < nt; tb += U * step) {
    int jxs[U], jys[U], jzs[U], js[U];
    float a0[U], a1[U], a2[U], b0[U], b1[U], b2[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool in = tb + u * step < nt;
      jxs[u] = in ? walk.jx + (nax ? 0 : i0) : 0;
      jys[u] = in ? walk.jy + (nax ? i0 : 0) : 0;
      jzs[u] = in ? walk.jz : 0;
      walk.next();
      const int j = (jxs[u] * n1 + jys[u]) * n2 + jzs[u];
      js[u] = j;
      a0[u] = ca[j];
      b0[u] = (order == 2) ? cb[j] : 0.0f;
      a1[u] = a2[u] = b1[u] = b2[u] = 0.0f;
      if (ysw && !corner) {
        const int sx = jxs[u] < P.vneg[0] ? -1 : (jxs[u] >= P.vpos[0] ? 1 : 0);
        const int64_t o1 = -(int64_t)sx * nv;
        a1[u] = ca[j + o1]; a2[u] = ca[j + 2 * o1];
        b1[u] = cb[j + o1]; b2[u] = cb[j + 2 * o1];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (tb + u * step >= nt) continue;
      const int j = js[u], jx = jxs[u], jy = jys[u], jz = jzs[u];
      const double vn = nax ? P.vtab[kMaxAxis + jy] : P.vtab[jx];
      const double an = fabs(vn);
      const double aw = an * ((P.omtab[jx] * P.omtab[kMaxAxis + jy]) * P.omtab[2 * kMaxAxis + jz]);
      double ha = a0[u], hb = b0[u];
      if (ysw) {
        if (corner) {
          ha = xswept_value(P, h, ax_, ay_, j, jx, jy, jz, nwl0, nwr0);
          hb = xswept_value(P, h, bx_, by_, j, jx, jy, jz, nwl1, nwr1);
        } else if (jx < P.vneg[0] || jx >= P.vpos[0]) {
          const float Cx = P.cour[jx], Cx2 = P.cour2[jx];
          ha = bw_update(a0[u], a1[u], a2[u], Cx, Cx2);
          hb = bw_update(b0[u], b1[u], b2[u], Cx, Cx2);
        }
      }
      double hh = ha;
      if (order == 2) {
        const double C = an * P.dt / dl;
        hh = ha + 0.5 * (1.0 - C) * (ha - hb);
      }
      b += aw * hh;
    }
  }
  return b;
}

// Face densities n_w = (A_w + eps B) / D_w, one workgroup per face, faces
// numbered left[ny], right[ny], bottom[nx], top[nx].  PHASE 0 handles the x
// faces (and, for order 1, the y faces too); PHASE 1 the y faces of order
// 2, whose face values come from the x-swept boundary rows and therefore
// need the x-face densities of the previous launch.  Cavity problems only.
constexpr int kWallBlock = 1024;

// Wall (and face position) of face f, faces numbered left[ny], right[ny],
// bottom[nx], top[nx].
__device__ __forceinline__ void face_of(const Params& P, int f, int& wall, int& pos) {
  if (f < P.ny) { wall = WALL_LEFT; pos = f; }
  else if (f < 2 * P.ny) { wall = WALL_RIGHT; pos = f - P.ny; }
  else if (f < 2 * P.ny + P.nx) { wall = WALL_BOTTOM; pos = f - 2 * P.ny; }
  else { wall = WALL_TOP; pos = f - 2 * P.ny - P.nx; }
}

template <int PHASE>
__device__ __forceinline__ void wall_face(const Params& P, const float* __restrict__ h, int f, double* red) {
  int wall, pos;
  face_of(P, f, wall, pos);
  double nwl0 = 0.0, nwl1 = 0.0, nwr0 = 0.0, nwr1 = 0.0;
  if (PHASE == 1) {
    const int ra = (wall == WALL_BOTTOM) ? 0 : P.ny - 1;
    const int rb = (wall == WALL_BOTTOM) ? 1 : P.ny - 2;
    nwl0 = P.nw[ra];
    nwl1 = P.nw[rb];
    nwr0 = P.nw[P.ny + ra];
    nwr1 = P.nw[P.ny + rb];
  }
  double s[1] = {face_b<8>(P, h, wall, pos, P.order, nwl0, nwl1, nwr0, nwr1, (int)threadIdx.x, kWallBlock)};
  block_sum<1>(s, red);
  if (threadIdx.x == 0) {
    const double* k = wall_consts(P, wall, pos);
    P.nw[f] = (k[0] + P.eps * s[0]) / k[1];
  }
}

template <int PHASE>
__global__ __launch_bounds__(kWallBlock) void wall_kernel(Params P, const float* __restrict__ h, int nface,
                                                          int per_xcd) {
  __shared__ double red[kWallBlock / 64];
  // neighbouring faces (which read overlapping cells) on the same XCD
  int f = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (f >= nface) return;
  if (PHASE == 1) f += 2 * P.ny;
  wall_face<PHASE>(P, h, f, red);
}

// The faces of every problem of a batch in one launch (start: first face of
// each problem in this launch; PHASE 1 numbers a problem's y faces from 0).
template <int PHASE>
__global__ __launch_bounds__(kWallBlock) void wall_batch_kernel(const BatchCav* __restrict__ cavs,
                                                                const int* __restrict__ start, int count,
                                                                const float* __restrict__ h, int per_xcd) {
  __shared__ double red[kWallBlock / 64];
  const int u = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (u >= start[count]) return;
  const int c = find_cav(start, count, u);
  const Params& P = cavs[c].P;
  int f = u - start[c];
  if (PHASE == 1) f += 2 * P.ny;
  wall_face<PHASE>(P, h + cavs[c].hoff, f, red);
}

// ------------------------------------------------------------------- S2 --
constexpr int kTX = 8, kTY = 8, kJ = 32, kStreamBlock = 256;

__device__ __forceinline__ int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// One workgroup: an 8x8 tile of cells and a chunk of 32 consecutive
// velocities.  The (8 + 2H)^2 x 32 block (H = order) is staged in LDS with
// 16-byte loads, but only on the upwind sides that the chunk's velocities
// need (jx, and within one jx also jy, increase with j, so the extreme nodes
// of the chunk decide).  Cells outside the cavity take the re-emitted value
// of the wall they lie beyond.  Order 2: the x sweep of every tile row
// (y-halo rows included) goes to a second LDS buffer, then the y sweep.
// STRETCH (order 1 only): Courant numbers of each cell from its own
// lengths, |v| dt / dx_i and |v| dt / dy_j (stretched spatial cells).
template <int ORDER, bool STRETCH = false>
__global__ __launch_bounds__(kStreamBlock) void stream_kernel(Params P, const float* __restrict__ hin,
                                                              float* __restrict__ hout, int tiles_x,
                                                              int tiles_y, int nchunks, int per_xcd) {
  static_assert(!STRETCH || ORDER == 1, "stretched spatial cells stream at first order");
  constexpr int H = ORDER;
  constexpr int AX = kTX + 2 * H, AY = kTY + 2 * H;
  constexpr int Q = kJ / 4;  // float4 per cell and chunk
  __shared__ float4 A4[AY * AX * Q];
  __shared__ float B[(ORDER == 2) ? AY * kTX * kJ : 1];
  float* A = reinterpret_cast<float*>(A4);
  // XCD-aware order: workgroups are dealt round-robin to the 8 XCDs; give
  // each XCD a contiguous range of (chunk, tile) units so that neighbouring
  // tiles (which share halos) run on the same L2.
  const int ntiles = tiles_x * tiles_y;
  const int total = ntiles * nchunks;
  const int unit = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (unit >= total) return;
  const int chunk = unit / ntiles, tile = unit % ntiles;
  const int ix0 = (tile % tiles_x) * kTX, iy0 = (tile / tiles_x) * kTY;
  const int j0 = chunk * kJ;
  const int nx = P.nx, ny = P.ny, nv = P.nv;
  const int n1 = P.n[1], n2 = P.n[2];
  const bool periodic = (P.bc == 1);
  // upwind sides needed by this chunk
  const int jlast = min(j0 + kJ, nv) - 1;
  int fx, fy, fz, lx, ly, lz;
  node_decode(j0, n1, n2, fx, fy, fz);
  node_decode(jlast, n1, n2, lx, ly, lz);
  const bool needL = P.vtab[lx] > 0.0, needR = P.vtab[fx] < 0.0;
  const bool oneX = (fx == lx);
  const bool needB = !oneX || P.vtab[kMaxAxis + ly] > 0.0;  // v_y > 0 reads cells below
  const bool needT = !oneX || P.vtab[kMaxAxis + fy] < 0.0;
  const int c_lo = needL ? 0 : H, c_hi = needR ? AX : AX - H;
  const int r_lo = needB ? 0 : H, r_hi = needT ? AY : AY - H;
  // ---- stage the block (16-byte loads; ghosts per component)
  const bool vec = (nv & 3) == 0;
  {
    const int q = threadIdx.x % Q;
    const int jq = j0 + 4 * q;
    for (int cidx = threadIdx.x / Q; cidx < AY * AX; cidx += kStreamBlock / Q) {
      const int r = cidx / AX, c = cidx % AX;
      if (r < r_lo || r >= r_hi || c < c_lo || c >= c_hi) continue;
      const int iy = iy0 - H + r, ix = ix0 - H + c;
      const bool inY = iy >= 0 && iy < ny, inX = ix >= 0 && ix < nx;
      float v4[4] = {0.f, 0.f, 0.f, 0.f};
      if (periodic || (inX && inY)) {
        const int64_t base = cell_off(P, periodic ? wrapi(ix, nx) : ix, periodic ? wrapi(iy, ny) : iy);
        if (vec && jq + 3 < nv) {
          const float4 t = *reinterpret_cast<const float4*>(hin + base + jq);
          v4[0] = t.x; v4[1] = t.y; v4[2] = t.z; v4[3] = t.w;
        } else {
          for (int e = 0; e < 4; ++e)
            if (jq + e < nv) v4[e] = hin[base + jq + e];
        }
      } else if (inY || (ORDER == 1 && inX)) {
        int wall;
        double nwv;
        if (inY) {
          wall = ix < 0 ? WALL_LEFT : WALL_RIGHT;
          nwv = P.nw[(wall == WALL_LEFT ? 0 : ny) + iy];
        } else {
          wall = iy < 0 ? WALL_BOTTOM : WALL_TOP;
          nwv = P.nw[2 * ny + (wall == WALL_BOTTOM ? 0 : nx) + ix];
        }
        for (int e = 0; e < 4; ++e)
          if (jq + e < nv) v4[e] = ghost_value(nwv, ratio_row(P, wall, inY ? iy : ix)[jq + e], P.inv_eps);
      }
      A4[cidx * Q + q] = make_float4(v4[0], v4[1], v4[2], v4[3]);
    }
  }
  const int jj = threadIdx.x & (kJ - 1);
  const int j = j0 + jj;
  const bool jok = j < nv;
  int jx = 0, jy = 0, jz = 0;
  if (jok) node_decode(j, n1, n2, jx, jy, jz);
  const double vx = P.vtab[jx], vy = P.vtab[kMaxAxis + jy];
  const int sx = vx > 0.0 ? 1 : (vx < 0.0 ? -1 : 0);
  const int sy = vy > 0.0 ? 1 : (vy < 0.0 ? -1 : 0);
  const float Cx = P.cour[jx], Cx2 = P.cour2[jx];
  const float Cy = P.cour[kMaxAxis + jy], Cy2 = P.cour2[kMaxAxis + jy];
  const int rstep = kStreamBlock / kJ;  // 8 tile cells per pass
  __syncthreads();
  if (ORDER == 2) {
    // ---- x sweep of the tile rows that the y sweep reads
    for (int cidx = threadIdx.x / kJ; cidx < AY * kTX; cidx += rstep) {
      const int r = cidx / kTX, c = cidx % kTX;
      if (r < r_lo || r >= r_hi) continue;
      const int iy = iy0 - 2 + r, ix = ix0 + c;
      float val = 0.0f;
      if (jok && ix < nx) {
        if (!periodic && (iy < 0 || iy >= ny)) {
          const int wall = iy < 0 ? WALL_BOTTOM : WALL_TOP;
          val = ghost_value(P.nw[2 * ny + (wall == WALL_BOTTOM ? 0 : nx) + ix], ratio_row(P, wall, ix)[j],
                            P.inv_eps);
        } else {
          const float* row = &A[(r * AX + c + 2) * kJ + jj];
          const float h0 = row[0];
          val = (sx == 0) ? h0 : bw_update(h0, row[-sx * kJ], row[-2 * sx * kJ], Cx, Cx2);
        }
      }
      B[cidx * kJ + jj] = val;
    }
    __syncthreads();
    // ---- y sweep and store
    for (int cidx = threadIdx.x / kJ; cidx < kTY * kTX; cidx += rstep) {
      const int r = cidx / kTX, c = cidx % kTX;
      const int iy = iy0 + r, ix = ix0 + c;
      if (!jok || ix >= nx || iy >= ny) continue;
      const float* col = &B[((r + 2) * kTX + c) * kJ + jj];
      const float h0 = col[0];
      const float out = (sy == 0) ? h0 : bw_update(h0, col[-sy * kTX * kJ], col[-2 * sy * kTX * kJ], Cy, Cy2);
      hout[cell_off(P, ix, iy) + j] = out;
    }
  } else {
    for (int cidx = threadIdx.x / kJ; cidx < kTY * kTX; cidx += rstep) {
      const int r = cidx / kTX, c = cidx % kTX;
      const int iy = iy0 + r, ix = ix0 + c;
      if (!jok || ix >= nx || iy >= ny) continue;
      const float* ctr = &A[((r + 1) * AX + c + 1) * kJ + jj];
      const float h0 = ctr[0];
      const float hxn = (sx == 0) ? h0 : ctr[-sx * kJ];
      const float hyn = (sy == 0) ? h0 : ctr[-sy * AX * kJ];
      float cx = Cx, cy = Cy;
      if (STRETCH) {
        cx = (float)(fabs(vx) * P.dt * P.inv_wx[ix]);
        cy = (float)(fabs(vy) * P.dt * P.inv_wy[iy]);
      }
      hout[cell_off(P, ix, iy) + j] = h0 + cx * (hxn - h0) + cy * (hyn - h0);
    }
  }
}

// Vector form of the stream kernel for velocity grids with n_z % 4 == 0
// (then every aligned group of four consecutive velocities shares (jx, jy):
// one sign and one Courant number per axis).  One workgroup: 16 x 8 cells
// and 32 velocities; thread (column c, group q) owns four velocities of one
// column.  The raw block with its upwind halo is staged in LDS; each thread
// then x-sweeps the rows of its column into registers and applies the y
// sweep from that register window (order 2), or the unsplit first-order
// stencil (order 1).  Same arithmetic per element as stream_kernel.  The
// tile shape TX x TY is a template parameter (16 x 8 for single problems;
// batches also offer 32 x 4, chosen by boltz_batch_tune); TX * 8 threads.
constexpr int kTX4 = 16, kTY4 = 8, kJ4 = 32, kStream4Block = kTX4 * (kJ4 / 4);
constexpr int kTX4b = 32, kTY4b = 4;
// Consecutive velocity chunks of one tile that are adjacent work units (at
// most kChunkGroup, at most the problem's chunk count): each cell is then
// read in runs of up to 2 KB rather than 128 B, about 10% faster on the
// 64x64 cavity than one chunk per group.
constexpr int kChunkGroup = 16;

__host__ __device__ inline int stream4_group(int nv) {
  const int nchunks = (nv + kJ4 - 1) / kJ4;
  return nchunks < kChunkGroup ? nchunks : kChunkGroup;
}

// work units of one problem: tiles x velocity chunks, rounded up to whole
// chunk groups
__host__ __device__ inline int64_t stream4_units(int nx, int ny, int nv, int tx = kTX4, int ty = kTY4) {
  const int64_t tiles = (int64_t)((nx + tx - 1) / tx) * ((ny + ty - 1) / ty);
  const int cg = stream4_group(nv);
  const int64_t groups = ((nv + kJ4 - 1) / kJ4 + cg - 1) / cg;
  return tiles * groups * cg;
}

// a / b for 0 <= a < 2^24, 0 < b < 2^12: the float quotient is within one
// of the truth, then corrected.
__device__ __forceinline__ int div_small(int a, int b) {
  int t = (int)((float)a * __frcp_rn((float)b));
  t -= (t * b > a) ? 1 : 0;
  t += ((t + 1) * b <= a) ? 1 : 0;
  return t;
}

__device__ __forceinline__ float4 ghost4(double nwv, const double* R, double inv_eps) {
  return make_float4(ghost_value(nwv, R[0], inv_eps), ghost_value(nwv, R[1], inv_eps),
                     ghost_value(nwv, R[2], inv_eps), ghost_value(nwv, R[3], inv_eps));
}

__device__ __forceinline__ float4 bw4(float4 h0, float4 h1, float4 h2, float C, float c2) {
  return make_float4(bw_update(h0.x, h1.x, h2.x, C, c2), bw_update(h0.y, h1.y, h2.y, C, c2),
                     bw_update(h0.z, h1.z, h2.z, C, c2), bw_update(h0.w, h1.w, h2.w, C, c2));
}

template <int ORDER, int TX = kTX4, int TY = kTY4>
struct Stream4LDS {
  static constexpr int AX = TX + 2 * ORDER, AY = TY + 2 * ORDER, Q = kJ4 / 4;
  float4 a[AY * AX * Q];
};

// Work unit `unit` (a chunk of 32 velocities of one 16 x 8 tile of cells)
// of one problem; tiles_x = ceil(nx / 16), tiles_y = ceil(ny / 8).  Units
// run chunk-group-major over the tiles, so that neighbouring tiles (which
// share halos) follow each other; within a group, stream4_group(nv)
// consecutive chunks of one tile.
template <int ORDER, int TX = kTX4, int TY = kTY4>
__device__ __forceinline__ void stream4_unit(const Params& P, const float* __restrict__ hin, float* __restrict__ hout,
                                             int tiles_x, int tiles_y, int unit, float4* A4) {
  constexpr int H = ORDER;
  constexpr int AX = TX + 2 * H, AY = TY + 2 * H;
  constexpr int NT = TX * (kJ4 / 4);
  constexpr int Q = kJ4 / 4;
  const int ntiles = tiles_x * tiles_y;
  const int gsz = stream4_group(P.nv);
  const int per_group = ntiles * gsz;
  const int cg = unit / per_group, rem = unit - (unit / per_group) * per_group;
  const int tile = rem / gsz, chunk = cg * gsz + (rem - (rem / gsz) * gsz);
  if (chunk * kJ4 >= P.nv) return;  // padding unit of the last group
  const int ix0 = (tile % tiles_x) * TX, iy0 = (tile / tiles_x) * TY;
  const int j0 = chunk * kJ4;
  const int nx = P.nx, ny = P.ny, nv = P.nv;
  const int n1 = P.n[1], n2 = P.n[2];
  const bool periodic = (P.bc == 1);
  const int jlast = min(j0 + kJ4, nv) - 1;
  int fx, fy, fz, lx, ly, lz;
  node_decode(j0, n1, n2, fx, fy, fz);
  node_decode(jlast, n1, n2, lx, ly, lz);
  const bool needL = P.vtab[lx] > 0.0, needR = P.vtab[fx] < 0.0;
  const bool oneX = (fx == lx);
  const bool needB = !oneX || P.vtab[kMaxAxis + ly] > 0.0;
  const bool needT = !oneX || P.vtab[kMaxAxis + fy] < 0.0;
  const int c_lo = needL ? 0 : H, c_hi = needR ? AX : AX - H;
  const int r_lo = needB ? 0 : H, r_hi = needT ? AY : AY - H;
  // ---- stage the block; outside the cavity: the wall's re-emitted values.
  // All loads of a thread are issued before its LDS stores (fixed trip
  // count), so their latencies overlap.
  {
    constexpr int kRows = NT / Q;                            // cells per pass
    constexpr int kIter = (AY * AX + kRows - 1) / kRows;     // passes
    const int q = threadIdx.x % Q;
    const int jq = j0 + 4 * q;
    // the block's corner cell (ix0 - H, iy0 - H) at this thread's velocity
    // (an address only: corner cells outside the cavity are never read)
    const int row_stride = nx * nv;
    const float* corner = hin + ((int64_t)(iy0 - H) * nx + (ix0 - H)) * nv + jq;
    float4 v[kIter];
#pragma unroll
    for (int it = 0; it < kIter; ++it) {
      const int cidx = threadIdx.x / Q + it * kRows;
      v[it] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (cidx >= AY * AX) continue;
      const int r = cidx / AX, c = cidx - r * AX;
      if (r < r_lo || r >= r_hi || c < c_lo || c >= c_hi || jq >= nv) continue;
      const int iy = iy0 - H + r, ix = ix0 - H + c;
      const bool inY = iy >= 0 && iy < ny, inX = ix >= 0 && ix < nx;
      if (periodic) {
        const int64_t base = cell_off(P, wrapi(ix, nx), wrapi(iy, ny));
        v[it] = *reinterpret_cast<const float4*>(hin + base + jq);
      } else if (inX && inY) {
        // 32-bit offset from the tile's corner (r, c >= 0, within 12 rows)
        v[it] = *reinterpret_cast<const float4*>(corner + (r * row_stride + c * nv));
      } else if (inY || (ORDER == 1 && inX)) {
        int wall;
        double nwv;
        if (inY) {
          wall = ix < 0 ? WALL_LEFT : WALL_RIGHT;
          nwv = P.nw[(wall == WALL_LEFT ? 0 : ny) + iy];
        } else {
          wall = iy < 0 ? WALL_BOTTOM : WALL_TOP;
          nwv = P.nw[2 * ny + (wall == WALL_BOTTOM ? 0 : nx) + ix];
        }
        v[it] = ghost4(nwv, ratio_row(P, wall, inY ? iy : ix) + jq, P.inv_eps);
      }
    }
#pragma unroll
    for (int it = 0; it < kIter; ++it) {
      const int cidx = threadIdx.x / Q + it * kRows;
      if (cidx < AY * AX) A4[cidx * Q + q] = v[it];
    }
  }
  const int q = threadIdx.x % Q, c = threadIdx.x / Q;
  const int jq = j0 + 4 * q;
  const int ix = ix0 + c;
  const bool ok = jq < nv && ix < nx;
  // velocity row (jx, jy) of this thread's quadruple, by a float reciprocal
  // (exact after one correction for the node counts here, < 2^24)
  int jx = 0, jy = 0;
  if (jq < nv) {
    const int row = div_small(jq, n2);
    jx = div_small(row, n1);
    jy = row - jx * n1;
  }
  const double vx = P.vtab[jx], vy = P.vtab[kMaxAxis + jy];
  const int sx = vx > 0.0 ? 1 : (vx < 0.0 ? -1 : 0);
  const int sy = vy > 0.0 ? 1 : (vy < 0.0 ? -1 : 0);
  const float Cx = P.cour[jx], Cx2 = P.cour2[jx];
  const float Cy = P.cour[kMaxAxis + jy], Cy2 = P.cour2[kMaxAxis + jy];
  __syncthreads();
  if (!ok) return;
  if (ORDER == 2) {
    // x-swept rows iy0 - 2 .. iy0 + TY + 1 of this column (only the rows
    // on the upwind side in y are formed)
    float4 hx[AY];
    const int xc = c + 2;
#pragma unroll
    for (int r = 0; r < AY; ++r) {
      hx[r] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (r < r_lo || r >= r_hi) continue;
      const int iy = iy0 - 2 + r;
      if (!periodic && (iy < 0 || iy >= ny)) {
        const int wall = iy < 0 ? WALL_BOTTOM : WALL_TOP;
        hx[r] = ghost4(P.nw[2 * ny + (wall == WALL_BOTTOM ? 0 : nx) + ix], ratio_row(P, wall, ix) + jq,
                       P.inv_eps);
      } else {
        const float4* row = &A4[(r * AX + xc) * Q + q];
        const float4 h0 = row[0];
        hx[r] = (sx == 0) ? h0 : bw4(h0, row[-sx * Q], row[-2 * sx * Q], Cx, Cx2);
      }
    }
    float* dst = hout + jq;
#pragma unroll
    for (int r = 0; r < TY; ++r) {
      const int iy = iy0 + r;
      if (iy >= ny) break;
      const float4 h0 = hx[r + 2];
      // the upwind neighbours are selected first (the sign of v_y varies
      // across the lanes of a wavefront), then one update is evaluated
      const float4 h1 = sy > 0 ? hx[r + 1] : hx[r + 3], h2 = sy > 0 ? hx[r] : hx[r + 4];
      const float4 out = (sy == 0) ? h0 : bw4(h0, h1, h2, Cy, Cy2);
      nt_store4(dst + cell_off(P, ix, iy), out);
    }
  } else {
    float* dst = hout + jq;
    // stretched spatial cells: the Courant numbers of each cell from its
    // own lengths
    const bool str = P.inv_wx != nullptr;
    const float cx = str ? (float)(fabs(vx) * P.dt * P.inv_wx[ix]) : Cx;
    const double avy = fabs(vy) * P.dt;
#pragma unroll
    for (int r = 0; r < TY; ++r) {
      const int iy = iy0 + r;
      if (iy >= ny) break;
      const float cy = str ? (float)(avy * P.inv_wy[iy]) : Cy;
      const float4* ctr = &A4[((r + 1) * AX + c + 1) * Q + q];
      const float4 h0 = ctr[0];
      const float4 hxn = (sx == 0) ? h0 : ctr[-sx * Q];
      const float4 hyn = (sy == 0) ? h0 : ctr[-sy * AX * Q];
      float4 out;
      out.x = h0.x + cx * (hxn.x - h0.x) + cy * (hyn.x - h0.x);
      out.y = h0.y + cx * (hxn.y - h0.y) + cy * (hyn.y - h0.y);
      out.z = h0.z + cx * (hxn.z - h0.z) + cy * (hyn.z - h0.z);
      out.w = h0.w + cx * (hxn.w - h0.w) + cy * (hyn.w - h0.w);
      nt_store4(dst + cell_off(P, ix, iy), out);
    }
  }
}

template <int ORDER>
__global__ __launch_bounds__(kStream4Block) void stream4_kernel(Params P, const float* __restrict__ hin,
                                                                float* __restrict__ hout, int tiles_x,
                                                                int tiles_y, int nunits, int per_xcd) {
  __shared__ Stream4LDS<ORDER> L;
  // XCD-aware order: contiguous (chunk, tile) ranges per XCD
  const int unit = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (unit >= nunits) return;
  stream4_unit<ORDER>(P, hin, hout, tiles_x, tiles_y, unit, L.a);
}

// Every problem of a batch in one launch (start: first unit of each problem;
// all problems have n_z % 4 == 0 and the same order).
template <int ORDER, int TX, int TY>
__global__ __launch_bounds__(TX * (kJ4 / 4)) void stream4_batch_kernel(const BatchCav* __restrict__ cavs,
                                                                       const int* __restrict__ start, int count,
                                                                       const float* __restrict__ hin,
                                                                       float* __restrict__ hout, int per_xcd) {
  __shared__ Stream4LDS<ORDER, TX, TY> L;
  const int u = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (u >= start[count]) return;
  const int c = find_cav(start, count, u);
  const Params& P = cavs[c].P;
  const int tiles_x = (P.nx + TX - 1) / TX, tiles_y = (P.ny + TY - 1) / TY;
  stream4_unit<ORDER, TX, TY>(P, hin + cavs[c].hoff, hout + cavs[c].hoff, tiles_x, tiles_y, u - start[c], L.a);
}

}  // namespace boltz

#include "collide.hpp"

namespace boltz {

// ------------------------------------------------------------------- S6 --
// One workgroup per cell.  The 11 sums w h {1, v, |v|^2, v_i v_k} come from
// z moments Z_p = sum_z omega_z v_z^p h (p <= 2) of each velocity row (one
// row per thread, the factors omega_z v_z^p from the table zmom through
// scalar loads, rows read four nodes at a time when nv_z % 4 == 0), then
// the row's terms: W = omega_x omega_y, a = v_x, b = v_y.
constexpr int kMomentsBlock = 512;

__global__ __launch_bounds__(kMomentsBlock) void moments_kernel(Params P, WallArgs W, const float* __restrict__ h,
                                                                double* __restrict__ mom, int want_lid) {
  __shared__ double red[20 * (kMomentsBlock / 64)];
  const int nv = P.nv, n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
  // the top row first: its workgroups also sum the lid face (longer), so
  // they start before the others rather than trail them
  const int64_t ncells = (int64_t)P.nx * P.ny;
  const int64_t cell = ((int64_t)blockIdx.x + (int64_t)(P.ny - 1) * P.nx) % ncells;
  const float* src = h + cell * nv;
  const const_f64* zc = (const const_f64*)P.zmom;
  const bool vec = (n2 & 3) == 0 && ((reinterpret_cast<uintptr_t>(src) & 15) == 0);
  double s[11];
#pragma unroll
  for (int i = 0; i < 11; ++i) s[i] = 0.0;
  for (int row = threadIdx.x; row < n0 * n1; row += kMomentsBlock) {
    const int jx = row / n1, jy = row - (row / n1) * n1;
    double Z0 = 0.0, Z1 = 0.0, Z2 = 0.0;
    auto node = [&](int jz, float hv) {
      const const_f64* z = zc + 8 * jz;
      const double x = (double)hv;
      Z0 = fma(z[0], x, Z0);
      Z1 = fma(z[1], x, Z1);
      Z2 = fma(z[2], x, Z2);
    };
    if (vec) {
      const f32x4* r4 = reinterpret_cast<const f32x4*>(src + row * n2);
      for (int q = 0; q < (n2 >> 2); ++q) {
        const f32x4 v = r4[q];
        node(4 * q, v.x);
        node(4 * q + 1, v.y);
        node(4 * q + 2, v.z);
        node(4 * q + 3, v.w);
      }
    } else {
      for (int jz = 0; jz < n2; ++jz) node(jz, src[row * n2 + jz]);
    }
    const double Wr = P.omtab[jx] * P.omtab[kMaxAxis + jy], a = P.vtab[jx], b = P.vtab[kMaxAxis + jy];
    const double T0 = Wr * Z0, T1 = Wr * Z1;
    s[0] += T0;
    s[1] += a * T0;
    s[2] += b * T0;
    s[3] += T1;
    s[5] += (a * a) * T0;
    s[6] += (a * b) * T0;
    s[7] += a * T1;
    s[8] += (b * b) * T0;
    s[9] += b * T1;
    s[10] += Wr * Z2;
  }
  s[4] = (s[5] + s[8]) + s[10];
  {
    // block sums through the 20-value wavefront fold (lanes 0..10 of
    // wavefront 0 receive the totals), then broadcast in wavefront 0
    double v[20];
#pragma unroll
    for (int i = 0; i < 20; ++i) v[i] = i < 11 ? s[i] : 0.0;
    const int rows = n0 * n1;
    const int nwd = rows >= kMomentsBlock ? kMomentsBlock / 64 : (rows + 63) / 64;
    const double t = block_sum20_w0<kMomentsBlock>(v, red, nwd);
    if (threadIdx.x < 64) {
#pragma unroll
      for (int i = 0; i < 11; ++i) s[i] = lane_value(t, i);
    }
  }
  if (threadIdx.x == 0) {
    // V0 units: n = 1 + eps rho, u = U/n, theta = ((2/3)E - rho)/n - (2/3) eps |u|^2,
    // Pi_ij = 2 P_ij - 2 eps n u_i u_j
    const double eps = P.eps;
    const double rho = s[0], n = 1.0 + eps * rho;
    const double u[3] = {s[1] / n, s[2] / n, s[3] / n};
    const double uu = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
    double* o = mom + cell * 11;
    o[0] = rho;
    o[1] = u[0];
    o[2] = u[1];
    o[3] = u[2];
    o[4] = ((2.0 / 3.0) * s[4] - rho) / n - (2.0 / 3.0) * eps * uu;
    const int ik[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    for (int k = 0; k < 6; ++k) o[5 + k] = 2.0 * s[5 + k] - 2.0 * eps * n * u[ik[k][0]] * u[ik[k][1]];
  }
  const int iy = (int)(cell / P.nx), ix = (int)(cell % P.nx);
  if (want_lid && iy == P.ny - 1) {
    // lid face: gas-side values of this top cell for v_y > 0, wall emission
    // with the first-order face density for v_y < 0
    __syncthreads();  // red is reused
    const double nwt = face_density(P, h, WALL_TOP, ix, 1, 0, 0, 0, 0, red);
    // Phi_w / Phi0 of the lid from its table (built for these walls; the
    // same values wall_ratio gives)
    const double* R = ratio_row(P, WALL_TOP, ix);
    double pxy[1] = {0.0};
    for (int j = threadIdx.x; j < nv; j += blockDim.x) {
      int jx, jy, jz;
      node_decode(j, n1, n2, jx, jy, jz);
      const double v1 = P.vtab[jx], v2 = P.vtab[kMaxAxis + jy];
      const double w = (P.omtab[jx] * P.omtab[kMaxAxis + jy]) * P.omtab[2 * kMaxAxis + jz];
      double hh = 0.0;
      if (v2 > 0.0) hh = (double)src[j];
      else if (v2 < 0.0) hh = (nwt * R[j] - 1.0) * P.inv_eps;
      pxy[0] += w * v1 * v2 * hh;
    }
    block_sum<1>(pxy, red);
    if (threadIdx.x == 0) P.dpart[ix] = 2.0 * pxy[0];
  }
}

__global__ void lid_reduce_kernel(Params P, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double t = 0.0;
    if (P.wx) {
      // stretched cells: the faces weighted by their lengths
      for (int i = 0; i < P.nx; ++i) t += P.wx[i] * P.dpart[i];
      *out = -t;
    } else {
      for (int i = 0; i < P.nx; ++i) t += P.dpart[i];
      *out = -t / P.nx;
    }
  }
}

}  // namespace boltz
