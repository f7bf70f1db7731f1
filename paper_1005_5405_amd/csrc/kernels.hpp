// kernels.hpp -- HIP kernels of one time-split step (CDNA4 / gfx950).
//
//   wall_kernel      S1  per boundary face: discrete zero-net-flux density n_w
//                        (Sec. 2, Eq. bcMax) and the per-wall ratio table
//                        Phi_w / Phi0 used for the re-emitted values
//   stream_kernel    S2  one HBM pass: (8x8 cells + halo) x 32 velocities per
//                        workgroup staged in LDS; order 1 = Eq. streaming2D,
//                        order 2 = Beam-Warming x sweep then y sweep
//   collide_kernel   S3-S5  one workgroup per spatial cell: the cell's h and
//                        Delta N tiles live in LDS, lanes draw Philox pairs,
//                        gather h_a, h_b and scatter gain/loss with LDS
//                        atomics (Eqs. monteCarloInt, collision_step), then
//                        FP64 moment sums, a 5x5 Cholesky solve and the
//                        correction of Eq. rinorm_a, one coalesced store
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
  int order, bc;
  int64_t n_pairs, sample_group;
  uint32_t key0, key1, cavity, mix16;
  double beta;            // mix16 / 16
  double dt, dx, dy, eps, inv_eps, qfac;
  double a[3], inv_cell[3];
  const double* vtab;     // [3][kMaxAxis] node velocities
  const double* omtab;    // [3][kMaxAxis] per-axis weights omega
  const float* omf;      // [3][kMaxAxis] omega in FP32 (importance weights)
  const float* pphi;      // [3][kMaxAxis] realised per-axis Maxwellian law
  const float* punif;     // [3][kMaxAxis] realised per-axis uniform law
  const uint8_t* icdf;    // [3][kFieldSize] Maxwellian inverse CDF on 12-bit fields
  const float* cour;      // [2][kMaxAxis] Courant number |v| dt / d{x,y}
  const float* cour2;     // [2][kMaxAxis] C (1 - C) / 2
  double* nw;             // [2 ny + 2 nx] face densities: left, right, bottom, top
  double* ratio;          // [4][nv] Phi_w / Phi0 per wall and node
  double* dpart;          // [nx] lid shear partial sums
  uint32_t* status;       // device status bits
};

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

// ------------------------------------------------------------------- S1 --
// x-swept value (order 2) of node j at (ix, iy), read straight from global
// memory; the same FP32 arithmetic as the stream kernel's x sweep.
__device__ float xswept_value(const Params& P, const WallArgs& W, const float* h, int ix, int iy,
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
      const double R = wall_ratio(vx, P.vtab[kMaxAxis + jy], P.vtab[2 * kMaxAxis + jz], 0.0,
                                  W.tau[wall], W.tfac[wall]);
      hn[d - 1] = ghost_value(i < 0 ? nwl : nwr, R, P.inv_eps);
    }
  }
  return bw_update(h0, hn[0], hn[1], P.cour[jx], P.cour2[jx]);
}

// Density n_w of one face.  A = sum_out |v_n| w_j, D = sum over the mirror
// images of the outgoing nodes of |v_n| w R (same order as A, so a wall at
// rest facing h = 0 gives n_w = 1 exactly), B = sum_out |v_n| w_j hhat_j;
// n_w = (A + eps B) / D.  `order` selects the face value: 1 = adjacent cell,
// 2 = Beam-Warming face value, from the x-swept state for y faces.
__device__ double face_density(const Params& P, const WallArgs& W, const float* h, int wall, int pos,
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
  const double Uw = (wall == WALL_TOP) ? W.lid_u : 0.0;
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
      const double R = wall_ratio(P.vtab[mx], P.vtab[kMaxAxis + my], P.vtab[2 * kMaxAxis + jz], Uw,
                                  W.tau[wall], W.tfac[wall]);
      double ha, hb = 0.0;
      if (ysw) {
        ha = xswept_value(P, W, h, ax_, ay_, j, jx, jy, jz, nwl0, nwr0);
        hb = xswept_value(P, W, h, bx_, by_, j, jx, jy, jz, nwl1, nwr1);
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

constexpr int kWallBlock = 512;

// One workgroup per boundary face, faces numbered left[ny], right[ny],
// bottom[nx], top[nx].  PHASE 0 handles the x faces (and, for order 1, the y
// faces too); PHASE 1 the y faces of order 2, whose face values come from
// the x-swept boundary rows and therefore need the x-face densities of the
// previous launch.  The first face of every wall also fills that wall's
// ratio table Phi_w / Phi0 for the stream kernel.  Cavity problems only.
template <int PHASE>
__global__ __launch_bounds__(kWallBlock) void wall_kernel(Params P, WallArgs W, const float* __restrict__ h) {
  __shared__ double red[3 * (kWallBlock / 64)];
  const bool ysplit = (P.order == 2);
  int f = blockIdx.x;
  if (PHASE == 1) f += 2 * P.ny;  // y faces only
  int wall, pos;
  if (f < P.ny) { wall = WALL_LEFT; pos = f; }
  else if (f < 2 * P.ny) { wall = WALL_RIGHT; pos = f - P.ny; }
  else if (f < 2 * P.ny + P.nx) { wall = WALL_BOTTOM; pos = f - 2 * P.ny; }
  else { wall = WALL_TOP; pos = f - 2 * P.ny - P.nx; }
  if (pos == 0) {
    const double Uw = (wall == WALL_TOP) ? W.lid_u : 0.0;
    NodeWalk walk(threadIdx.x, blockDim.x, P.n[1], P.n[2]);
    for (int j = threadIdx.x; j < P.nv; j += blockDim.x, walk.next()) {
      P.ratio[(int64_t)wall * P.nv + j] = wall_ratio(P.vtab[walk.jx], P.vtab[kMaxAxis + walk.jy],
                                                     P.vtab[2 * kMaxAxis + walk.jz], Uw, W.tau[wall],
                                                     W.tfac[wall]);
    }
  }
  double nwl0 = 0.0, nwl1 = 0.0, nwr0 = 0.0, nwr1 = 0.0;
  if (PHASE == 1) {
    // x-wall densities of the two boundary rows next to this y face
    const int ra = (wall == WALL_BOTTOM) ? 0 : P.ny - 1;
    const int rb = (wall == WALL_BOTTOM) ? 1 : P.ny - 2;
    nwl0 = P.nw[ra];
    nwl1 = P.nw[rb];
    nwr0 = P.nw[P.ny + ra];
    nwr1 = P.nw[P.ny + rb];
  }
  const double nwv = face_density(P, W, h, wall, pos, P.order, nwl0, nwl1, nwr0, nwr1, red);
  (void)ysplit;
  if (threadIdx.x == 0) P.nw[f] = nwv;
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
template <int ORDER>
__global__ __launch_bounds__(kStreamBlock) void stream_kernel(Params P, const float* __restrict__ hin,
                                                              float* __restrict__ hout, int tiles_x,
                                                              int tiles_y, int nchunks, int per_xcd) {
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
          if (jq + e < nv) v4[e] = ghost_value(nwv, P.ratio[(int64_t)wall * nv + jq + e], P.inv_eps);
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
          val = ghost_value(P.nw[2 * ny + (wall == WALL_BOTTOM ? 0 : nx) + ix],
                            P.ratio[(int64_t)wall * nv + j], P.inv_eps);
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
      hout[cell_off(P, ix, iy) + j] = h0 + Cx * (hxn - h0) + Cy * (hyn - h0);
    }
  }
}

// --------------------------------------------------------------- S3, S4 --
// LDS copies of the per-axis tables used by the pair sampler.
struct SamplerLDS {
  double* v;        // [n0 + n1 + n2] node velocities
  double* om;       // [n0 + n1 + n2] omega (FP64, moment sums)
  float* omf;       // [n0 + n1 + n2] omega (FP32, weights)
  float* pphi;      // [n0 + n1 + n2]
  float* punif;     // [n0 + n1 + n2]
  uint8_t* icdf;    // [3 * kFieldSize]
};

// w_a / p~_a in FP32: midpoint weight of Phi0 over the probability of drawing
// node (i, j, k) from (1 - beta) Maxwellian law + beta uniform law.
__device__ __forceinline__ float node_ratio(const SamplerLDS& T, float beta, int i, int j, int k, int n0,
                                            int n1) {
  const float w = (T.omf[i] * T.omf[n0 + j]) * T.omf[n0 + n1 + k];
  const float pm = (T.pphi[i] * T.pphi[n0 + j]) * T.pphi[n0 + n1 + k];
  const float pu = (T.punif[i] * T.punif[n0 + j]) * T.punif[n0 + n1 + k];
  return w / ((1.0f - beta) * pm + beta * pu);
}

struct Pair {
  int a, b, as, bs;  // node indices; as = bs = -1 when discarded
  float q;
};

// One Monte Carlo collision sample from one Philox4x32-10 block with counter
// (m, group, step, cavity):
//   r0 = [a_x:12][a_y:12][choice_a:4][choice_b:4]
//   r1 = [a_z:12][b_x:12][phi_hi:8]   r2 = [b_y:12][b_z:12][phi_lo:8]   r3 = u
// nodes from the Maxwellian law, or the uniform law when the choice nibble
// is below mix16; k_z = 2 (r3 + 1/2) 2^-32 - 1, azimuth 2 pi (phi + 1/2) 2^-16;
// v* = v_a + (v_r.k) k, v1* = v_b - (v_r.k) k with v_r = v_b - v_a;
// post-collision cells floor((x + a) n / 2a), discard outside the box;
// q = qfac |v_r.k| (w_a/p~_a)(w_b/p~_b), qfac = dt K / N_t.
__device__ __forceinline__ Pair sample_pair(const Params& P, const SamplerLDS& T, uint32_t group,
                                            uint32_t step, uint32_t m, u32x4* words) {
  const int n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
  const u32x4 c = {m, group, step, P.cavity};
  const u32x4 r = philox4x32_10(c, P.key0, P.key1);
  if (words) words[0] = r;
  const bool ua = ((r.x >> 4) & 15u) < P.mix16;
  const bool ub = (r.x & 15u) < P.mix16;
  const uint32_t fax = r.x >> 20, fay = (r.x >> 8) & 0xFFFu, faz = r.y >> 20;
  const uint32_t fbx = (r.y >> 8) & 0xFFFu, fby = r.z >> 20, fbz = (r.z >> 8) & 0xFFFu;
  const int iax = ua ? uniform_draw(fax, n0) : (int)T.icdf[fax];
  const int iay = ua ? uniform_draw(fay, n1) : (int)T.icdf[kFieldSize + fay];
  const int iaz = ua ? uniform_draw(faz, n2) : (int)T.icdf[2 * kFieldSize + faz];
  const int ibx = ub ? uniform_draw(fbx, n0) : (int)T.icdf[fbx];
  const int iby = ub ? uniform_draw(fby, n1) : (int)T.icdf[kFieldSize + fby];
  const int ibz = ub ? uniform_draw(fbz, n2) : (int)T.icdf[2 * kFieldSize + fbz];
  const uint32_t phi = ((r.y & 0xFFu) << 8) | (r.z & 0xFFu);
  const double u6 = ((double)r.w + 0.5) * 0x1p-32;
  const double u7 = ((double)phi + 0.5) * 0x1p-16;
  const double kz = 2.0 * u6 - 1.0;
  const double s = sqrt((1.0 - kz) * (1.0 + kz));
  double cp, sp;
  cos_sin_2pi(u7, cp, sp);
  const double kx = s * cp, ky = s * sp;
  const double* vx = T.v;
  const double* vy = T.v + n0;
  const double* vz = T.v + n0 + n1;
  const double vax = vx[iax], vay = vy[iay], vaz = vz[iaz];
  const double vbx = vx[ibx], vby = vy[iby], vbz = vz[ibz];
  const double vrx = vbx - vax, vry = vby - vay, vrz = vbz - vaz;
  const double alpha = (vrx * kx + vry * ky) + vrz * kz;
  const double ddx = alpha * kx, ddy = alpha * ky, ddz = alpha * kz;
  const double tsx = floor((vax + ddx + P.a[0]) * P.inv_cell[0]);
  const double tsy = floor((vay + ddy + P.a[1]) * P.inv_cell[1]);
  const double tsz = floor((vaz + ddz + P.a[2]) * P.inv_cell[2]);
  const double ttx = floor((vbx - ddx + P.a[0]) * P.inv_cell[0]);
  const double tty = floor((vby - ddy + P.a[1]) * P.inv_cell[1]);
  const double ttz = floor((vbz - ddz + P.a[2]) * P.inv_cell[2]);
  const bool kept = tsx >= 0.0 && tsx < (double)n0 && tsy >= 0.0 && tsy < (double)n1 && tsz >= 0.0 &&
                    tsz < (double)n2 && ttx >= 0.0 && ttx < (double)n0 && tty >= 0.0 &&
                    tty < (double)n1 && ttz >= 0.0 && ttz < (double)n2;
  Pair p;
  p.a = (iax * n1 + iay) * n2 + iaz;
  p.b = (ibx * n1 + iby) * n2 + ibz;
  if (kept) {
    p.as = ((int)tsx * n1 + (int)tsy) * n2 + (int)tsz;
    p.bs = ((int)ttx * n1 + (int)tty) * n2 + (int)ttz;
    const float beta = (float)P.beta;
    p.q = ((float)(P.qfac * fabs(alpha)) * node_ratio(T, beta, iax, iay, iaz, n0, n1)) *
          node_ratio(T, beta, ibx, iby, ibz, n0, n1);
  } else {
    p.as = -1;
    p.bs = -1;
    p.q = 0.0f;
  }
  return p;
}

// Layout of the dynamic LDS of the collide kernel: h^s and Delta N tiles,
// then the sampler tables.
struct CollideLDS {
  static __host__ __device__ size_t tables_bytes(int nsum) {
    return 2 * (size_t)nsum * sizeof(double) + 3 * (size_t)nsum * sizeof(float) + 3 * kFieldSize;
  }
  static __host__ __device__ size_t bytes(int nv, int nsum) {
    size_t b = 2 * (size_t)nv * sizeof(float);
    b = (b + 7) & ~(size_t)7;
    return b + tables_bytes(nsum);
  }
};

__device__ __forceinline__ void load_sampler_tables(const Params& P, unsigned char* base, SamplerLDS& T) {
  const int n0 = P.n[0], n1 = P.n[1], n2 = P.n[2], ns = n0 + n1 + n2;
  T.v = reinterpret_cast<double*>(base);
  T.om = T.v + ns;
  T.omf = reinterpret_cast<float*>(T.om + ns);
  T.pphi = T.omf + ns;
  T.punif = T.pphi + ns;
  T.icdf = reinterpret_cast<uint8_t*>(T.punif + ns);
  for (int i = threadIdx.x; i < ns; i += blockDim.x) {
    const int k = i < n0 ? 0 : (i < n0 + n1 ? 1 : 2);
    const int o = i - (k == 0 ? 0 : (k == 1 ? n0 : n0 + n1));
    T.v[i] = P.vtab[k * kMaxAxis + o];
    T.om[i] = P.omtab[k * kMaxAxis + o];
    T.omf[i] = P.omf[k * kMaxAxis + o];
    T.pphi[i] = P.pphi[k * kMaxAxis + o];
    T.punif[i] = P.punif[k * kMaxAxis + o];
  }
  const uint32_t* src = reinterpret_cast<const uint32_t*>(P.icdf);
  uint32_t* dst = reinterpret_cast<uint32_t*>(T.icdf);
  for (int i = threadIdx.x; i < 3 * kFieldSize / 4; i += blockDim.x) dst[i] = src[i];
}

// Test hook kernel: the pairs of (cell, step, m0 + i) from the same sampler.
__global__ __launch_bounds__(256) void debug_pairs_kernel(Params P, int64_t cell, uint32_t step, int64_t m0,
                                                          int64_t count, int32_t* idx4, double* q,
                                                          uint32_t* words) {
  extern __shared__ __align__(16) unsigned char dsm[];
  SamplerLDS T;
  load_sampler_tables(P, dsm, T);
  __syncthreads();
  const uint32_t group = (P.sample_group == 0) ? 0u : (uint32_t)(cell / P.sample_group);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    u32x4 w;
    const Pair p = sample_pair(P, T, group, step, (uint32_t)(m0 + i), &w);
    idx4[4 * i + 0] = p.a;
    idx4[4 * i + 1] = p.b;
    idx4[4 * i + 2] = p.as;
    idx4[4 * i + 3] = p.bs;
    q[i] = (double)p.q;
    if (words) {
      words[4 * i + 0] = w.x;
      words[4 * i + 1] = w.y;
      words[4 * i + 2] = w.z;
      words[4 * i + 3] = w.w;
    }
  }
}

// Shared-sample mode (G != 1): one pass draws the N_t pairs of every sample
// group once per step into 16-byte records {a | b << 16, a* | b* << 16,
// q bits, 0}; a discarded pair is stored with a* = a, b* = b and q = 0.
__global__ __launch_bounds__(256) void sample_kernel(Params P, uint32_t step, uint4* __restrict__ table) {
  extern __shared__ __align__(16) unsigned char dsm[];
  SamplerLDS T;
  load_sampler_tables(P, dsm, T);
  __syncthreads();
  const int64_t nt = P.n_pairs;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t group = blockIdx.y;
  if (i >= nt) return;
  const Pair p = sample_pair(P, T, group, step, (uint32_t)i, nullptr);
  uint4 rec;
  rec.x = (uint32_t)p.a | ((uint32_t)p.b << 16);
  rec.y = p.as >= 0 ? ((uint32_t)p.as | ((uint32_t)p.bs << 16)) : rec.x;
  rec.z = __float_as_uint(p.q);
  rec.w = 0u;
  table[(int64_t)group * nt + i] = rec;
}

// ------------------------------------------------------------------- S5 --
// Cholesky solve of the 5x5 SPD system (packed upper triangle of 15 sums).
__device__ bool solve5(const double* S, const double* r, double* x) {
  double M[5][5];
  int t = 0;
  for (int k = 0; k < 5; ++k)
    for (int l = k; l < 5; ++l) {
      M[k][l] = S[t];
      M[l][k] = S[t];
      ++t;
    }
  double L[5][5];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) L[i][j] = 0.0;
  for (int i = 0; i < 5; ++i) {
    for (int j = 0; j <= i; ++j) {
      double s = M[i][j];
      for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
      if (i == j) {
        if (!(s > 0.0)) return false;
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
  return true;
}

// One workgroup per spatial cell (blockIdx.x = cell).  TABLE: the pairs come
// from the records of sample_kernel (cells of one group share them) instead
// of being drawn by the workgroup itself.
template <int BLOCK, bool TABLE>
__global__ __launch_bounds__(BLOCK) void collide_kernel(Params P, const float* __restrict__ hs_g,
                                                        float* __restrict__ hout_g, uint32_t step,
                                                        uint32_t flags, double* __restrict__ defect,
                                                        const uint4* __restrict__ table) {
  extern __shared__ __align__(16) unsigned char dsm[];
  __shared__ double red[20 * (BLOCK / 64)];
  __shared__ double xs[5];
  const int nv = P.nv, n1 = P.n[1], n2 = P.n[2], n0 = P.n[0];
  const int64_t cell = blockIdx.x;
  float* hs = reinterpret_cast<float*>(dsm);
  float* dN = hs + nv;
  size_t off = (2 * (size_t)nv * sizeof(float) + 7) & ~(size_t)7;
  SamplerLDS T;
  load_sampler_tables(P, dsm + off, T);
  const double* om = T.om;
  const float* src = hs_g + cell * nv;
  if ((nv & 3) == 0) {
    const float4* s4 = reinterpret_cast<const float4*>(src);
    float4* h4 = reinterpret_cast<float4*>(hs);
    float4* d4 = reinterpret_cast<float4*>(dN);
    for (int i = threadIdx.x; i < (nv >> 2); i += BLOCK) {
      h4[i] = s4[i];
      d4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  } else {
    for (int i = threadIdx.x; i < nv; i += BLOCK) {
      hs[i] = src[i];
      dN[i] = 0.0f;
    }
  }
  __syncthreads();
  // ---- S3 + S4: Jacobi gain/loss, every sample reads the post-stream h
  const uint32_t group = (P.sample_group == 0) ? 0u : (uint32_t)(cell / P.sample_group);
  const float epsf = (float)P.eps;
  const uint32_t nt = (uint32_t)P.n_pairs;
  if (TABLE) {
    const uint4* rec = table + (int64_t)group * nt;
    for (uint32_t m = threadIdx.x; m < nt; m += BLOCK) {
      const uint4 r = rec[m];
      const int a = (int)(r.x & 0xFFFFu), b = (int)(r.x >> 16);
      const int as = (int)(r.y & 0xFFFFu), bs = (int)(r.y >> 16);
      const float ha = hs[a], hb = hs[b];
      const float g = (ha + hb) + (epsf * ha) * hb;
      const float qg = __uint_as_float(r.z) * g;
      lds_add(&dN[as], qg);
      lds_add(&dN[bs], qg);
      lds_add(&dN[a], -qg);
      lds_add(&dN[b], -qg);
    }
  } else {
    for (uint32_t m = threadIdx.x; m < nt; m += BLOCK) {
      const Pair p = sample_pair(P, T, group, step, m, nullptr);
      if (p.as >= 0) {
        const float ha = hs[p.a], hb = hs[p.b];
        const float g = (ha + hb) + (epsf * ha) * hb;
        const float qg = p.q * g;
        lds_add(&dN[p.as], qg);
        lds_add(&dN[p.bs], qg);
        lds_add(&dN[p.a], -qg);
        lds_add(&dN[p.b], -qg);
      }
    }
  }
  __syncthreads();
  const double* vx = T.v;
  const double* vy = T.v + n0;
  const double* vz = T.v + n0 + n1;
  const double* omx = om;
  const double* omy = om + n0;
  const double* omz = om + n0 + n1;
  const bool correct = !(flags & 1u);
  const double eps = P.eps;
  // ---- S5: h^c = h^s + dN / w, FP64 sums M_kl = sum w F^c psi_k psi_l and
  // r_k = -eps sum psi_k dN; h^c replaces dN in LDS.
  double acc[20];
#pragma unroll
  for (int i = 0; i < 20; ++i) acc[i] = 0.0;
  {
    NodeWalk nw(threadIdx.x, BLOCK, n1, n2);
    for (int j = threadIdx.x; j < nv; j += BLOCK, nw.next()) {
      const int jx = nw.jx, jy = nw.jy, jz = nw.jz;
      const double w = (omx[jx] * omy[jy]) * omz[jz];
      const double dn = (double)dN[j];
      const float hc = (float)((double)hs[j] + dn / w);
      dN[j] = hc;
      if (correct) {
        const double v1 = vx[jx], v2 = vy[jy], v3 = vz[jz];
        const double vv = fma(v1, v1, fma(v2, v2, v3 * v3));
        const double wF = w * fma(eps, (double)hc, 1.0);
        const double psi[5] = {1.0, v1, v2, v3, vv};
        int t = 0;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          const double wk = wF * psi[k];
#pragma unroll
          for (int l = k; l < 5; ++l) acc[t] = fma(wk, psi[l], acc[t]), ++t;
        }
        const double edn = -eps * dn;
#pragma unroll
        for (int k = 0; k < 5; ++k) acc[15 + k] = fma(edn, psi[k], acc[15 + k]);
      }
    }
  }
  if (correct) {
    block_sum<20>(acc, red);
    if (threadIdx.x == 0) {
      double x[5];
      if (!solve5(acc, acc + 15, x)) {
        for (int k = 0; k < 5; ++k) x[k] = 0.0;
        atomicOr(P.status, 1u);
      }
      for (int k = 0; k < 5; ++k) xs[k] = x[k];
    }
  }
  __syncthreads();
  double x[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (correct) {
#pragma unroll
    for (int k = 0; k < 5; ++k) x[k] = xs[k];
  }
  // ---- h^{n+1} = h^c + F^c (x . psi) / eps, one coalesced store
  double dsum[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  bool finite = true;
  float* dst = hout_g + cell * nv;
  NodeWalk nw2(threadIdx.x, BLOCK, n1, n2);
  for (int j = threadIdx.x; j < nv; j += BLOCK, nw2.next()) {
    const int jx = nw2.jx, jy = nw2.jy, jz = nw2.jz;
    const double v1 = vx[jx], v2 = vy[jy], v3 = vz[jz];
    const double vv = fma(v1, v1, fma(v2, v2, v3 * v3));
    const double hc = (double)dN[j];
    float out = (float)hc;
    if (correct) {
      const double xpsi = fma(x[4], vv, fma(x[3], v3, fma(x[2], v2, fma(x[1], v1, x[0]))));
      out = (float)fma(fma(eps, hc, 1.0) * xpsi, P.inv_eps, hc);
    }
    finite = finite && isfinite(out);
    dst[j] = out;
    if (defect) {
      const double w = (omx[jx] * omy[jy]) * omz[jz];
      const double diff = eps * ((double)out - (double)hs[j]) * w;
      dsum[0] += diff;
      dsum[1] += v1 * diff;
      dsum[2] += v2 * diff;
      dsum[3] += v3 * diff;
      dsum[4] += vv * diff;
    }
  }
  if (!finite) atomicOr(P.status, 2u);
  if (defect) {
    block_sum<5>(dsum, red);
    if (threadIdx.x < 5) defect[cell * 5 + threadIdx.x] = dsum[threadIdx.x];
  }
}

// ------------------------------------------------------------------- S6 --
__global__ __launch_bounds__(256) void moments_kernel(Params P, WallArgs W, const float* __restrict__ h,
                                                      double* __restrict__ mom, int want_lid) {
  __shared__ double red[11 * 4];
  const int nv = P.nv, n1 = P.n[1], n2 = P.n[2];
  const int64_t cell = blockIdx.x;
  const float* src = h + cell * nv;
  double s[11];
#pragma unroll
  for (int i = 0; i < 11; ++i) s[i] = 0.0;
  for (int j = threadIdx.x; j < nv; j += blockDim.x) {
    int jx, jy, jz;
    node_decode(j, n1, n2, jx, jy, jz);
    const double v1 = P.vtab[jx], v2 = P.vtab[kMaxAxis + jy], v3 = P.vtab[2 * kMaxAxis + jz];
    const double w = (P.omtab[jx] * P.omtab[kMaxAxis + jy]) * P.omtab[2 * kMaxAxis + jz];
    const double wh = w * (double)src[j];
    s[0] += wh;
    s[1] += wh * v1;
    s[2] += wh * v2;
    s[3] += wh * v3;
    s[4] += wh * ((v1 * v1 + v2 * v2) + v3 * v3);
    s[5] += wh * v1 * v1;
    s[6] += wh * v1 * v2;
    s[7] += wh * v1 * v3;
    s[8] += wh * v2 * v2;
    s[9] += wh * v2 * v3;
    s[10] += wh * v3 * v3;
  }
  block_sum<11>(s, red);
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
    const double nwt = face_density(P, W, h, WALL_TOP, ix, 1, 0, 0, 0, 0, red);
    double pxy[1] = {0.0};
    for (int j = threadIdx.x; j < nv; j += blockDim.x) {
      int jx, jy, jz;
      node_decode(j, n1, n2, jx, jy, jz);
      const double v1 = P.vtab[jx], v2 = P.vtab[kMaxAxis + jy], v3 = P.vtab[2 * kMaxAxis + jz];
      const double w = (P.omtab[jx] * P.omtab[kMaxAxis + jy]) * P.omtab[2 * kMaxAxis + jz];
      double hh = 0.0;
      if (v2 > 0.0) hh = (double)src[j];
      else if (v2 < 0.0)
        hh = (nwt * wall_ratio(v1, v2, v3, W.lid_u, W.tau[WALL_TOP], W.tfac[WALL_TOP]) - 1.0) * P.inv_eps;
      pxy[0] += w * v1 * v2 * hh;
    }
    block_sum<1>(pxy, red);
    if (threadIdx.x == 0) P.dpart[ix] = 2.0 * pxy[0];
  }
}

__global__ void lid_reduce_kernel(Params P, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < P.nx; ++i) t += P.dpart[i];
    *out = -t / P.nx;
  }
}

}  // namespace boltz
