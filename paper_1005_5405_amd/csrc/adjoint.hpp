// adjoint.hpp -- reverse mode of one time-split step on gfx950.
//
// The paper has no adjoint; every kernel here is the transpose of the
// linearisation of the forward kernel it names, for fixed Philox samples:
//   collide_adj_kernel  S3-S5 (forward recomputed per cell in LDS)
//   wall_adj_kernel     S1    adjoint of the face densities n_w and of the
//                             re-emitted ghosts, wall-parameter partials
//   sweep_adj_kernel    S2    Beam-Warming sweep transposed (order 2)
//   order1_adj_kernel   S2    first-order unsplit step transposed
//   lid_adj_kernel      S6    adjoint of the lid shear D
//   grad_reduce_kernel        per-face partials -> parameter gradient
// Adjoints are FP64, cell-major like h.  Wall parameters theta are indexed
//   0 lid_u, 1 tau_left, 2 tau_right, 3 tau_top, 4 + ix: tau of bottom face ix.
#pragma once

#include "kernels.hpp"

namespace boltz {

// -------------------------------------------------------- collision --
// Adjoint of the gain/loss pass: lI is the adjoint of the increment of h
// (FP32 tile).  A sample adds dJ/dg (1 + eps h_b) to the adjoint of h_a and
// dJ/dg (1 + eps h_a) to that of h_b, with
// dJ/dg = k_a* lI_a* + k_b* lI_b* - k_a lI_a - k_b lI_b and the sample's own
// coefficients k (FP32 table records or the FP64 values of the draw).
// FIXED: the terms, divided by the cell's power-of-two scale S (inv_s =
// 1/S), go to the 64-bit fixed-point accumulators acc (large ones to the
// FP32 array ovf) as in the forward pass; else they are added in FP64 to ls
// by compare-and-swap.
template <bool FIXED>
__device__ __forceinline__ void adj_add(double* ls, unsigned long long* acc, float* ovf, int j, double lg,
                                        double inv_s, double f) {
  if (FIXED) lds_add_hybrid(acc, ovf, j, lg * inv_s, f);
  else lds_add_f64(&ls[j], lg * f);
}

template <int BLOCK, bool TABLE, bool FIXED>
__device__ __forceinline__ void gain_loss_adj(const Params& P, const TablesLDS& T, const float* hs,
                                              const float* lI, double* ls, unsigned long long* acc, float* ovf,
                                              double inv_s, uint32_t group, uint32_t step,
                                              const uint2* __restrict__ tidx,
                                              const float4* __restrict__ tcoef) {
  const int tid = threadIdx.x;
  const double eps = P.eps;
  const uint32_t nt = (uint32_t)P.n_pairs;
  if (TABLE) {
    constexpr int PU = 4;
    const uint2* ri = tidx + (int64_t)group * nt;
    const float4* rk = tcoef + (int64_t)group * nt;
    // one pass: PU records per thread; in the masked (last) pass slots past
    // the end of the table load and add nothing
    auto pass = [&](uint32_t m0, const bool masked) {
      uint2 id[PU];
      float4 kk[PU];
      bool ok[PU];
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        const uint32_t m = m0 + u * BLOCK;
        ok[u] = !masked || m < nt;
        id[u] = ok[u] ? ri[m] : make_uint2(0u, 0u);
        kk[u] = ok[u] ? rk[m] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        if (!ok[u]) continue;
        const int a = (int)(id[u].x & 0xFFFFu), b = (int)(id[u].x >> 16);
        const int as = (int)(id[u].y & 0xFFFFu), bs = (int)(id[u].y >> 16);
        const double lg = fma((double)kk[u].x, (double)lI[as], (double)kk[u].y * (double)lI[bs]) -
                          fma((double)kk[u].z, (double)lI[a], (double)kk[u].w * (double)lI[b]);
        const double ha = (double)hs[a], hb = (double)hs[b];
        if (FIXED) {
          // both values first; straight-line adds when the whole wavefront
          // has them in the fixed-point window (a discarded sample adds 0)
          const double ks = lg * inv_s, fa = fma(eps, hb, 1.0), fb = fma(eps, ha, 1.0);
          const long long da = fixed_of(ks, fa), db = fixed_of(ks, fb);
          if (__all(in_fixed_window(da) & in_fixed_window(db))) {
            __hip_atomic_fetch_add(&acc[a], (unsigned long long)da, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_add(&acc[b], (unsigned long long)db, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          } else {
            lds_add_fixed_or(acc, ovf, a, da, ks, fa);
            lds_add_fixed_or(acc, ovf, b, db, ks, fb);
          }
        } else if (lg != 0.0) {
          adj_add<FIXED>(ls, acc, ovf, a, lg, inv_s, fma(eps, hb, 1.0));
          adj_add<FIXED>(ls, acc, ovf, b, lg, inv_s, fma(eps, ha, 1.0));
        }
      }
    };
    uint32_t m0 = tid;
    for (; m0 + (PU - 1) * BLOCK < nt; m0 += PU * BLOCK) pass(m0, false);
    if (m0 < nt) pass(m0, true);
  } else {
    for (uint32_t m = tid; m < nt; m += BLOCK) {
      const Pair p = sample_pair(P, T, group, step, m, nullptr);
      if (p.as >= 0) {
        const double lg = fma(p.kas, (double)lI[p.as], p.kbs * (double)lI[p.bs]) -
                          fma(p.ka, (double)lI[p.a], p.kb * (double)lI[p.b]);
        const double ha = (double)hs[p.a], hb = (double)hs[p.b];
        adj_add<FIXED>(ls, acc, ovf, p.a, lg, inv_s, fma(eps, hb, 1.0));
        adj_add<FIXED>(ls, acc, ovf, p.b, lg, inv_s, fma(eps, ha, 1.0));
      }
    }
  }
}

// Dynamic LDS of the collide adjoint: the collide kernel's fixed-point layout
// (h^s tile, FP32 array, 64-bit accumulators), with FIXED a second FP32
// array (large terms of the adjoint sums), then the tables and the per-axis
// table of y . psi.
__host__ __device__ inline size_t collide_adj_lds(int nv, int ns, bool sampler, bool fixed) {
  return CollideLDS::tile(nv) + CollideLDS::acc(nv, ACC_FIXED) + (fixed ? CollideLDS::tile(nv) : 0) +
         TablesLDS::bytes(ns, sampler) + 8 * (size_t)ns;
}

// static LDS of the collide adjoint (reduction scratch)
__host__ __device__ inline size_t collide_adj_static_lds(int block) {
  return (20 * (size_t)(block / 64) + 20) * sizeof(double);
}

// Reverse mode of collide_kernel: lo = adjoint of h^{n+1}, ls = adjoint of
// h^s (FP64; ls may equal lo, each cell is read before it is written).  Per
// cell the forward pass is recomputed in LDS (h^c and the correction's x);
// then with z_k = sum_j lo_j F^c_j psi_k / eps and M y = z,
//   lhc_j = lo_j (1 + x.psi_j) - eps w_j (y.psi_j)(x.psi_j)   (adjoint of h^c)
//   lI_j  = lhc_j - eps w_j (y.psi_j)      (adjoint of the increment of h)
// and ls = lhc plus the sample terms of gain_loss_adj.  Without the
// correction, or when M is not positive definite (status bit 1, as in the
// forward pass), x = y = 0.  LDS reuse: h^c is overwritten by lI (FP32), the
// forward's fixed-point accumulators by the adjoint sums: FIXED, 64-bit fixed
// point in units of S 2^-32 with S the power of two above the cell's
// max |lhc| (terms of 2^18 S or more in a second FP32 array); else FP64.
template <int BLOCK, bool TABLE, bool FIXED>
__global__ __launch_bounds__(BLOCK) void collide_adj_kernel(Params P, const float* __restrict__ hs_g,
                                                            const double* lo_g, double* ls_g, uint32_t step,
                                                            uint32_t flags, const uint2* __restrict__ tidx,
                                                            const float4* __restrict__ tcoef) {
  extern __shared__ __align__(16) unsigned char dsm[];
  __shared__ double red[20 * (BLOCK / 64)];
  __shared__ double tot[20];
  const int nv = P.nv, n0 = P.n[0], n1 = P.n[1], n2 = P.n[2], ns = n0 + n1 + n2;
  const int64_t ncells = (int64_t)P.nx * P.ny;
  const int tid = threadIdx.x;
  float* hs = reinterpret_cast<float*>(dsm);
  float* accf = reinterpret_cast<float*>(dsm + CollideLDS::tile(nv));
  unsigned long long* acc64 = reinterpret_cast<unsigned long long*>(dsm + 2 * CollideLDS::tile(nv));
  double* lsh = reinterpret_cast<double*>(acc64);
  unsigned char* after = dsm + CollideLDS::tile(nv) + CollideLDS::acc(nv, ACC_FIXED);
  float* ovf = FIXED ? reinterpret_cast<float*>(after) : nullptr;
  unsigned char* tb = after + (FIXED ? CollideLDS::tile(nv) : 0);
  TablesLDS T;
  load_tables(P, tb, !TABLE, T);
  double* yt = reinterpret_cast<double*>(tb + TablesLDS::bytes(ns, !TABLE));
  const double* vx = T.v;
  const double* vy = T.v + n0;
  const double* vz = T.v + n0 + n1;
  const double* omx = T.om;
  const double* omy = T.om + n0;
  const double* omz = T.om + n0 + n1;
  const bool correct = !(flags & 1u);
  const double eps = P.eps;
  // adjoint of h^c at node j = (jx, jy, jz)
  auto lam_hc = [&](double l, int jx, int jy, int jz, double& lI) -> double {
    if (!correct) {
      lI = l;
      return l;
    }
    const double xpsi = (T.xt[jx] + T.xt[n0 + jy]) + T.xt[n0 + n1 + jz];
    const double ypsi = (yt[jx] + yt[n0 + jy]) + yt[n0 + n1 + jz];
    const double ewy = eps * ((omx[jx] * omy[jy]) * omz[jz]) * ypsi;
    const double lhc = fma(l, xpsi, l) - ewy * xpsi;
    lI = lhc - ewy;
    return lhc;
  };
  for (int64_t cell = blockIdx.x; cell < ncells; cell += gridDim.x) {
    const float* src = hs_g + cell * nv;
    const double* lo = lo_g + cell * nv;
    if ((nv & 3) == 0 && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
      const float4* s4 = reinterpret_cast<const float4*>(src);
      float4* d4 = reinterpret_cast<float4*>(hs);
#pragma unroll 4
      for (int j = tid; j < (nv >> 2); j += BLOCK) d4[j] = s4[j];
    } else {
      for (int j = tid; j < nv; j += BLOCK) hs[j] = src[j];
    }
    {
      uint4* z = reinterpret_cast<uint4*>(accf);
      const int nz = (int)(CollideLDS::acc(nv, ACC_FIXED) / 16);
      for (int i = tid; i < nz; i += BLOCK) z[i] = make_uint4(0u, 0u, 0u, 0u);
    }
    __syncthreads();
    // ---- forward: increments and h^c
    const uint32_t group = (P.sample_group == 0) ? 0u : (uint32_t)(cell / P.sample_group);
    gain_loss<BLOCK, TABLE, ACC_FIXED>(P, T, hs, accf, acc64, group, step, tidx, tcoef);
    __syncthreads();
    for (int j = tid; j < nv; j += BLOCK) {
      const double dh = (double)accf[j] + from_fixed(acc64[j]);
      accf[j] = (float)((double)hs[j] + dh);
    }
    if (correct) {
      __syncthreads();
      double acc[20];
      correction_sums<BLOCK>(T, P.zmom, hs, accf, n0, n1, n2, acc);
      block_sum20_lds<BLOCK>(acc, red, tot);
      double zs[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      NodeWalk walk(tid, BLOCK, n1, n2);
      // (unrolled: the global loads of lo of several nodes in flight together)
#pragma unroll 4
      for (int j = tid; j < nv; j += BLOCK, walk.next()) {
        const double u = lo[j] * fma(eps, (double)accf[j], 1.0);
        const double a = vx[walk.jx], b = vy[walk.jy], c = vz[walk.jz];
        zs[0] += u;
        zs[1] += a * u;
        zs[2] += b * u;
        zs[3] += c * u;
        zs[4] += ((a * a + b * b) + c * c) * u;
      }
      block_sum<5, BLOCK>(zs, red);
      if (tid < 64) {
        // wavefront 0: M x = r and M y = z, then x . psi and y . psi per axis
        double M[15], r[5], z[5], x[5], y[5];
#pragma unroll
        for (int k = 0; k < 15; ++k) M[k] = T.m0[k] + eps * tot[k];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          r[k] = -eps * tot[15 + k];
          z[k] = zs[k] * P.inv_eps;
        }
        const bool ok = solve5(M, r, x);
        solve5(M, z, y);
        if (!ok) {
#pragma unroll
          for (int k = 0; k < 5; ++k) x[k] = y[k] = 0.0;
          if (tid == 0) atomicOr(P.status, 1u);
        }
        for (int i = tid; i < ns; i += 64) {
          const double v = T.v[i], v2 = v * v;
          T.xt[i] = i < n0 ? x[1] * v + x[4] * v2 : (i < n0 + n1 ? x[2] * v + x[4] * v2 : x[0] + x[3] * v + x[4] * v2);
          yt[i] = i < n0 ? y[1] * v + y[4] * v2 : (i < n0 + n1 ? y[2] * v + y[4] * v2 : y[0] + y[3] * v + y[4] * v2);
        }
      }
      __syncthreads();
    }
    // ---- adjoints of h^c and of the increment (each thread its own nodes)
    double scale = 1.0, inv_scale = 1.0;
    {
      double mx = 0.0;
      NodeWalk walk(tid, BLOCK, n1, n2);
#pragma unroll 4
      for (int j = tid; j < nv; j += BLOCK, walk.next()) {
        double lI;
        const double lhc = lam_hc(lo[j], walk.jx, walk.jy, walk.jz, lI);
        accf[j] = (float)lI;
        if (FIXED) {
          acc64[j] = 0ull;
          ovf[j] = 0.0f;
          mx = fmax(mx, fabs(lhc));
        } else {
          lsh[j] = lhc;
        }
      }
      if (FIXED) {
        // S = 2^e > max |lhc| of the cell (1 for an all-zero or non-finite cell)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
        if ((tid & 63) == 0) red[tid >> 6] = mx;
      }
    }
    __syncthreads();
    if (FIXED) {
      double mx = 0.0;
      for (int w = 0; w < BLOCK / 64; ++w) mx = fmax(mx, red[w]);
      if (mx > 0.0 && isfinite(mx)) {
        const int e = ilogb(mx) + 1;
        scale = ldexp(1.0, e);
        inv_scale = ldexp(1.0, -e);
      }
    }
    gain_loss_adj<BLOCK, TABLE, FIXED>(P, T, hs, accf, lsh, acc64, ovf, inv_scale, group, step, tidx, tcoef);
    __syncthreads();
    bool finite = true;
    double* dst = ls_g + cell * nv;
    {
      NodeWalk walk(tid, BLOCK, n1, n2);
#pragma unroll 4
      for (int j = tid; j < nv; j += BLOCK, walk.next()) {
        double v;
        if (FIXED) {
          double lI;
          v = lam_hc(lo[j], walk.jx, walk.jy, walk.jz, lI) + scale * (from_fixed(acc64[j]) + (double)ovf[j]);
        } else {
          v = lsh[j];
        }
        finite = finite && isfinite(v);
        dst[j] = v;
      }
    }
    if (!finite) atomicOr(P.status, 2u);
    __syncthreads();
  }
}

// ------------------------------------------------------------ walls --
// dR/dU and dR/dtau of R = tau^-3/2 exp(|v|^2 - |v - U e_x|^2 / tau), from R.
__device__ __forceinline__ void wall_ratio_grad(double R, double vx, double vy, double vz, double U, double tau,
                                                double& dU, double& dtau) {
  const double ux = vx - U;
  const double c2 = (ux * ux + vy * vy) + vz * vz;
  dU = R * 2.0 * ux / tau;
  dtau = R * (c2 / (tau * tau) - 1.5 / tau);
}

__device__ __forceinline__ double face_tau(const Params& P, const WallArgs& W, int wall, int pos) {
  return wall == WALL_BOTTOM ? P.tau_b[pos] : W.tau[wall];
}

// One workgroup per face f = f0 + (its index): lam is the adjoint of the
// output of the streaming pass that read the face's ghosts (the y sweep for
// y faces of order 2, the x sweep for x faces, the unsplit step for order
// 1).  For the incoming nodes (v . n > 0) the ghost h_w = (n_w R - 1)/eps
// enters the sweep with weight a1 + a2 at the adjacent cell and a2 at the
// next one (order 2: both ghost layers), or C (order 1); with lg_j its
// adjoint,
//   dJ/dn_w   = sum_in lg_j R_j / eps
//   dJ/dtheta = n_w sum_in lg_j dR_j/dtheta / eps
//               - dJ/dn_w (n_w / D) sum_in |v_n| w_j dR_j/dtheta,
// the last term from n_w = (A + eps B)/D, D = sum_in |v_n| w R (the sum over
// the mirror images of the outgoing nodes, which are the incoming ones).
// Writes lnw[f] and the partials gpart[2f] (lid velocity, top faces only)
// and gpart[2f + 1] (the face's temperature).
constexpr int kWallAdjBlock = 256;

__global__ __launch_bounds__(kWallAdjBlock) void wall_adj_kernel(Params P, WallArgs W, const double* __restrict__ lam,
                                                                 double* __restrict__ lnw, double* __restrict__ gpart,
                                                                 int f0, int nface, int per_xcd) {
  __shared__ double red[5 * (kWallAdjBlock / 64)];
  int f = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (f >= nface) return;
  f += f0;
  int wall, pos;
  face_of(P, f, wall, pos);
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
  const double* la = lam + cell_off(P, ax_, ay_);
  const double* lb = lam + cell_off(P, bx_, by_);
  const double* R = ratio_row(P, wall, pos);
  const double dl = nax ? P.dy : P.dx;
  const double U = (wall == WALL_TOP) ? W.lid_u : 0.0;
  const double tau = face_tau(P, W, wall, pos);
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  NodeWalk walk(threadIdx.x, kWallAdjBlock, n1, n2);
  for (int j = threadIdx.x; j < nv; j += kWallAdjBlock, walk.next()) {
    const int jx = walk.jx, jy = walk.jy, jz = walk.jz;
    const double v1 = P.vtab[jx], v2 = P.vtab[kMaxAxis + jy], v3 = P.vtab[2 * kMaxAxis + jz];
    const double vn = nax ? v2 : v1;
    if (!(sgn * vn > 0.0)) continue;  // incoming nodes only
    const double an = fabs(vn);
    const double C = an * P.dt / dl;
    double lg;
    if (P.order == 2) {
      const double c2 = 0.5 * C * (1.0 - C);
      const double a1 = C + 2.0 * c2, a2 = -c2;
      lg = (a1 + a2) * la[j] + a2 * lb[j];
    } else {
      lg = C * la[j];
    }
    const double Rj = R[j];
    double dU, dT;
    wall_ratio_grad(Rj, v1, v2, v3, U, tau, dU, dT);
    const double aw = an * ((P.omtab[jx] * P.omtab[kMaxAxis + jy]) * P.omtab[2 * kMaxAxis + jz]);
    s[0] += lg * Rj;
    s[1] += lg * dU;
    s[2] += lg * dT;
    s[3] += aw * dU;
    s[4] += aw * dT;
  }
  block_sum<5>(s, red);
  if (threadIdx.x == 0) {
    const double nw = P.nw[f];
    const double D = wall_consts(P, wall, pos)[1];
    const double l = s[0] * P.inv_eps;
    const double q = l * nw / D;
    lnw[f] = l;
    gpart[2 * f] = (wall == WALL_TOP) ? nw * s[1] * P.inv_eps - q * s[3] : 0.0;
    gpart[2 * f + 1] = nw * s[2] * P.inv_eps - q * s[4];
  }
}

// ---------------------------------------------------------- streaming --
// Transposed Beam-Warming sweep along axis AX (0: x, 1: y) of order 2:
// out_i = a0 in_i + a1 in_{i-s} + a2 in_{i-2s} gives
//   li_i = a0 lo_i + a1 lo_{i+s} + a2 lo_{i+2s}
// over the downstream cells inside the cavity (wrapped when periodic; the
// ghost terms were taken by wall_adj_kernel), plus, at the two cells next to
// each wall across AX, the adjoint of that wall's face density through the
// gas-side face value hhat = h_a + (1 - C)(h_a - h_a')/2 of its outgoing
// nodes: dJ/dhhat_j = dJ/dn_w eps |v_n| w_j / D.  One workgroup: one line of
// cells along AX and 256 consecutive velocities; each thread walks its line
// against its node's direction with a two-value register window, so every
// element is read and written once.
constexpr int kSweepAdjBlock = 256;

template <int AX>
__global__ __launch_bounds__(kSweepAdjBlock) void sweep_adj_kernel(Params P, const double* __restrict__ lo,
                                                                   double* __restrict__ li,
                                                                   const double* __restrict__ lnw, int nchunks,
                                                                   int per_xcd) {
  const int nlines = AX == 0 ? P.ny : P.nx;
  const int unit = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (unit >= nlines * nchunks) return;
  const int line = unit / nchunks, chunk = unit - (unit / nchunks) * nchunks;
  const int nv = P.nv, n1 = P.n[1], n2 = P.n[2];
  const int j = chunk * kSweepAdjBlock + threadIdx.x;
  if (j >= nv) return;
  int jx, jy, jz;
  node_decode(j, n1, n2, jx, jy, jz);
  const int n = AX == 0 ? P.nx : P.ny;
  const int64_t stride = AX == 0 ? (int64_t)nv : (int64_t)P.nx * nv;
  const int64_t base = (AX == 0 ? cell_off(P, 0, line) : cell_off(P, line, 0)) + j;
  const double v = AX == 0 ? P.vtab[jx] : P.vtab[kMaxAxis + jy];
  const double an = fabs(v);
  const double C = an * P.dt / (AX == 0 ? P.dx : P.dy);
  const double c2 = 0.5 * C * (1.0 - C);
  double a0 = (1.0 - C) - c2, a1 = C + 2.0 * c2, a2 = -c2;
  const int s = v > 0.0 ? 1 : -1;
  if (v == 0.0) { a0 = 1.0; a1 = 0.0; a2 = 0.0; }
  const bool periodic = P.bc == 1;
  // face term of the wall on the outgoing side of this node
  double fa = 0.0, fb = 0.0;
  int ia = -1, ib = -1;
  if (!periodic && v != 0.0) {
    const int f = (AX == 0 ? (s < 0 ? 0 : P.ny) : 2 * P.ny + (s < 0 ? 0 : P.nx)) + line;
    int wall, pos;
    face_of(P, f, wall, pos);
    const double w = (P.omtab[jx] * P.omtab[kMaxAxis + jy]) * P.omtab[2 * kMaxAxis + jz];
    const double lh = lnw[f] * P.eps * an * w / wall_consts(P, wall, pos)[1];
    fa = lh * (1.0 + 0.5 * (1.0 - C));
    fb = -lh * 0.5 * (1.0 - C);
    ia = s < 0 ? 0 : n - 1;
    ib = s < 0 ? 1 : n - 2;
  }
  auto at = [&](int i) -> double {
    if (i >= 0 && i < n) return lo[base + i * stride];
    if (!periodic) return 0.0;
    return lo[base + (int64_t)wrapi(i, n) * stride];
  };
  const int i0 = s > 0 ? n - 1 : 0;
  double d1 = at(i0 + s), d2 = at(i0 + 2 * s);
  for (int k = 0; k < n; ++k) {
    const int i = i0 - k * s;
    const double c0 = lo[base + i * stride];
    double out = fma(a0, c0, fma(a1, d1, a2 * d2));
    if (i == ia) out += fa;
    if (i == ib) out += fb;
    li[base + i * stride] = out;
    d2 = d1;
    d1 = c0;
  }
}

// Transposed first-order unsplit step:
//   li = (1 - Cx - Cy) lo + Cx lo(downstream in x) + Cy lo(downstream in y)
// plus, at the cell next to each wall, dJ/dn_w eps |v_n| w_j / D for the
// wall's outgoing nodes (face value = the adjacent cell).  One thread per
// (cell, node).
constexpr int kOrder1AdjBlock = 256;

__global__ __launch_bounds__(kOrder1AdjBlock) void order1_adj_kernel(Params P, const double* __restrict__ lo,
                                                                     double* __restrict__ li,
                                                                     const double* __restrict__ lnw, int nchunks) {
  const int64_t cell = blockIdx.x / nchunks;
  const int chunk = blockIdx.x - (int)(cell * nchunks);
  const int nv = P.nv, n1 = P.n[1], n2 = P.n[2], nx = P.nx, ny = P.ny;
  const int j = chunk * kOrder1AdjBlock + threadIdx.x;
  if (j >= nv) return;
  int jx, jy, jz;
  node_decode(j, n1, n2, jx, jy, jz);
  const int ix = (int)(cell % nx), iy = (int)(cell / nx);
  const double vx = P.vtab[jx], vy = P.vtab[kMaxAxis + jy];
  const double Cx = fabs(vx) * P.dt / P.dx, Cy = fabs(vy) * P.dt / P.dy;
  const bool periodic = P.bc == 1;
  const int64_t o = cell * nv + j;
  double out = ((1.0 - Cx) - Cy) * lo[o];
  const double w = (P.omtab[jx] * P.omtab[kMaxAxis + jy]) * P.omtab[2 * kMaxAxis + jz];
  for (int ax = 0; ax < 2; ++ax) {
    const double v = ax == 0 ? vx : vy;
    if (v == 0.0) continue;
    const int s = v > 0.0 ? 1 : -1;
    const int n = ax == 0 ? nx : ny;
    const int i = (ax == 0 ? ix : iy) + s;
    const double Cv = ax == 0 ? Cx : Cy;
    if (i >= 0 && i < n) {
      out += Cv * lo[(ax == 0 ? cell_off(P, i, iy) : cell_off(P, ix, i)) + j];
    } else if (periodic) {
      const int iw = wrapi(i, n);
      out += Cv * lo[(ax == 0 ? cell_off(P, iw, iy) : cell_off(P, ix, iw)) + j];
    }
    // a cell next to the wall that this node leaves through
    const int ib = (ax == 0 ? ix : iy);
    if (!periodic && ((s < 0 && ib == 0) || (s > 0 && ib == n - 1))) {
      const int f = (ax == 0 ? (s < 0 ? 0 : ny) + iy : 2 * ny + (s < 0 ? 0 : nx) + ix);
      int wall, pos;
      face_of(P, f, wall, pos);
      out += lnw[f] * P.eps * fabs(v) * w / wall_consts(P, wall, pos)[1];
    }
  }
  li[o] = out;
}

// Per-face partials into the gradient (added to grad, fixed summation order):
// lid velocity from the top faces, the temperatures of the left, right and
// top walls, one entry per bottom face.  faces: 1 = x faces, 2 = y faces.
__global__ __launch_bounds__(256) void grad_reduce_kernel(Params P, const double* __restrict__ gpart,
                                                          double* __restrict__ grad, int faces) {
  const int nx = P.nx, ny = P.ny, t = threadIdx.x, lane = t & 63, w = t >> 6;
  // wavefront w sums the face partials of wall parameter w, all loads of a
  // lane issued together, then a wavefront tree sum
  {
    const bool on = (w == 0 || w == 3) ? (faces & 2) != 0 : (faces & 1) != 0;
    const int n = (w == 0 || w == 3) ? nx : ny;
    double s = 0.0;
    if (on) {
      for (int i = lane; i < n; i += 64) {
        const int k = w == 0 ? 2 * (2 * ny + nx + i) : (w == 1 ? 2 * i + 1 : (w == 2 ? 2 * (ny + i) + 1
                                                                                   : 2 * (2 * ny + nx + i) + 1));
        s += gpart[k];
      }
    }
    s = wave_sum(s);
    if (lane == 0) grad[w] += s;
  }
  if (faces & 2)
    for (int i = t; i < nx; i += blockDim.x) grad[4 + i] += gpart[2 * (2 * ny + i) + 1];
}

// ---------------------------------------------------------- lid shear --
// Adjoint of weight * D, D = -(1/nx) sum over lid faces of 2 sum_j w_j v_x v_y
// hhat_j with hhat the gas-side value of the top cell for v_y > 0 and the
// wall emission with the first-order face density for v_y < 0: one
// workgroup per top face adds its part to lam (top cells, v_y > 0 nodes)
// and writes the face's partials gpart[2 ix] (lid velocity) and
// gpart[2 ix + 1] (lid temperature).
// One workgroup of kLidAdjBlock threads per top face (the three node loops
// are latency bound: more threads per face, fewer nodes per thread).
constexpr int kLidAdjBlock = 1024;

__global__ __launch_bounds__(kLidAdjBlock) void lid_adj_kernel(Params P, WallArgs W, const float* __restrict__ h,
                                                               double weight, double* __restrict__ lam,
                                                               double* __restrict__ gpart) {
  __shared__ double red[5 * (kLidAdjBlock / 64)];
  const int ix = blockIdx.x;
  const int nv = P.nv, n1 = P.n[1], n2 = P.n[2];
  const double nwt = face_density(P, h, WALL_TOP, ix, 1, 0, 0, 0, 0, red);
  const double* R = ratio_row(P, WALL_TOP, ix);
  const double U = W.lid_u, tau = W.tau[WALL_TOP];
  const double c0 = weight * (-2.0 / P.nx);
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  NodeWalk walk(threadIdx.x, blockDim.x, n1, n2);
  for (int j = threadIdx.x; j < nv; j += blockDim.x, walk.next()) {
    const int jx = walk.jx, jy = walk.jy, jz = walk.jz;
    const double v1 = P.vtab[jx], v2 = P.vtab[kMaxAxis + jy], v3 = P.vtab[2 * kMaxAxis + jz];
    if (!(v2 < 0.0)) continue;
    const double w = (P.omtab[jx] * P.omtab[kMaxAxis + jy]) * P.omtab[2 * kMaxAxis + jz];
    const double coef = c0 * w * v1 * v2;
    const double Rj = R[j];
    double dU, dT;
    wall_ratio_grad(Rj, v1, v2, v3, U, tau, dU, dT);
    const double aw = fabs(v2) * w;
    s[0] += coef * Rj;
    s[1] += coef * dU;
    s[2] += coef * dT;
    s[3] += aw * dU;
    s[4] += aw * dT;
  }
  block_sum<5>(s, red);
  const double l = s[0] * P.inv_eps;
  const double D = wall_consts(P, WALL_TOP, ix)[1];
  double* dst = lam + cell_off(P, ix, P.ny - 1);
  NodeWalk walk2(threadIdx.x, blockDim.x, n1, n2);
  for (int j = threadIdx.x; j < nv; j += blockDim.x, walk2.next()) {
    const int jx = walk2.jx, jy = walk2.jy, jz = walk2.jz;
    const double v1 = P.vtab[jx], v2 = P.vtab[kMaxAxis + jy];
    if (!(v2 > 0.0)) continue;
    const double w = (P.omtab[jx] * P.omtab[kMaxAxis + jy]) * P.omtab[2 * kMaxAxis + jz];
    dst[j] += c0 * w * v1 * v2 + l * P.eps * v2 * w / D;
  }
  if (threadIdx.x == 0) {
    const double q = l * nwt / D;
    gpart[2 * ix] = nwt * s[1] * P.inv_eps - q * s[3];
    gpart[2 * ix + 1] = nwt * s[2] * P.inv_eps - q * s[4];
  }
}

// Lid-shear partials into grad[0] (lid velocity) and grad[3] (lid temperature).
__global__ void lid_grad_kernel(Params P, const double* __restrict__ gpart, double* __restrict__ grad) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double su = 0.0, st = 0.0;
    for (int i = 0; i < P.nx; ++i) {
      su += gpart[2 * i];
      st += gpart[2 * i + 1];
    }
    grad[0] += su;
    grad[3] += st;
  }
}

}  // namespace boltz
