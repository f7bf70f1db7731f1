// collide.hpp -- S3-S5 of one step on gfx950: the Monte Carlo pair sampler
// (Sec. 3, Eqs. coll8Dim, monteCarloInt), the shared-sample table pass, and
// the collision kernel with its conservation correction (Eqs.
// collision_step, rinorm_a, correzione).  Included by kernels.hpp.
#pragma once

#include "device_math.hpp"

namespace boltz {

// ---------------------------------------------------------------- tables --
// LDS copies of the per-axis tables, ns = n0 + n1 + n2 entries each:
//   v, om, xt        always (moment sums and the correction)
//   nq, rw, icdf     only where pairs are drawn
struct TablesLDS {
  double* v;      // node velocities
  double* om;     // omega, FP64
  double* xt;     // per-axis parts of x . psi of the correction (per cell)
  double* m0;     // [16] sum_j w_j psi_k psi_l (packed k <= l), constant
  float4* nq;     // {omega, p_phi, p_unif, 0}, FP32
  double* rw;     // 1 / omega, FP64
  uint8_t* icdf;  // [3 * kFieldSize] Maxwellian inverse CDF on 12-bit fields
  double* edge;   // [ns + 3] cell edges per axis (n + 1 each), for the search
                  // of post-collision cells on stretched grids

  static __host__ __device__ size_t bytes(int ns, bool sampler) {
    size_t b = 24 * (size_t)ns + 16 * sizeof(double);
    if (sampler) b += 32 * (size_t)ns + 24 + 3 * (size_t)kFieldSize;
    return b;
  }
};

// base: 16-byte aligned LDS.  The caller synchronises before use.
__device__ __forceinline__ void load_tables(const Params& P, unsigned char* base, bool sampler, TablesLDS& T) {
  const int n0 = P.n[0], n1 = P.n[1], n2 = P.n[2], ns = n0 + n1 + n2;
  T.v = reinterpret_cast<double*>(base);
  T.om = T.v + ns;
  T.xt = T.om + ns;
  T.m0 = T.xt + ns;
  T.nq = reinterpret_cast<float4*>(T.m0 + 16);
  T.rw = reinterpret_cast<double*>(T.nq + ns);
  T.edge = T.rw + ns;
  T.icdf = reinterpret_cast<uint8_t*>(T.edge + ns + 3);
  for (int i = threadIdx.x; i < ns; i += blockDim.x) {
    const int k = i < n0 ? 0 : (i < n0 + n1 ? 1 : 2);
    const int o = k * kMaxAxis + i - (k == 0 ? 0 : (k == 1 ? n0 : n0 + n1));
    T.v[i] = P.vtab[o];
    T.om[i] = P.omtab[o];
    if (sampler) {
      T.nq[i] = P.nqtab[o];
      T.rw[i] = P.rwtab[o];
    }
  }
  if (sampler) {
    // n + 1 edges per axis, axis k at offset n0 + ... + n_{k-1} + k
    for (int i = threadIdx.x; i < ns + 3; i += blockDim.x) {
      const int k = i < n0 + 1 ? 0 : (i < n0 + n1 + 2 ? 1 : 2);
      const int o = i - (k == 0 ? 0 : (k == 1 ? n0 + 1 : n0 + n1 + 2));
      T.edge[i] = P.edgetab[k * (kMaxAxis + 1) + o];
    }
  }
  if (threadIdx.x < 15) T.m0[threadIdx.x] = P.m0[threadIdx.x];
  if (sampler) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(P.icdf);
    uint32_t* dst = reinterpret_cast<uint32_t*>(T.icdf);
    for (int i = threadIdx.x; i < 3 * kFieldSize / 4; i += blockDim.x) dst[i] = src[i];
  }
}

// ----------------------------------------------------------------- S3 --
// Importance weights of a drawn node (i, j, k): r = w / p~ and s = 1 / p~,
// with w the midpoint weight of Phi0 and p~ = (1 - beta) p_phi + beta p_unif
// the probability of drawing it from the mixture law.  FP32.
struct NodeWeight {
  float r, s;
};

__device__ __forceinline__ NodeWeight node_weight(const TablesLDS& T, float beta, float obeta, int i, int j, int k,
                                                  int n0, int n1) {
  const float4 x = T.nq[i], y = T.nq[n0 + j], z = T.nq[n0 + n1 + k];
  const float w = (x.x * y.x) * z.x;
  const float pm = (x.y * y.y) * z.y;
  const float pu = (x.z * y.z) * z.z;
  const float s = 1.0f / (obeta * pm + beta * pu);
  NodeWeight o;
  o.r = w * s;
  o.s = s;
  return o;
}

// Cell of x among n stretched cells with edges e[0] = -a < ... < e[n] = a:
// the largest i with e[i] <= x (an x on an edge belongs to the upper cell),
// -1 outside [e[0], e[n]).  Binary search, the same number of steps in
// every lane.
__device__ __forceinline__ int edge_search(const double* e, int n, double x) {
  int lo = 0, hi = n;  // e[lo] <= x < e[hi] while inside
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    const bool up = x >= e[mid];
    lo = up ? mid : lo;
    hi = up ? hi : mid;
  }
  return (x >= e[0] && x < e[n]) ? lo : -1;
}

// One Monte Carlo collision sample.  The four coefficients are the weight q
// of Eq. coll8Dim divided by the midpoint weight of the node it lands on, so
// that the sample changes h by +k g at a*, b* and by -k g at a, b with
// g = h_a + h_b + eps h_a h_b (Eqs. monteCarloInt, collision_step).
struct Pair {
  int a, b, as, bs;   // node indices; as = bs = -1 when discarded
  double q;           // dt K |v_r . k| (w_a / p~_a)(w_b / p~_b) / N_t
  double kas, kbs;    // q / w_{a*}, q / w_{b*}
  double ka, kb;      // q / w_a, q / w_b
};

// One Philox4x32-10 block with counter (m, group, step, cavity) per sample:
//   r0 = [a_x:12][a_y:12][choice_a:4][choice_b:4]
//   r1 = [a_z:12][b_x:12][phi_hi:8]   r2 = [b_y:12][b_z:12][phi_lo:8]   r3 = u
// nodes from the Maxwellian law, or the uniform law when the choice nibble
// is below mix16; k_z = 2 (r3 + 1/2) 2^-32 - 1, azimuth 2 pi (phi + 1/2) 2^-16;
// v* = v_a + (v_r.k) k, v1* = v_b - (v_r.k) k with v_r = v_b - v_a;
// post-collision cells floor((x + a) n / 2a), discard outside the box.
__device__ __forceinline__ Pair sample_pair_continuous(const Params& P, const TablesLDS& T, uint32_t group,
                                                       uint32_t step, uint32_t m, u32x4* words);

__device__ __forceinline__ Pair sample_pair_node(const Params& P, const TablesLDS& T, uint32_t group,
                                                 uint32_t step, uint32_t m, u32x4* words) {
  const int n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
  const u32x4 c = {m, group, step, P.cavity};
  uint32_t k0 = P.key0, k1 = P.key1;
  // an empty statement that keeps the key words opaque, so the round keys
  // are rebuilt by scalar adds inside the caller's loop instead of being
  // hoisted into twenty scalar registers
  asm volatile("" : "+s"(k0), "+s"(k1));
  const u32x4 r = philox4x32_10(c, k0, k1);
  if (words) words[0] = r;
  const bool ua = ((r.x >> 4) & 15u) < P.mix16;
  const bool ub = (r.x & 15u) < P.mix16;
  const uint32_t fax = r.x >> 20, fay = (r.x >> 8) & 0xFFFu, faz = r.y >> 20;
  const uint32_t fbx = (r.y >> 8) & 0xFFFu, fby = r.z >> 20, fbz = (r.z >> 8) & 0xFFFu;
  // both laws evaluated, then selected (no divergent branch)
  const int max_ = (int)T.icdf[fax], may = (int)T.icdf[kFieldSize + fay], maz = (int)T.icdf[2 * kFieldSize + faz];
  const int mbx = (int)T.icdf[fbx], mby = (int)T.icdf[kFieldSize + fby], mbz = (int)T.icdf[2 * kFieldSize + fbz];
  const int iax = ua ? uniform_draw(fax, n0) : max_;
  const int iay = ua ? uniform_draw(fay, n1) : may;
  const int iaz = ua ? uniform_draw(faz, n2) : maz;
  const int ibx = ub ? uniform_draw(fbx, n0) : mbx;
  const int iby = ub ? uniform_draw(fby, n1) : mby;
  const int ibz = ub ? uniform_draw(fbz, n2) : mbz;
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
  int sx, sy, sz, tx, ty, tz;
  if (P.stretched) {
    // stretched cells (Sec. 5.1): binary search over the edges
    const double* ex = T.edge;
    const double* ey = T.edge + n0 + 1;
    const double* ez = T.edge + n0 + n1 + 2;
    sx = edge_search(ex, n0, vax + ddx);
    sy = edge_search(ey, n1, vay + ddy);
    sz = edge_search(ez, n2, vaz + ddz);
    tx = edge_search(ex, n0, vbx - ddx);
    ty = edge_search(ey, n1, vby - ddy);
    tz = edge_search(ez, n2, vbz - ddz);
  } else {
    const double tsx = floor((vax + ddx + P.a[0]) * P.inv_cell[0]);
    const double tsy = floor((vay + ddy + P.a[1]) * P.inv_cell[1]);
    const double tsz = floor((vaz + ddz + P.a[2]) * P.inv_cell[2]);
    const double ttx = floor((vbx - ddx + P.a[0]) * P.inv_cell[0]);
    const double tty = floor((vby - ddy + P.a[1]) * P.inv_cell[1]);
    const double ttz = floor((vbz - ddz + P.a[2]) * P.inv_cell[2]);
    // inside the box iff 0 <= floor < n per component (the integer
    // conversion saturates, so far-out values fail the unsigned test as well)
    sx = (int)tsx;
    sy = (int)tsy;
    sz = (int)tsz;
    tx = (int)ttx;
    ty = (int)tty;
    tz = (int)ttz;
  }
  const bool kept = ((unsigned)sx < (unsigned)n0) & ((unsigned)sy < (unsigned)n1) & ((unsigned)sz < (unsigned)n2) &
                    ((unsigned)tx < (unsigned)n0) & ((unsigned)ty < (unsigned)n1) & ((unsigned)tz < (unsigned)n2);
  Pair p;
  p.a = (iax * n1 + iay) * n2 + iaz;
  p.b = (ibx * n1 + iby) * n2 + ibz;
  if (kept) {
    p.as = (sx * n1 + sy) * n2 + sz;
    p.bs = (tx * n1 + ty) * n2 + tz;
    const float beta = (float)P.beta;
    const NodeWeight wa = node_weight(T, beta, 1.0f - beta, iax, iay, iaz, n0, n1);
    const NodeWeight wb = node_weight(T, beta, 1.0f - beta, ibx, iby, ibz, n0, n1);
    const double qa = P.qfac * fabs(alpha);
    const double ra = (double)wa.r, rb = (double)wb.r;
    p.q = (qa * ra) * rb;
    p.ka = (qa * (double)wa.s) * rb;
    p.kb = (qa * ra) * (double)wb.s;
    p.kas = p.q * ((T.rw[sx] * T.rw[n0 + sy]) * T.rw[n0 + n1 + sz]);
    p.kbs = p.q * ((T.rw[tx] * T.rw[n0 + ty]) * T.rw[n0 + n1 + tz]);
  } else {
    p.as = -1;
    p.bs = -1;
    p.q = 0.0;
    p.kas = p.kbs = p.ka = p.kb = 0.0;
  }
  return p;
}

// Cell of velocity component x on axis k (n cells), -1 outside the box: the
// floor of the uniform grid or the edge search of stretched cells.
__device__ __forceinline__ int velocity_cell(const Params& P, const TablesLDS& T, int k, int n, double x) {
  if (P.stretched) {
    const double* e = T.edge + (k == 0 ? 0 : (k == 1 ? P.n[0] + 1 : P.n[0] + P.n[1] + 2));
    return edge_search(e, n, x);
  }
  const int t = (int)floor((x + P.a[k]) * P.inv_cell[k]);
  return (unsigned)t < (unsigned)n ? t : -1;
}

// The continuous variant (problem flag BOLTZ_CONTINUOUS_PAIRS; the sampling
// kernel of Sec. 4): v and v1 from the Maxwellian Phi0 (components normal
// with variance 1/2) by the Box-Muller method, k as in sample_pair, every
// velocity binned to its cell.  Two Philox blocks: A with counter
// (m, group, step, cavity), B with (m, group | 2^31, step, cavity); radii
// sqrt(-ln((w + 1) 2^-32)), angles 2 pi (w + 1/2) 2^-32:
//   (v_x, v_y) from (A0, A1), (v_z, v1_x) from (A2, A3), (v1_y, v1_z) from
//   (B0, B1), k_z = 2 (B2 + 1/2) 2^-32 - 1, azimuth 2 pi (B3 + 1/2) 2^-32.
// Weight q = dt K |v_r . k| / N_t (Phi0 is the sampling density); a pair
// with any velocity outside the box is discarded, a and b then -1 when v or
// v1 is outside.  words: block A.
__device__ __forceinline__ Pair sample_pair_continuous(const Params& P, const TablesLDS& T, uint32_t group,
                                                       uint32_t step, uint32_t m, u32x4* words) {
  const int n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
  uint32_t k0 = P.key0, k1 = P.key1;
  asm volatile("" : "+s"(k0), "+s"(k1));
  const u32x4 A = philox4x32_10(u32x4{m, group, step, P.cavity}, k0, k1);
  const u32x4 B = philox4x32_10(u32x4{m, group | 0x80000000u, step, P.cavity}, k0, k1);
  if (words) words[0] = A;
  double nv[6];
  const uint32_t rad[3] = {A.x, A.z, B.x}, ang[3] = {A.y, A.w, B.y};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double r = sqrt(neg_ln_unit(((double)rad[i] + 1.0) * 0x1p-32));
    double cs, sn;
    cos_sin_2pi(((double)ang[i] + 0.5) * 0x1p-32, cs, sn);
    nv[2 * i] = r * cs;
    nv[2 * i + 1] = r * sn;
  }
  const double vax = nv[0], vay = nv[1], vaz = nv[2], vbx = nv[3], vby = nv[4], vbz = nv[5];
  const double kz = 2.0 * (((double)B.z + 0.5) * 0x1p-32) - 1.0;
  const double s = sqrt((1.0 - kz) * (1.0 + kz));
  double cp, sp;
  cos_sin_2pi(((double)B.w + 0.5) * 0x1p-32, cp, sp);
  const double kx = s * cp, ky = s * sp;
  const double vrx = vbx - vax, vry = vby - vay, vrz = vbz - vaz;
  const double alpha = (vrx * kx + vry * ky) + vrz * kz;
  const double ddx = alpha * kx, ddy = alpha * ky, ddz = alpha * kz;
  const int ax = velocity_cell(P, T, 0, n0, vax), ay = velocity_cell(P, T, 1, n1, vay),
            az = velocity_cell(P, T, 2, n2, vaz);
  const int bx = velocity_cell(P, T, 0, n0, vbx), by = velocity_cell(P, T, 1, n1, vby),
            bz = velocity_cell(P, T, 2, n2, vbz);
  const int sx = velocity_cell(P, T, 0, n0, vax + ddx), sy = velocity_cell(P, T, 1, n1, vay + ddy),
            sz = velocity_cell(P, T, 2, n2, vaz + ddz);
  const int tx = velocity_cell(P, T, 0, n0, vbx - ddx), ty = velocity_cell(P, T, 1, n1, vby - ddy),
            tz = velocity_cell(P, T, 2, n2, vbz - ddz);
  const bool in_a = (ax >= 0) & (ay >= 0) & (az >= 0), in_b = (bx >= 0) & (by >= 0) & (bz >= 0);
  const bool kept = in_a & in_b & (sx >= 0) & (sy >= 0) & (sz >= 0) & (tx >= 0) & (ty >= 0) & (tz >= 0);
  Pair p;
  p.a = in_a ? (ax * n1 + ay) * n2 + az : -1;
  p.b = in_b ? (bx * n1 + by) * n2 + bz : -1;
  if (kept) {
    p.as = (sx * n1 + sy) * n2 + sz;
    p.bs = (tx * n1 + ty) * n2 + tz;
    p.q = P.qfac * fabs(alpha);
    p.ka = p.q * ((T.rw[ax] * T.rw[n0 + ay]) * T.rw[n0 + n1 + az]);
    p.kb = p.q * ((T.rw[bx] * T.rw[n0 + by]) * T.rw[n0 + n1 + bz]);
    p.kas = p.q * ((T.rw[sx] * T.rw[n0 + sy]) * T.rw[n0 + n1 + sz]);
    p.kbs = p.q * ((T.rw[tx] * T.rw[n0 + ty]) * T.rw[n0 + n1 + tz]);
  } else {
    p.as = -1;
    p.bs = -1;
    p.q = 0.0;
    p.kas = p.kbs = p.ka = p.kb = 0.0;
  }
  return p;
}

// The sampler of the problem: the node law, or continuous pairs.  Loops
// that draw pairs per cell choose once, outside the loop (each loop is then
// compiled with one sampler's registers).
__device__ __forceinline__ Pair sample_pair(const Params& P, const TablesLDS& T, uint32_t group, uint32_t step,
                                            uint32_t m, u32x4* words) {
  return P.continuous ? sample_pair_continuous(P, T, group, step, m, words)
                      : sample_pair_node(P, T, group, step, m, words);
}

// Test hook kernel: the pairs of (cell, step, m0 + i) from the same sampler.
__global__ __launch_bounds__(256) void debug_pairs_kernel(Params P, int64_t cell, uint32_t step, int64_t m0,
                                                          int64_t count, int32_t* idx4, double* q,
                                                          uint32_t* words) {
  extern __shared__ __align__(16) unsigned char dsm[];
  TablesLDS T;
  load_tables(P, dsm, true, T);
  __syncthreads();
  const uint32_t group = (P.sample_group == 0) ? 0u : (uint32_t)(cell / P.sample_group);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    u32x4 w;
    const Pair p = sample_pair(P, T, group, step, (uint32_t)(m0 + i), &w);
    idx4[4 * i + 0] = p.a;
    idx4[4 * i + 1] = p.b;
    idx4[4 * i + 2] = p.as;
    idx4[4 * i + 3] = p.bs;
    q[i] = p.q;
    if (words) {
      words[4 * i + 0] = w.x;
      words[4 * i + 1] = w.y;
      words[4 * i + 2] = w.z;
      words[4 * i + 3] = w.w;
    }
  }
}

// Shared-sample mode (G != 1): the N_t pairs of every sample group are drawn
// once per step into two arrays, idx = {a | b << 16, a* | b* << 16} and
// coef = {q/w_a*, q/w_b*, q/w_a, q/w_b} in FP32; a discarded pair is stored
// with a* = a, b* = b and zero coefficients.
__device__ __forceinline__ void sample_pair_record(const Params& P, const TablesLDS& T, uint32_t step,
                                                   uint32_t group, int64_t i, uint2& id, float4& coef) {
  const Pair p = sample_pair(P, T, group, step, (uint32_t)i, nullptr);
  // a discarded continuous pair may have no cell for v or v1: node 0 then
  // (its coefficients are zero)
  const uint32_t a = p.a < 0 ? 0u : (uint32_t)p.a, b = p.b < 0 ? 0u : (uint32_t)p.b;
  id.x = a | (b << 16);
  id.y = p.as >= 0 ? ((uint32_t)p.as | ((uint32_t)p.bs << 16)) : id.x;
  coef = make_float4((float)p.kas, (float)p.kbs, (float)p.ka, (float)p.kb);
}

// Records are drawn by blocks of kSampleBlock threads, one record each.
// The collision hands record m to lane m % 64 of a wavefront, and the sum
// over the records does not depend on their order; so each full block of
// 1024 records is stored dealt to lanes: the records whose first node a has
// a % 64 == k fill lane k of the block's 16 wavefronts in record order, and
// the ones beyond 16 fill the lanes left empty, in record order (key k, then
// wavefront).  The 64 gathers of h^s[a] and the 64 adds at a of one
// wavefront then mostly fall into distinct LDS banks.  All threads of the
// block call this (valid: the thread holds a record; n_blk: the block's
// record count; deal: permute, else store in place).  sh: 1280 words of LDS.
constexpr int kSampleBlock = 1024;

__device__ __forceinline__ void store_records(uint2 id, float4 coef, bool valid, int n_blk, bool deal,
                                              uint2* __restrict__ tidx, float4* __restrict__ tcoef,
                                              unsigned* sh) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (!deal || n_blk < kSampleBlock) {
    if (valid) {
      tidx[tid] = id;
      tcoef[tid] = coef;
    }
    return;
  }
  constexpr int NW = kSampleBlock / 64, CAP = NW;
  unsigned* cnt = sh;              // [NW][64] per-wavefront key counts, then their prefixes
  unsigned* tot = sh + NW * 64;    // [64] records per key
  unsigned* overp = tot + 64;      // [64] exclusive prefix of max(0, tot - CAP)
  unsigned* defp = overp + 64;     // [64] exclusive prefix of max(0, CAP - tot)
  const int key = (int)(id.x & 63u);
  // rank among the wavefront's records with the same key (record order)
  unsigned rin = 0;
  for (int k = 0; k < 64; ++k) {
    const unsigned long long m = __ballot(key == k);
    if (key == k) rin = (unsigned)__popcll(m & ((1ull << lane) - 1ull));
    if (lane == k) cnt[w * 64 + k] = (unsigned)__popcll(m);
  }
  __syncthreads();
  if (tid < 64) {
    unsigned run = 0;
    for (int v = 0; v < NW; ++v) {
      const unsigned c = cnt[v * 64 + tid];
      cnt[v * 64 + tid] = run;
      run += c;
    }
    tot[tid] = run;
    // exclusive prefixes over the keys of the overflow and of the free lanes
    unsigned ov = run > CAP ? run - CAP : 0u, df = run < CAP ? CAP - run : 0u;
    unsigned sov = ov, sdf = df;
    for (int d = 1; d < 64; d <<= 1) {
      const unsigned a = __shfl_up(sov, d, 64), b = __shfl_up(sdf, d, 64);
      if (lane >= d) {
        sov += a;
        sdf += b;
      }
    }
    overp[tid] = sov - ov;
    defp[tid] = sdf - df;
  }
  __syncthreads();
  const unsigned rho = cnt[w * 64 + key] + rin;
  int slot;
  if (rho < (unsigned)CAP) {
    slot = 64 * (int)rho + key;
  } else {
    // the L-th record past its key's lanes takes the L-th free lane
    const unsigned L = overp[key] + (rho - CAP);
    int lo = 0, hi = 63;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (defp[mid] <= L) lo = mid;
      else hi = mid - 1;
    }
    // the last key with defp <= L: keys without free lanes repeat the
    // next key's prefix, so it is the key whose free lanes hold L
    slot = 64 * (int)(tot[lo] + (L - defp[lo])) + lo;
  }
  tidx[slot] = id;
  tcoef[slot] = coef;
}

// One block of kSampleBlock records of a sample group, from record base:
// drawn (one per thread), then stored through store_records.
__device__ __forceinline__ void sample_block(const Params& P, const TablesLDS& T, uint32_t step, uint32_t group,
                                             int64_t base, bool deal, uint2* __restrict__ tidx,
                                             float4* __restrict__ tcoef, unsigned* sh) {
  const int64_t nt = P.n_pairs;
  const int n_blk = (int)(nt - base < kSampleBlock ? nt - base : kSampleBlock);
  const bool valid = (int)threadIdx.x < n_blk;
  uint2 id = make_uint2(0u, 0u);
  float4 coef = make_float4(0.f, 0.f, 0.f, 0.f);
  if (valid) sample_pair_record(P, T, step, group, base + threadIdx.x, id, coef);
  store_records(id, coef, valid, n_blk, deal, tidx + (int64_t)group * nt + base, tcoef + (int64_t)group * nt + base,
                sh);
}

// Grid: (ceil(N_t / kSampleBlock), groups).  deal: no sort follows (the
// records go straight to the collision), so they are dealt to lanes.
__global__ __launch_bounds__(kSampleBlock) void sample_kernel(Params P, uint32_t step, uint2* __restrict__ tidx,
                                                              float4* __restrict__ tcoef, int deal) {
  extern __shared__ __align__(16) unsigned char dsm[];
  __shared__ unsigned sh[1280];
  TablesLDS T;
  load_tables(P, dsm, true, T);
  __syncthreads();
  sample_block(P, T, step, blockIdx.y, (int64_t)blockIdx.x * kSampleBlock, deal != 0, tidx, tcoef, sh);
}

// Pattern of a shared-sample record for the split accumulation: bit k is
// set when its k-th target (a*, b*, a, b) lies in the upper half of the
// velocity index.
__device__ __forceinline__ unsigned split_pattern(uint2 id, unsigned h2) {
  return ((id.y & 0xFFFFu) >= h2 ? 1u : 0u) | ((id.y >> 16) >= h2 ? 2u : 0u) | ((id.x & 0xFFFFu) >= h2 ? 4u : 0u) |
         ((id.x >> 16) >= h2 ? 8u : 0u);
}

// Counting sort of the N_t records of one sample group by split_pattern
// (one workgroup per group), from (sidx, scoef) into (tidx, tcoef): the
// wavefronts of the collision then see records of one pattern, so each of
// the two passes skips the adds (and records) whose targets all lie in the
// other half.  The order within a pattern is that of the atomic cursors,
// which the fixed-point sums do not depend on.
constexpr int kSortBlock = 1024;

__device__ __forceinline__ void split_sort_group(const uint2* __restrict__ sidx, const float4* __restrict__ scoef,
                                                 uint2* __restrict__ tidx, float4* __restrict__ tcoef, int64_t nt,
                                                 unsigned h2) {
  __shared__ unsigned cnt[16];
  if (threadIdx.x < 16) cnt[threadIdx.x] = 0u;
  __syncthreads();
  for (int64_t m = threadIdx.x; m < nt; m += blockDim.x) atomicAdd(&cnt[split_pattern(sidx[m], h2)], 1u);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned run = 0;
    for (int k = 0; k < 16; ++k) {
      const unsigned c = cnt[k];
      cnt[k] = run;
      run += c;
    }
  }
  __syncthreads();
  for (int64_t m = threadIdx.x; m < nt; m += blockDim.x) {
    const uint2 id = sidx[m];
    const unsigned pos = atomicAdd(&cnt[split_pattern(id, h2)], 1u);
    tidx[pos] = id;
    tcoef[pos] = scoef[m];
  }
}

__global__ __launch_bounds__(kSortBlock) void split_sort_kernel(const uint2* __restrict__ sidx,
                                                                const float4* __restrict__ scoef,
                                                                uint2* __restrict__ tidx, float4* __restrict__ tcoef,
                                                                int64_t nt, unsigned h2) {
  const int64_t g = blockIdx.x;
  split_sort_group(sidx + g * nt, scoef + g * nt, tidx + g * nt, tcoef + g * nt, nt, h2);
}

// The records of every shared-sample problem of a batch in one launch:
// start[c] = first block of problem c, which has ceil(N_t / kSampleBlock)
// blocks per group; the step number is read from the device.
__global__ __launch_bounds__(kSampleBlock) void sample_batch_kernel(const BatchCav* __restrict__ cavs,
                                                                    const int* __restrict__ start, int count,
                                                                    const uint32_t* __restrict__ step_dev) {
  extern __shared__ __align__(16) unsigned char dsm[];
  __shared__ unsigned sh[1280];
  const int u = blockIdx.x;
  if (u >= start[count]) return;
  const int c = find_cav(start, count, u);
  const BatchCav& C = cavs[c];
  const Params& P = C.P;
  const int nb = (int)((P.n_pairs + kSampleBlock - 1) / kSampleBlock);
  const int local = u - start[c];
  const uint32_t group = (uint32_t)(local / nb);
  TablesLDS T;
  load_tables(P, dsm, true, T);
  __syncthreads();
  sample_block(P, T, *step_dev, group, (int64_t)(local - (int)group * nb) * kSampleBlock, C.sidx == C.tidx, C.sidx,
               C.scoef, sh);
}

// The split-pattern sort of every ACC_SPLIT shared-sample problem of a
// batch: start[c] = first workgroup of problem c, one per sample group.
__global__ __launch_bounds__(kSortBlock) void split_sort_batch_kernel(const BatchCav* __restrict__ cavs,
                                                                      const int* __restrict__ start, int count) {
  const int u = blockIdx.x;
  if (u >= start[count]) return;
  const int c = find_cav(start, count, u);
  const BatchCav& C = cavs[c];
  const int64_t nt = C.P.n_pairs, g = u - start[c];
  split_sort_group(C.sidx + g * nt, C.scoef + g * nt, C.tidx + g * nt, C.tcoef + g * nt, nt,
                   (unsigned)((C.P.nv + 1) / 2));
}

// ------------------------------------------------------------------- S5 --
// Solve of the 5x5 SPD system M x = r, M given by the packed upper triangle
// of its 15 sums (row k, columns l >= k), by the LDL^T factorisation (unit
// lower L, diagonal D): five reciprocals of the pivots, no square roots.
//   E_ij = L_ij D_j = M_ij - sum_{k<j} L_ik E_jk,  L_ij = E_ij / D_j,
//   D_i = M_ii - sum_{k<i} L_ik E_ik;  L y = r, x = L^-T (D^-1 y).
// false when a pivot is not positive (M not positive definite).
// 1 / d for a normal d > 0: the hardware estimate refined by two
// Newton-Raphson steps r <- r + r (1 - d r) (each doubles the correct bits),
// a shorter dependent chain than the IEEE division sequence.
__device__ __forceinline__ double recip_pos(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

__device__ __forceinline__ bool solve5(const double* S, const double* r, double* x) {
  double A[5][5];
  int t = 0;
#pragma unroll
  for (int k = 0; k < 5; ++k)
#pragma unroll
    for (int l = k; l < 5; ++l) A[l][k] = S[t++];
  double L[5][5], E[5][5], rd[5];
  bool ok = true;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    double d = A[i][i];
#pragma unroll
    for (int j = 0; j < i; ++j) {
      double e = A[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) e -= L[i][k] * E[j][k];
      E[i][j] = e;
      L[i][j] = e * rd[j];
      d -= L[i][j] * e;
    }
    ok = ok && (d > 0.0);
    rd[i] = recip_pos(d > 0.0 ? d : 1.0);
  }
  double y[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    double v = r[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= L[i][k] * y[k];
    y[i] = v;
  }
#pragma unroll
  for (int i = 4; i >= 0; --i) {
    double v = y[i] * rd[i];
#pragma unroll
    for (int k = i + 1; k < 5; ++k) v -= L[k][i] * x[k];
    x[i] = v;
  }
  return ok;
}

// ------------------------------------------------------------ collision --
// Accumulation of the increments of h in LDS:
//   ACC_FIXED  64-bit fixed point for every node plus an FP32 array for large
//              values (16 B/node with the h^s tile)
//   ACC_SPLIT  the same for half of the nodes at a time: the pairs are read
//              twice, each pass keeping the increments of one half of the
//              velocity index (10 B/node; grids too large for ACC_FIXED)
//   ACC_CAS    FP32 compare-and-swap for every node (8 B/node)
//   ACC_HYBRID one pass for grids too large for ACC_FIXED: 64-bit fixed point
//              for the inner x-slabs of the velocity grid, FP32 (the LDS
//              float atomic) for the outer slabs (rarely reached), next to
//              the full h^s tile; h^c is not stored but formed again from
//              h^s and the accumulators where it is read
//   ACC_PART   one pass with 64-bit fixed point for every node (grids too
//              large for ACC_FIXED): the h^s tile of the central x-slabs
//              sits in LDS after the accumulators, the outer slabs' h^s is
//              read from the cell's row in global memory (gathers of the
//              few samples that reach them, rows in the node phases); h^c
//              is formed again where it is read (12 B/node or less)
enum : int { ACC_CAS = 0, ACC_FIXED = 1, ACC_SPLIT = 2, ACC_HYBRID = 3, ACC_PART = 4 };

// Dynamic LDS of the collide kernel: the h^s tile (FP32), the accumulators,
// then the tables.  The region after the tile holds h^c after the pair pass
// (ACC_CAS, ACC_FIXED: the FP32 array, which comes first).
struct CollideLDS {
  static __host__ __device__ size_t tile(int nv) { return ((size_t)nv * 4 + 15) & ~(size_t)15; }
  static __host__ __device__ int half(int nv) { return (nv + 1) / 2; }
  // 64-bit accumulators of ACC_SPLIT (then its FP32 array)
  static __host__ __device__ size_t split64(int nv) { return ((size_t)half(nv) * 8 + 15) & ~(size_t)15; }
  static __host__ __device__ size_t acc(int nv, int mode) {
    if (mode == ACC_SPLIT) return split64(nv) + (((size_t)half(nv) * 4 + 15) & ~(size_t)15);
    return tile(nv) + (mode == ACC_FIXED ? (((size_t)nv * 8 + 15) & ~(size_t)15) : 0);
  }
  static __host__ __device__ size_t bytes(int nv, int ns, int mode, bool sampler) {
    return tile(nv) + acc(nv, mode) + TablesLDS::bytes(ns, sampler);
  }
  // ACC_HYBRID with nin inner nodes: 64-bit accumulators, then the FP32 ones
  static __host__ __device__ size_t hyb64(int nin) { return ((size_t)nin * 8 + 15) & ~(size_t)15; }
  static __host__ __device__ size_t hyb_acc(int nv, int nin) {
    return hyb64(nin) + (((size_t)(nv - nin) * 4 + 15) & ~(size_t)15);
  }
  static __host__ __device__ size_t hyb_bytes(int nv, int nin, int ns, bool sampler) {
    return tile(nv) + hyb_acc(nv, nin) + TablesLDS::bytes(ns, sampler);
  }
  // ACC_PART with nin nodes in the LDS tile: 64-bit accumulators of every
  // node, the tile, the tables
  static __host__ __device__ size_t part64(int nv) { return ((size_t)nv * 8 + 15) & ~(size_t)15; }
  static __host__ __device__ size_t part_bytes(int nv, int nin, int ns, bool sampler) {
    return part64(nv) + tile(nin) + TablesLDS::bytes(ns, sampler);
  }
};

// Accumulators of ACC_HYBRID: nodes lo .. lo + n - 1 in in[node - lo]
// (64-bit fixed point), the others in out[slot] (FP32; slot = node below
// lo, node - n above); ovf: the workgroup's global row for terms beyond the
// 64-bit range, with flag (LDS) raised when it is used.
struct Hyb {
  unsigned long long* in;
  float* out;
  int lo;
  unsigned n;
  float* ovf;
  unsigned* flag;
  __device__ __forceinline__ bool inner(int j) const { return (unsigned)(j - lo) < n; }
  __device__ __forceinline__ int slot(int j) const { return j < lo ? j : j - (int)n; }
};

// An inner term outside the fast 64-bit window (far tails): the exact 64-bit
// conversion, or beyond its range (or non-finite) the workgroup's global row.
__device__ __forceinline__ void hyb_wide(const Hyb& H, int j, double k, double g) {
  const double x = k * g;
  unsigned long long v;
  if (fixed_exact(x, v)) {
    __hip_atomic_fetch_add(&H.in[j - H.lo], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  } else {
    atomicAdd(&H.ovf[j], (float)x);
    *H.flag = 1u;
  }
}

// One term of a sample: a 64-bit add for an inner target inside the fast
// window, an FP32 add (the LDS's own float atomic, cheap for the few lanes
// that take it) for an outer target; both run predicated per lane, without
// a branch.  Returns whether the term needs hyb_wide.
__device__ __forceinline__ bool hyb_term(const Hyb& H, int j, double k, double g) {
  const long long d = fixed_of(k, g);
  const bool in = H.inner(j);
  const bool fast = in && in_fixed_window(d);
  if (fast) __hip_atomic_fetch_add(&H.in[j - H.lo], (unsigned long long)d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  if (!in) atomicAdd(&H.out[H.slot(j)], (float)(k * g));
  return in && !fast;
}

// The four terms of a sample (the rare wide inner terms after a wavefront
// test).
__device__ __forceinline__ void scatter_hybrid(const Hyb& H, int a, int b, int as, int bs, double kas, double kbs,
                                               double ka, double kb, float g) {
  const double gd = (double)g;
  const bool w0 = hyb_term(H, as, kas, gd), w1 = hyb_term(H, bs, kbs, gd);
  const bool w2 = hyb_term(H, a, -ka, gd), w3 = hyb_term(H, b, -kb, gd);
  if (__any(w0 || w1 || w2 || w3)) {
    if (w0) hyb_wide(H, as, kas, gd);
    if (w1) hyb_wide(H, bs, kbs, gd);
    if (w2) hyb_wide(H, a, -ka, gd);
    if (w3) hyb_wide(H, b, -kb, gd);
  }
}

// ACC_PART state of one cell: accumulators acc[node]; h^s of nodes lo ..
// lo + n - 1 in tile[node - lo] (LDS), of the others in hg[node] (the
// cell's row in global memory); ovf, flag: the workgroup's global row for
// terms beyond the 64-bit range, as in ACC_HYBRID.
struct Part {
  unsigned long long* acc;
  float* tile;
  const float* hg;
  int lo;
  unsigned n;
  float* ovf;
  unsigned* flag;
  __device__ __forceinline__ bool inner(int j) const { return (unsigned)(j - lo) < n; }
};

// A term outside the fast window: the exact 64-bit conversion, or beyond its
// range (or non-finite) the workgroup's global row.
__device__ __forceinline__ void part_wide(const Part& Q, int j, double k, double g) {
  const double x = k * g;
  unsigned long long v;
  if (fixed_exact(x, v)) {
    __hip_atomic_fetch_add(&Q.acc[j], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  } else {
    atomicAdd(&Q.ovf[j], (float)x);
    *Q.flag = 1u;
  }
}

// The four terms of a sample, 64-bit adds at every target; the wide terms
// (far tails) after a wavefront test.
__device__ __forceinline__ void scatter_part(const Part& Q, int a, int b, int as, int bs, double kas, double kbs,
                                             double ka, double kb, float g) {
  const double gd = (double)g;
  const long long d0 = fixed_of(kas, gd), d1 = fixed_of(kbs, gd), d2 = fixed_of(-ka, gd), d3 = fixed_of(-kb, gd);
  const bool f0 = in_fixed_window(d0), f1 = in_fixed_window(d1), f2 = in_fixed_window(d2), f3 = in_fixed_window(d3);
  if (__all(f0 & f1 & f2 & f3)) {
    __hip_atomic_fetch_add(&Q.acc[as], (unsigned long long)d0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add(&Q.acc[bs], (unsigned long long)d1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add(&Q.acc[a], (unsigned long long)d2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add(&Q.acc[b], (unsigned long long)d3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  } else {
    if (f0) __hip_atomic_fetch_add(&Q.acc[as], (unsigned long long)d0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else part_wide(Q, as, kas, gd);
    if (f1) __hip_atomic_fetch_add(&Q.acc[bs], (unsigned long long)d1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else part_wide(Q, bs, kbs, gd);
    if (f2) __hip_atomic_fetch_add(&Q.acc[a], (unsigned long long)d2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else part_wide(Q, a, -ka, gd);
    if (f3) __hip_atomic_fetch_add(&Q.acc[b], (unsigned long long)d3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else part_wide(Q, b, -kb, gd);
  }
}

// nodes per thread of one ACC_SPLIT half kept in registers between passes
template <int BLOCK>
constexpr int split_regs() { return 8192 / BLOCK; }

// float4 registers per thread holding the next cell's h^s tile: 4, or with
// 1024 threads 2 (enough for 8192 nodes), 4 for the full 24^3 tile of
// ACC_HYBRID, 3 for the 20 inner slabs of ACC_PART at 24^3
template <int BLOCK, int MODE = ACC_FIXED>
constexpr int prefetch_regs() {
  return BLOCK < 1024 ? 4 : (MODE == ACC_HYBRID ? 4 : (MODE == ACC_PART ? 3 : 2));
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

template <int NR>
struct Prefetch {
  f32x4 r[NR];
  // every lane loads (indices clamped into the tile) so the registers are
  // always defined and the loads stay in flight until the next tile store
  // (loads under a branch each wait for the previous one: the compiler
  // cannot tell that the registers' earlier loads have retired).  The
  // loads, like the stores of h^{n+1}, are non-temporal: each tile is read
  // once, and the shared pair records, read by every cell, stay in L2.
  __device__ __forceinline__ void load(const float* src, int i, int stride, int n) {
    const f32x4* s4 = reinterpret_cast<const f32x4*>(src);
#pragma unroll
    for (int k = 0; k < NR; ++k) r[k] = __builtin_nontemporal_load(&s4[min(i + k * stride, n - 1)]);
  }
  __device__ __forceinline__ void store(float* dst, int i, int stride, int n) const {
    f32x4* d4 = reinterpret_cast<f32x4*>(dst);
#pragma unroll
    for (int k = 0; k < NR; ++k)
      if (i + k * stride < n) d4[i + k * stride] = r[k];
  }
};

// Scatter of one sample: +k_as g at a*, +k_bs g at b*, -k_a g at a, -k_b g
// at b, in units of h (the increment Delta N / w of Eq. collision_step).
// accf: the FP32 accumulators (ACC_CAS) or the FP32 array of large values.
// ACC_SPLIT: only the nodes lo .. lo + n - 1, at index node - lo.
template <int MODE>
__device__ __forceinline__ void scatter(float* accf, unsigned long long* acc64, int lo, unsigned n, int a, int b,
                                        int as, int bs, double kas, double kbs, double ka, double kb, float g) {
  if (MODE == ACC_SPLIT) {
    // each add is skipped by the whole wavefront when none of its lanes has
    // that target in range (the shared records are sorted by target half)
    const double gd = (double)g;
    const bool ias = (unsigned)(as - lo) < n, ibs = (unsigned)(bs - lo) < n;
    const bool ia = (unsigned)(a - lo) < n, ib = (unsigned)(b - lo) < n;
    if (__any(ias)) {
      if (ias) lds_add_hybrid(acc64, accf, as - lo, kas, gd);
    }
    if (__any(ibs)) {
      if (ibs) lds_add_hybrid(acc64, accf, bs - lo, kbs, gd);
    }
    if (__any(ia)) {
      if (ia) lds_add_hybrid(acc64, accf, a - lo, -ka, gd);
    }
    if (__any(ib)) {
      if (ib) lds_add_hybrid(acc64, accf, b - lo, -kb, gd);
    }
  } else if (MODE == ACC_FIXED) {
    // the four values are formed first; when every lane has them all in the
    // fixed-point window (all but about 2% of the wavefronts) the adds run
    // without a branch per target
    const double gd = (double)g;
    const long long d0 = fixed_of(kas, gd), d1 = fixed_of(kbs, gd), d2 = fixed_of(-ka, gd), d3 = fixed_of(-kb, gd);
    const bool fast = in_fixed_window(d0) & in_fixed_window(d1) & in_fixed_window(d2) & in_fixed_window(d3);
    if (__all(fast)) {
      __hip_atomic_fetch_add(&acc64[as], (unsigned long long)d0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      __hip_atomic_fetch_add(&acc64[bs], (unsigned long long)d1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      __hip_atomic_fetch_add(&acc64[a], (unsigned long long)d2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      __hip_atomic_fetch_add(&acc64[b], (unsigned long long)d3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    } else {
      lds_add_fixed_or(acc64, accf, as, d0, kas, gd);
      lds_add_fixed_or(acc64, accf, bs, d1, kbs, gd);
      lds_add_fixed_or(acc64, accf, a, d2, -ka, gd);
      lds_add_fixed_or(acc64, accf, b, d3, -kb, gd);
    }
  } else {
    float* acc = accf;
    lds_add(&acc[as], (float)kas * g);
    lds_add(&acc[bs], (float)kbs * g);
    lds_add(&acc[a], -((float)ka * g));
    lds_add(&acc[b], -((float)kb * g));
  }
}

// S3 + S4 for one cell (Eqs. monteCarloInt, collision_step in Jacobi form):
// every sample reads the post-stream tile hs and adds its gain and loss to
// the accumulators.  TABLE: the pairs are the records of sample_kernel for
// the cell's group, four per thread and pass so that their loads and
// gathers are in flight together; else they are drawn here.
// DRAW (pairs drawn here, not TABLE): 1 the node law, 2 continuous pairs,
// 0 whichever the problem asks for (chosen once, outside the loop).
template <int BLOCK, bool TABLE, int MODE, int PU = 4, int DRAW = 0>
__device__ __forceinline__ void gain_loss(const Params& P, const TablesLDS& T, const float* hs, float* accf,
                                          unsigned long long* acc64, uint32_t group, uint32_t step,
                                          const uint2* __restrict__ tidx, const float4* __restrict__ tcoef,
                                          int lo = 0, unsigned n = 0, const Hyb* H = nullptr) {
  const int tid = threadIdx.x;
  const float epsf = (float)P.eps;
  const uint32_t nt = (uint32_t)P.n_pairs;
  if (TABLE) {
    const uint2* ri = tidx + (int64_t)group * nt;
    const float4* rk = tcoef + (int64_t)group * nt;
    // one pass: PU records per thread, loads and gathers in flight together;
    // in the masked (last) pass slots past the end of the table load and
    // add nothing
    auto pass = [&](uint32_t m, const bool masked) {
      uint2 id[PU];
      float4 kk[PU];
      bool ok[PU];
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        const uint32_t mu = m + u * BLOCK;
        ok[u] = !masked || mu < nt;
        id[u] = ok[u] ? ri[mu] : make_uint2(0u, 0u);
        kk[u] = ok[u] ? rk[mu] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
      float ha[PU], hb[PU];
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        if (MODE == ACC_SPLIT) {
          // a record with no target in this half adds nothing: its gathers
          // are skipped when that holds for the whole wavefront
          const unsigned a = id[u].x & 0xFFFFu, b = id[u].x >> 16, as = id[u].y & 0xFFFFu, bs = id[u].y >> 16;
          const bool live = ((a - (unsigned)lo) < n) | ((b - (unsigned)lo) < n) | ((as - (unsigned)lo) < n) |
                            ((bs - (unsigned)lo) < n);
          ha[u] = hb[u] = 0.0f;
          if (__any(live)) {
            ha[u] = hs[a];
            hb[u] = hs[b];
          }
        } else {
          ha[u] = hs[id[u].x & 0xFFFFu];
          hb[u] = hs[id[u].x >> 16];
        }
      }
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        const float g = (ha[u] + hb[u]) + (epsf * ha[u]) * hb[u];
        if (MODE == ACC_HYBRID) {
          if (ok[u])
            scatter_hybrid(*H, (int)(id[u].x & 0xFFFFu), (int)(id[u].x >> 16), (int)(id[u].y & 0xFFFFu),
                           (int)(id[u].y >> 16), kk[u].x, kk[u].y, kk[u].z, kk[u].w, g);
        } else if (ok[u]) {
          scatter<MODE>(accf, acc64, lo, n, (int)(id[u].x & 0xFFFFu), (int)(id[u].x >> 16),
                        (int)(id[u].y & 0xFFFFu), (int)(id[u].y >> 16), kk[u].x, kk[u].y, kk[u].z, kk[u].w, g);
        }
      }
    };
    uint32_t m = tid;
    for (; m + (PU - 1) * BLOCK < nt; m += PU * BLOCK) pass(m, false);
    if (m < nt) pass(m, true);
  } else {
    auto draw = [&](auto&& sampler) {
      for (uint32_t m = tid; m < nt; m += BLOCK) {
        const Pair p = sampler(P, T, group, step, m, nullptr);
        if (p.as >= 0) {
          const float ha = hs[p.a], hb = hs[p.b];
          const float g = (ha + hb) + (epsf * ha) * hb;
          if (MODE == ACC_HYBRID) scatter_hybrid(*H, p.a, p.b, p.as, p.bs, p.kas, p.kbs, p.ka, p.kb, g);
          else scatter<MODE>(accf, acc64, lo, n, p.a, p.b, p.as, p.bs, p.kas, p.kbs, p.ka, p.kb, g);
        }
      }
    };
    if constexpr (DRAW == 1) draw(sample_pair_node);
    else if constexpr (DRAW == 2) draw(sample_pair_continuous);
    else if (P.continuous) draw(sample_pair_continuous);
    else draw(sample_pair_node);
  }
}

// S3 + S4 in the ACC_PART layout: gain_loss with h^s of a sample's nodes
// from the LDS tile, or for the outer slabs from the cell's row in global
// memory (a load for the few lanes that need it, issued after every LDS
// gather of the pass).  BLOCK threads take part, tid = 0 .. BLOCK - 1 (a
// multiple of 64, so shared record m stays with lane m mod 64).
template <int BLOCK, bool TABLE, int PU = 4, int DRAW = 0>
__device__ __forceinline__ void gain_loss_part(const Params& P, const TablesLDS& T, const Part& Q, uint32_t group,
                                               uint32_t step, const uint2* __restrict__ tidx,
                                               const float4* __restrict__ tcoef, int tid) {
  const float epsf = (float)P.eps;
  const uint32_t nt = (uint32_t)P.n_pairs;
  if (TABLE) {
    const uint2* ri = tidx + (int64_t)group * nt;
    const float4* rk = tcoef + (int64_t)group * nt;
    auto pass = [&](uint32_t m, const bool masked) {
      uint2 id[PU];
      float4 kk[PU];
      bool ok[PU];
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        const uint32_t mu = m + u * BLOCK;
        ok[u] = !masked || mu < nt;
        id[u] = ok[u] ? ri[mu] : make_uint2(0u, 0u);
        kk[u] = ok[u] ? rk[mu] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
      float ha[PU], hb[PU];
      bool ia[PU], ib[PU];
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        const int a = (int)(id[u].x & 0xFFFFu), b = (int)(id[u].x >> 16);
        ia[u] = Q.inner(a);
        ib[u] = Q.inner(b);
        ha[u] = Q.tile[ia[u] ? a - Q.lo : 0];
        hb[u] = Q.tile[ib[u] ? b - Q.lo : 0];
      }
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        if (!ia[u]) ha[u] = Q.hg[id[u].x & 0xFFFFu];
        if (!ib[u]) hb[u] = Q.hg[id[u].x >> 16];
      }
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        const float g = (ha[u] + hb[u]) + (epsf * ha[u]) * hb[u];
        if (ok[u])
          scatter_part(Q, (int)(id[u].x & 0xFFFFu), (int)(id[u].x >> 16), (int)(id[u].y & 0xFFFFu),
                       (int)(id[u].y >> 16), kk[u].x, kk[u].y, kk[u].z, kk[u].w, g);
      }
    };
    uint32_t m = tid;
    for (; m + (PU - 1) * BLOCK < nt; m += PU * BLOCK) pass(m, false);
    if (m < nt) pass(m, true);
  } else {
    auto draw = [&](auto&& sampler) {
      for (uint32_t m = tid; m < nt; m += BLOCK) {
        const Pair p = sampler(P, T, group, step, m, nullptr);
        if (p.as >= 0) {
          const float ha = Q.inner(p.a) ? Q.tile[p.a - Q.lo] : Q.hg[p.a];
          const float hb = Q.inner(p.b) ? Q.tile[p.b - Q.lo] : Q.hg[p.b];
          const float g = (ha + hb) + (epsf * ha) * hb;
          scatter_part(Q, p.a, p.b, p.as, p.bs, p.kas, p.kbs, p.ka, p.kb, g);
        }
      }
    };
    if constexpr (DRAW == 1) draw(sample_pair_node);
    else if constexpr (DRAW == 2) draw(sample_pair_continuous);
    else if (P.continuous) draw(sample_pair_continuous);
    else draw(sample_pair_node);
  }
}

// FP64 sums of the correction (Eqs. rinorm_a, correzione), one velocity row
// (jx, jy) per thread:
//   M = M0 + eps sum_j w_j h^c_j psi_j psi_j^T  (M0 = sum w psi psi^T),
//   r = -eps sum_j w_j psi_j (h^c_j - h^s_j),  psi = (1, v, |v|^2),
// from the z moments S_p = sum_z omega_z h^c v_z^p (p <= 4) and
// R_p = sum_z omega_z (h^c - h^s) v_z^p (p <= 2) of the row, one FMA per
// moment and node with the factors omega_z v_z^p of the table zmom.  All
// threads visit the same z node at the same time, so the factors are read
// through the constant address space into scalar registers; a row is read
// four nodes at a time when nv_z is a multiple of 4 (rows 16-byte aligned,
// no bank conflicts between neighbouring rows).  acc[0..15) are the sums
// of h^c psi_k psi_l (packed k <= l), acc[15..20) those of
// (h^c - h^s) psi_k, per thread.
typedef __attribute__((address_space(4))) const double const_f64;

// The factors omega_z v_z^p (p <= 4) of four consecutive z nodes, loaded
// together before any is used: the sums then wait once per quadruple for
// the scalar loads, not once per node.
struct ZQuad {
  double f[4][5];
  __device__ __forceinline__ void load(const const_f64* zc, int jz) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int p = 0; p < 5; ++p) f[k][p] = zc[8 * (jz + k) + p];
  }
};

template <int BLOCK>
__device__ __forceinline__ void correction_sums(const TablesLDS& T, const double* zmom, const float* hs,
                                                const float* hc_t, int n0, int n1, int n2, double (&acc)[20]) {
  const double* vx = T.v;
  const double* vy = T.v + n0;
  const double* omx = T.om;
  const double* omy = T.om + n0;
  const const_f64* zc = (const const_f64*)zmom;
  const bool vec = (n2 & 3) == 0;
#pragma unroll
  for (int i = 0; i < 20; ++i) acc[i] = 0.0;
  for (int row = threadIdx.x; row < n0 * n1; row += BLOCK) {
    const int jx = row / n1, jy = row - (row / n1) * n1;
    double S0 = 0.0, S1 = 0.0, S2 = 0.0, S3 = 0.0, S4 = 0.0, R0 = 0.0, R1 = 0.0, R2 = 0.0;
    auto node = [&](int jz, float hcf, float hsf) {
      const const_f64* z = zc + 8 * jz;
      const double hc = (double)hcf, d = hc - (double)hsf;
      S0 = fma(z[0], hc, S0);
      S1 = fma(z[1], hc, S1);
      S2 = fma(z[2], hc, S2);
      S3 = fma(z[3], hc, S3);
      S4 = fma(z[4], hc, S4);
      R0 = fma(z[0], d, R0);
      R1 = fma(z[1], d, R1);
      R2 = fma(z[2], d, R2);
    };
    if (vec) {
      const f32x4* hcr = reinterpret_cast<const f32x4*>(hc_t + row * n2);
      const f32x4* hsr = reinterpret_cast<const f32x4*>(hs + row * n2);
      for (int q = 0; q < (n2 >> 2); ++q) {
        ZQuad zq;
        zq.load(zc, 4 * q);
        const f32x4 c4 = hcr[q], s4 = hsr[q];
        const float hcq[4] = {c4.x, c4.y, c4.z, c4.w}, hsq[4] = {s4.x, s4.y, s4.z, s4.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double hc = (double)hcq[k], d = hc - (double)hsq[k];
          S0 = fma(zq.f[k][0], hc, S0);
          S1 = fma(zq.f[k][1], hc, S1);
          S2 = fma(zq.f[k][2], hc, S2);
          S3 = fma(zq.f[k][3], hc, S3);
          S4 = fma(zq.f[k][4], hc, S4);
          R0 = fma(zq.f[k][0], d, R0);
          R1 = fma(zq.f[k][1], d, R1);
          R2 = fma(zq.f[k][2], d, R2);
        }
      }
    } else {
      for (int jz = 0; jz < n2; ++jz) node(jz, hc_t[row * n2 + jz], hs[row * n2 + jz]);
    }
    const double W = omx[jx] * omy[jy], a = vx[jx], b = vy[jy], c2 = a * a + b * b;
    const double T0 = W * S0, T1 = W * S1, T2 = W * S2, T3 = W * S3, T4 = W * S4;
    const double E0 = c2 * T0 + T2;  // sum w h^c |v|^2
    acc[0] += T0;
    acc[1] += a * T0;
    acc[2] += b * T0;
    acc[3] += T1;
    acc[4] += E0;
    acc[5] += (a * a) * T0;
    acc[6] += (a * b) * T0;
    acc[7] += a * T1;
    acc[8] += a * E0;
    acc[9] += (b * b) * T0;
    acc[10] += b * T1;
    acc[11] += b * E0;
    acc[12] += T2;
    acc[13] += c2 * T1 + T3;
    acc[14] += (c2 * c2) * T0 + 2.0 * c2 * T2 + T4;
    const double Q0 = W * R0, Q1 = W * R1, Q2 = W * R2;
    acc[15] += Q0;
    acc[16] += a * Q0;
    acc[17] += b * Q0;
    acc[18] += Q1;
    acc[19] += c2 * Q0 + Q2;
  }
}

// ---------------------------------------------------- ACC_HYBRID cells --
// Increment of h at node j from its accumulator (and the workgroup's global
// row when the cell used it).
__device__ __forceinline__ double hyb_dh(const Hyb& H, int j, bool flagged) {
  double dh = H.inner(j) ? from_fixed(H.in[j - H.lo]) : (double)H.out[H.slot(j)];
  if (flagged) dh += (double)H.ovf[j];
  return dh;
}

// correction_sums with h^c formed from h^s and the accumulators (rows are
// whole x-slab members, so a row is inner or outer as a whole).
template <int BLOCK>
__device__ __forceinline__ void correction_sums_hybrid(const TablesLDS& T, const double* zmom, const float* hs,
                                                       const Hyb& H, bool flagged, int n0, int n1, int n2,
                                                       double (&acc)[20]) {
  const double* vx = T.v;
  const double* vy = T.v + n0;
  const double* omx = T.om;
  const double* omy = T.om + n0;
  const const_f64* zc = (const const_f64*)zmom;
  const bool vec = (n2 & 3) == 0 && !flagged;
#pragma unroll
  for (int i = 0; i < 20; ++i) acc[i] = 0.0;
  for (int row = threadIdx.x; row < n0 * n1; row += BLOCK) {
    const int jx = row / n1, jy = row - (row / n1) * n1;
    const int j0 = row * n2;
    double S0 = 0.0, S1 = 0.0, S2 = 0.0, S3 = 0.0, S4 = 0.0, R0 = 0.0, R1 = 0.0, R2 = 0.0;
    auto node = [&](int jz, float hsf, double dh) {
      const const_f64* z = zc + 8 * jz;
      const float hcf = (float)((double)hsf + dh);
      const double hc = (double)hcf, d = hc - (double)hsf;
      S0 = fma(z[0], hc, S0);
      S1 = fma(z[1], hc, S1);
      S2 = fma(z[2], hc, S2);
      S3 = fma(z[3], hc, S3);
      S4 = fma(z[4], hc, S4);
      R0 = fma(z[0], d, R0);
      R1 = fma(z[1], d, R1);
      R2 = fma(z[2], d, R2);
    };
    if (vec) {
      const f32x4* hsr = reinterpret_cast<const f32x4*>(hs + j0);
      if (H.inner(j0)) {
        const u64x2* q = reinterpret_cast<const u64x2*>(H.in + (j0 - H.lo));
        for (int c = 0; c < (n2 >> 2); ++c) {
          const f32x4 s4 = hsr[c];
          const u64x2 qa = q[2 * c], qb = q[2 * c + 1];
          node(4 * c, s4.x, from_fixed(qa.x));
          node(4 * c + 1, s4.y, from_fixed(qa.y));
          node(4 * c + 2, s4.z, from_fixed(qb.x));
          node(4 * c + 3, s4.w, from_fixed(qb.y));
        }
      } else {
        const f32x4* o = reinterpret_cast<const f32x4*>(H.out + H.slot(j0));
        for (int c = 0; c < (n2 >> 2); ++c) {
          const f32x4 s4 = hsr[c], o4 = o[c];
          node(4 * c, s4.x, (double)o4.x);
          node(4 * c + 1, s4.y, (double)o4.y);
          node(4 * c + 2, s4.z, (double)o4.z);
          node(4 * c + 3, s4.w, (double)o4.w);
        }
      }
    } else {
      for (int jz = 0; jz < n2; ++jz) node(jz, hs[j0 + jz], hyb_dh(H, j0 + jz, flagged));
    }
    const double W = omx[jx] * omy[jy], a = vx[jx], b = vy[jy], c2 = a * a + b * b;
    const double T0 = W * S0, T1 = W * S1, T2 = W * S2, T3 = W * S3, T4 = W * S4;
    const double E0 = c2 * T0 + T2;
    acc[0] += T0;
    acc[1] += a * T0;
    acc[2] += b * T0;
    acc[3] += T1;
    acc[4] += E0;
    acc[5] += (a * a) * T0;
    acc[6] += (a * b) * T0;
    acc[7] += a * T1;
    acc[8] += a * E0;
    acc[9] += (b * b) * T0;
    acc[10] += b * T1;
    acc[11] += b * E0;
    acc[12] += T2;
    acc[13] += c2 * T1 + T3;
    acc[14] += (c2 * c2) * T0 + 2.0 * c2 * T2 + T4;
    const double Q0 = W * R0, Q1 = W * R1, Q2 = W * R2;
    acc[15] += Q0;
    acc[16] += a * Q0;
    acc[17] += b * Q0;
    acc[18] += Q1;
    acc[19] += c2 * Q0 + Q2;
  }
}

// One cell in the ACC_HYBRID layout (h^s tile in LDS, accumulators cleared,
// a barrier passed): S3 + S4 pair pass, S5 sums and solve with h^c formed
// from h^s and the accumulators, then the store pass, which forms h^c once
// more, applies the correction, writes h^{n+1} and clears the accumulators
// (and the global row when used).  next(): after the pair pass.  Ends with
// a barrier.
template <int BLOCK, bool TABLE, int DRAW = 0, class Next>
__device__ __forceinline__ void collide_body_hybrid(const Params& P, const TablesLDS& T, float* hs, const Hyb& H,
                                                    double* red, uint32_t group, uint32_t step, uint32_t flags,
                                                    float* dst, double* defect, const uint2* __restrict__ tidx,
                                                    const float4* __restrict__ tcoef, Next&& next) {
  const int tid = threadIdx.x;
  const int nv = P.nv, n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
  const bool correct = !(flags & 1u);
  const bool vec4 = ((n2 & 3) == 0) && ((reinterpret_cast<uintptr_t>(dst) & 15) == 0);
  const double eps = P.eps;
  gain_loss<BLOCK, TABLE, ACC_HYBRID, 4, DRAW>(P, T, hs, nullptr, nullptr, group, step, tidx, tcoef, 0, 0u, &H);
  __syncthreads();
  next();
  const bool flagged = *H.flag != 0u;
  if (correct) {
    double acc[20];
    correction_sums_hybrid<BLOCK>(T, P.zmom, hs, H, flagged, n0, n1, n2, acc);
    const int rows = n0 * n1;
    const double t = block_sum20_w0<BLOCK>(acc, red, rows >= BLOCK ? BLOCK / 64 : (rows + 63) / 64);
    const const_f64* m0c = (const const_f64*)P.m0;
    if (tid < 64) {
      double M[15], r[5], x[5];
#pragma unroll
      for (int k = 0; k < 15; ++k) M[k] = m0c[k] + eps * lane_value(t, k);
#pragma unroll
      for (int k = 0; k < 5; ++k) r[k] = -eps * lane_value(t, 15 + k);
      if (!solve5(M, r, x)) {
#pragma unroll
        for (int k = 0; k < 5; ++k) x[k] = 0.0;
        if (tid == 0) atomicOr(P.status, 1u);
      }
      for (int i = tid; i < n0 + n1 + n2; i += 64) {
        const double v = T.v[i];
        T.xt[i] = i < n0 ? x[1] * v + x[4] * (v * v)
                         : (i < n0 + n1 ? x[2] * v + x[4] * (v * v) : x[0] + x[3] * v + x[4] * (v * v));
      }
    }
    __syncthreads();
  }
  // ---- h^{n+1} = h^c + F^c (x . psi) / eps, h^c formed again; the
  // accumulators (and the global row) are left cleared for the next cell
  bool finite = true;
  auto out_of = [&](double hc, double xpsi) { return (float)fma(fma(eps, hc, 1.0) * xpsi, P.inv_eps, hc); };
  if (vec4 && !defect && !flagged) {
    f32x4* d4 = reinterpret_cast<f32x4*>(dst);
    const f32x4* s4 = reinterpret_cast<const f32x4*>(hs);
    NodeWalk nw4(4 * tid, 4 * BLOCK, n1, n2);
#pragma unroll 1
    for (int i = tid; i < (nv >> 2); i += BLOCK, nw4.next()) {
      const int j = 4 * i;
      const f32x4 hv = s4[i];
      double dh[4];
      if (H.inner(j)) {
        u64x2* q = reinterpret_cast<u64x2*>(H.in + (j - H.lo));
        const u64x2 qa = q[0], qb = q[1];
        q[0] = u64x2{0ull, 0ull};
        q[1] = u64x2{0ull, 0ull};
        dh[0] = from_fixed(qa.x);
        dh[1] = from_fixed(qa.y);
        dh[2] = from_fixed(qb.x);
        dh[3] = from_fixed(qb.y);
      } else {
        f32x4* o = reinterpret_cast<f32x4*>(H.out + H.slot(j));
        const f32x4 ov = o[0];
        o[0] = f32x4{0.f, 0.f, 0.f, 0.f};
        dh[0] = ov.x;
        dh[1] = ov.y;
        dh[2] = ov.z;
        dh[3] = ov.w;
      }
      const float c0 = (float)((double)hv.x + dh[0]), c1 = (float)((double)hv.y + dh[1]);
      const float c2 = (float)((double)hv.z + dh[2]), c3 = (float)((double)hv.w + dh[3]);
      f32x4 o;
      if (correct) {
        const double xa = T.xt[nw4.jx] + T.xt[n0 + nw4.jy];
        const double* xz = T.xt + n0 + n1 + nw4.jz;
        o.x = out_of((double)c0, xa + xz[0]);
        o.y = out_of((double)c1, xa + xz[1]);
        o.z = out_of((double)c2, xa + xz[2]);
        o.w = out_of((double)c3, xa + xz[3]);
      } else {
        o = f32x4{c0, c1, c2, c3};
      }
      finite = finite && isfinite(o.x) && isfinite(o.y) && isfinite(o.z) && isfinite(o.w);
      __builtin_nontemporal_store(o, &d4[i]);
    }
  } else {
    const double* vx = T.v;
    const double* vy = T.v + n0;
    const double* vz = T.v + n0 + n1;
    const double* omx = T.om;
    const double* omy = T.om + n0;
    const double* omz = T.om + n0 + n1;
    double dsum[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    NodeWalk nw2(tid, BLOCK, n1, n2);
#pragma unroll 1
    for (int j = tid; j < nv; j += BLOCK, nw2.next()) {
      const int jx = nw2.jx, jy = nw2.jy, jz = nw2.jz;
      const float hsj = hs[j];
      const double hc = (double)(float)((double)hsj + hyb_dh(H, j, flagged));
      if (H.inner(j)) H.in[j - H.lo] = 0ull;
      else H.out[H.slot(j)] = 0.0f;
      if (flagged) H.ovf[j] = 0.0f;
      float out = (float)hc;
      if (correct) out = out_of(hc, (T.xt[jx] + T.xt[n0 + jy]) + T.xt[n0 + n1 + jz]);
      finite = finite && isfinite(out);
      dst[j] = out;
      if (defect) {
        const double v1 = vx[jx], v2 = vy[jy], v3 = vz[jz];
        const double vv = fma(v1, v1, fma(v2, v2, v3 * v3));
        const double w = (omx[jx] * omy[jy]) * omz[jz];
        const double diff = eps * ((double)out - (double)hsj) * w;
        dsum[0] += diff;
        dsum[1] += v1 * diff;
        dsum[2] += v2 * diff;
        dsum[3] += v3 * diff;
        dsum[4] += vv * diff;
      }
    }
    if (defect) {
      block_sum<5>(dsum, red);
      if (tid < 5) defect[tid] = dsum[tid];
    }
  }
  if (!finite) atomicOr(P.status, 2u);
  __syncthreads();
}

// ---------------------------------------------------- ACC_PART cells --
// correction_sums with h^c formed from h^s (LDS tile or global row) and the
// 64-bit accumulators (rows are whole x-slab members, so a row's h^s comes
// from one place).  With whole z quadruples and no overflow row, wavefronts
// take units of work: 64 inner rows (whole rows from the tile), or 64 outer
// rows times one pair of z quadruples (from global memory, both loads in
// flight together, where one thread per outer row would wait for n2/4 loads
// one after another).  The quadruples of a unit are the same for all its
// lanes, so their z factors are scalar loads.  The row terms are linear in a
// row's z sums, so every unit adds its own part.  keep (the vector store
// pass follows): the inner units write h^c over h^s in the tile and clear
// their accumulators.  Returns the number of threads that hold sums (a
// multiple of 64, or n0 * n1).
template <int BLOCK>
__device__ __forceinline__ int correction_sums_part(const TablesLDS& T, const double* zmom, const Part& Q,
                                                    bool flagged, bool vec, int n0, int n1, int n2,
                                                    double (&acc)[20], bool keep) {
  const double* vx = T.v;
  const double* vy = T.v + n0;
  const double* omx = T.om;
  const double* omy = T.om + n0;
  const const_f64* zc = (const const_f64*)zmom;
#pragma unroll
  for (int i = 0; i < 20; ++i) acc[i] = 0.0;
  // the terms of row (jx, jy) from its z sums: S of h^c, R of h^c - h^s
  auto add_row = [&](int jx, int jy, double S0, double S1, double S2, double S3, double S4, double R0, double R1,
                     double R2) {
    const double W = omx[jx] * omy[jy], a = vx[jx], b = vy[jy], c2 = a * a + b * b;
    const double T0 = W * S0, T1 = W * S1, T2 = W * S2, T3 = W * S3, T4 = W * S4;
    const double E0 = c2 * T0 + T2;
    acc[0] += T0;
    acc[1] += a * T0;
    acc[2] += b * T0;
    acc[3] += T1;
    acc[4] += E0;
    acc[5] += (a * a) * T0;
    acc[6] += (a * b) * T0;
    acc[7] += a * T1;
    acc[8] += a * E0;
    acc[9] += (b * b) * T0;
    acc[10] += b * T1;
    acc[11] += b * E0;
    acc[12] += T2;
    acc[13] += c2 * T1 + T3;
    acc[14] += (c2 * c2) * T0 + 2.0 * c2 * T2 + T4;
    const double Q0 = W * R0, Q1 = W * R1, Q2 = W * R2;
    acc[15] += Q0;
    acc[16] += a * Q0;
    acc[17] += b * Q0;
    acc[18] += Q1;
    acc[19] += c2 * Q0 + Q2;
  };
  if (vec && !flagged) {
    const int nq = n2 >> 2;
    // inner rows r_lo .. r_hi - 1 (the tile holds whole x slabs)
    const int r_lo = Q.lo / n2, r_hi = (Q.lo + (int)Q.n) / n2;
    const int n_in = r_hi - r_lo, n_out = n0 * n1 - n_in;
    const int w_in = (n_in + 63) >> 6, b_out = (n_out + 63) >> 6, g_out = (nq + 1) >> 1;
    const int units = w_in + g_out * b_out;
    const int lane = (int)threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const f32x4* g4 = reinterpret_cast<const f32x4*>(Q.hg);
    for (int un = wid; un < units; un += BLOCK / 64) {
      double S0 = 0.0, S1 = 0.0, S2 = 0.0, S3 = 0.0, S4 = 0.0, R0 = 0.0, R1 = 0.0, R2 = 0.0;
      // quadruple c (uniform) of a row: s4 its h^s, q the row's
      // accumulators; with hc4, h^c goes back to the tile in place of h^s and
      // the accumulators are cleared (the store pass then reads h^c there)
      auto quad = [&](int c, const f32x4 s4, u64x2* q, f32x4* hc4) {
        ZQuad zq;
        zq.load(zc, 4 * c);
        const u64x2 qa = q[2 * c], qb = q[2 * c + 1];
        const float hsq[4] = {s4.x, s4.y, s4.z, s4.w};
        const double dhq[4] = {from_fixed(qa.x), from_fixed(qa.y), from_fixed(qb.x), from_fixed(qb.y)};
        float hcq[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float hcf = (float)((double)hsq[k] + dhq[k]);
          hcq[k] = hcf;
          const double hc = (double)hcf, d = hc - (double)hsq[k];
          S0 = fma(zq.f[k][0], hc, S0);
          S1 = fma(zq.f[k][1], hc, S1);
          S2 = fma(zq.f[k][2], hc, S2);
          S3 = fma(zq.f[k][3], hc, S3);
          S4 = fma(zq.f[k][4], hc, S4);
          R0 = fma(zq.f[k][0], d, R0);
          R1 = fma(zq.f[k][1], d, R1);
          R2 = fma(zq.f[k][2], d, R2);
        }
        if (hc4) {
          hc4[c] = f32x4{hcq[0], hcq[1], hcq[2], hcq[3]};
          q[2 * c] = u64x2{0ull, 0ull};
          q[2 * c + 1] = u64x2{0ull, 0ull};
        }
      };
      if (un < w_in) {
        const int i = un * 64 + lane;
        if (i < n_in) {
          const int row = r_lo + i;
          f32x4* hsr = reinterpret_cast<f32x4*>(Q.tile) + ((row * n2 - Q.lo) >> 2);
          u64x2* q = reinterpret_cast<u64x2*>(Q.acc + row * n2);
          for (int c = 0; c < nq; ++c) quad(c, hsr[c], q, keep ? hsr : nullptr);
          add_row(row / n1, row - (row / n1) * n1, S0, S1, S2, S3, S4, R0, R1, R2);
        }
      } else {
        const int v = un - w_in, g = v / b_out, o = (v - g * b_out) * 64 + lane;
        const int c0 = 2 * g;
        const bool two = c0 + 1 < nq;
        if (o < n_out) {
          const int row = o < r_lo ? o : r_hi + (o - r_lo);
          const f32x4* hsr = g4 + ((row * n2) >> 2);
          u64x2* q = reinterpret_cast<u64x2*>(Q.acc + row * n2);
          const f32x4 sa = hsr[c0], sb = hsr[two ? c0 + 1 : c0];
          quad(c0, sa, q, nullptr);
          if (two) quad(c0 + 1, sb, q, nullptr);
          add_row(row / n1, row - (row / n1) * n1, S0, S1, S2, S3, S4, R0, R1, R2);
        }
      }
    }
    return units * 64;
  }
  for (int row = threadIdx.x; row < n0 * n1; row += BLOCK) {
    const int jx = row / n1, jy = row - (row / n1) * n1;
    const int j0 = row * n2;
    const bool in = Q.inner(j0);
    double S0 = 0.0, S1 = 0.0, S2 = 0.0, S3 = 0.0, S4 = 0.0, R0 = 0.0, R1 = 0.0, R2 = 0.0;
    for (int jz = 0; jz < n2; ++jz) {
      const int j = j0 + jz;
      double dh = from_fixed(Q.acc[j]);
      if (flagged) dh += (double)Q.ovf[j];
      const float hsf = in ? Q.tile[j - Q.lo] : Q.hg[j];
      const const_f64* z = zc + 8 * jz;
      const float hcf = (float)((double)hsf + dh);
      const double hc = (double)hcf, d = hc - (double)hsf;
      S0 = fma(z[0], hc, S0);
      S1 = fma(z[1], hc, S1);
      S2 = fma(z[2], hc, S2);
      S3 = fma(z[3], hc, S3);
      S4 = fma(z[4], hc, S4);
      R0 = fma(z[0], d, R0);
      R1 = fma(z[1], d, R1);
      R2 = fma(z[2], d, R2);
    }
    add_row(jx, jy, S0, S1, S2, S3, S4, R0, R1, R2);
  }
  return n0 * n1;
}

// One cell in the ACC_PART layout (inner h^s tile in LDS, Q.hg the cell's
// row, accumulators cleared, a barrier passed): as collide_body_hybrid.
// vec: rows of whole z quadruples and a 16-byte aligned global row.
template <int BLOCK, bool TABLE, class Next, int PU = 4, int DRAW = 0>
__device__ __forceinline__ void collide_body_part(const Params& P, const TablesLDS& T, const Part& Q, double* red,
                                                  bool vec, uint32_t group, uint32_t step, uint32_t flags,
                                                  float* dst, double* defect, const uint2* __restrict__ tidx,
                                                  const float4* __restrict__ tcoef, Next&& next) {
  const int tid = threadIdx.x;
  const int nv = P.nv, n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
  const bool correct = !(flags & 1u);
  const bool vec4 = vec && ((reinterpret_cast<uintptr_t>(dst) & 15) == 0);
  const double eps = P.eps;
  gain_loss_part<BLOCK, TABLE, PU, DRAW>(P, T, Q, group, step, tidx, tcoef, tid);
  __syncthreads();
  next();
  const bool flagged = *Q.flag != 0u;
  // the row sums leave h^c of the inner slabs in the tile (and their
  // accumulators cleared) when the vector store below follows them
  const bool hc_tile = correct && vec4 && !defect && !flagged;
  if (correct) {
    double acc[20];
    const int items = correction_sums_part<BLOCK>(T, P.zmom, Q, flagged, vec, n0, n1, n2, acc, hc_tile);
    const double t = block_sum20_w0<BLOCK>(acc, red, items >= BLOCK ? BLOCK / 64 : (items + 63) / 64);
    const const_f64* m0c = (const const_f64*)P.m0;
    if (tid < 64) {
      double M[15], r[5], x[5];
#pragma unroll
      for (int k = 0; k < 15; ++k) M[k] = m0c[k] + eps * lane_value(t, k);
#pragma unroll
      for (int k = 0; k < 5; ++k) r[k] = -eps * lane_value(t, 15 + k);
      if (!solve5(M, r, x)) {
#pragma unroll
        for (int k = 0; k < 5; ++k) x[k] = 0.0;
        if (tid == 0) atomicOr(P.status, 1u);
      }
      for (int i = tid; i < n0 + n1 + n2; i += 64) {
        const double v = T.v[i];
        T.xt[i] = i < n0 ? x[1] * v + x[4] * (v * v)
                         : (i < n0 + n1 ? x[2] * v + x[4] * (v * v) : x[0] + x[3] * v + x[4] * (v * v));
      }
    }
    __syncthreads();
  }
  // ---- h^{n+1} = h^c + F^c (x . psi) / eps, h^c formed again; the
  // accumulators (and the global row) are left cleared for the next cell.
  // Each thread reads a node's h^s before it writes that node's output, so
  // h_s may be the output array.
  bool finite = true;
  auto out_of = [&](double hc, double xpsi) { return (float)fma(fma(eps, hc, 1.0) * xpsi, P.inv_eps, hc); };
  if (vec4 && !defect && !flagged) {
    f32x4* d4 = reinterpret_cast<f32x4*>(dst);
    const f32x4* t4 = reinterpret_cast<const f32x4*>(Q.tile);
    const f32x4* g4 = reinterpret_cast<const f32x4*>(Q.hg);
    NodeWalk nw4(4 * tid, 4 * BLOCK, n1, n2);
#pragma unroll 1
    for (int i = tid; i < (nv >> 2); i += BLOCK, nw4.next()) {
      const int j = 4 * i;
      const bool in = Q.inner(j);
      const f32x4 hv = in ? t4[(j - Q.lo) >> 2] : g4[i];
      float c0, c1, c2, c3;
      if (hc_tile && in) {
        // h^c, formed by the row sums
        c0 = hv.x;
        c1 = hv.y;
        c2 = hv.z;
        c3 = hv.w;
      } else {
        u64x2* q = reinterpret_cast<u64x2*>(Q.acc + j);
        const u64x2 qa = q[0], qb = q[1];
        q[0] = u64x2{0ull, 0ull};
        q[1] = u64x2{0ull, 0ull};
        c0 = (float)((double)hv.x + from_fixed(qa.x));
        c1 = (float)((double)hv.y + from_fixed(qa.y));
        c2 = (float)((double)hv.z + from_fixed(qb.x));
        c3 = (float)((double)hv.w + from_fixed(qb.y));
      }
      f32x4 o;
      if (correct) {
        const double xa = T.xt[nw4.jx] + T.xt[n0 + nw4.jy];
        const double* xz = T.xt + n0 + n1 + nw4.jz;
        o.x = out_of((double)c0, xa + xz[0]);
        o.y = out_of((double)c1, xa + xz[1]);
        o.z = out_of((double)c2, xa + xz[2]);
        o.w = out_of((double)c3, xa + xz[3]);
      } else {
        o = f32x4{c0, c1, c2, c3};
      }
      finite = finite && isfinite(o.x) && isfinite(o.y) && isfinite(o.z) && isfinite(o.w);
      __builtin_nontemporal_store(o, &d4[i]);
    }
  } else {
    const double* vx = T.v;
    const double* vy = T.v + n0;
    const double* vz = T.v + n0 + n1;
    const double* omx = T.om;
    const double* omy = T.om + n0;
    const double* omz = T.om + n0 + n1;
    double dsum[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    NodeWalk nw2(tid, BLOCK, n1, n2);
#pragma unroll 1
    for (int j = tid; j < nv; j += BLOCK, nw2.next()) {
      const int jx = nw2.jx, jy = nw2.jy, jz = nw2.jz;
      const float hsj = Q.inner(j) ? Q.tile[j - Q.lo] : Q.hg[j];
      double dh = from_fixed(Q.acc[j]);
      Q.acc[j] = 0ull;
      if (flagged) {
        dh += (double)Q.ovf[j];
        Q.ovf[j] = 0.0f;
      }
      const double hc = (double)(float)((double)hsj + dh);
      float out = (float)hc;
      if (correct) out = out_of(hc, (T.xt[jx] + T.xt[n0 + jy]) + T.xt[n0 + n1 + jz]);
      finite = finite && isfinite(out);
      dst[j] = out;
      if (defect) {
        const double v1 = vx[jx], v2 = vy[jy], v3 = vz[jz];
        const double vv = fma(v1, v1, fma(v2, v2, v3 * v3));
        const double w = (omx[jx] * omy[jy]) * omz[jz];
        const double diff = eps * ((double)out - (double)hsj) * w;
        dsum[0] += diff;
        dsum[1] += v1 * diff;
        dsum[2] += v2 * diff;
        dsum[3] += v3 * diff;
        dsum[4] += vv * diff;
      }
    }
    if (defect) {
      block_sum<5>(dsum, red);
      if (tid < 5) defect[tid] = dsum[tid];
    }
  }
  if (!finite) atomicOr(P.status, 2u);
  __syncthreads();
}

// One cell after its h^s tile is in LDS and the accumulators are cleared
// (and a barrier passed): S3 + S4 pair pass, h^c, S5 correction, one
// coalesced store of h^{n+1} to dst.  next() is called once the pair pass is
// over (the persistent kernel requests the next tile there); early() is
// called by every thread while wavefront 0 solves for the correction (the
// others right away), after the last reads of h^s and of the 64-bit
// accumulators (the persistent kernel stages the next cell there); defect:
// the cell's five values or null.  Ends with a barrier, so the LDS can be
// refilled.
template <int BLOCK, bool TABLE, int MODE, int PU = 4, int DRAW = 0, class Next, class Early>
__device__ __forceinline__ void collide_body(const Params& P, const TablesLDS& T, float* hs, float* accf,
                                             unsigned long long* acc64, double* red, uint32_t group,
                                             uint32_t step, uint32_t flags, float* dst, double* defect,
                                             const uint2* __restrict__ tidx, const float4* __restrict__ tcoef,
                                             Next&& next, Early&& early) {
  const int tid = threadIdx.x;
  const int nv = P.nv, n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
  const double* vx = T.v;
  const double* vy = T.v + n0;
  const double* vz = T.v + n0 + n1;
  const double* omx = T.om;
  const double* omy = T.om + n0;
  const double* omz = T.om + n0 + n1;
  // node loops are unrolled where the register budget allows it (at most
  // 256 VGPRs below 1024 threads per workgroup, 128 at 1024)
  constexpr int NU = BLOCK <= 512 ? 4 : 1;
  const bool correct = !(flags & 1u);
  // node phases four nodes at a time: rows of whole z quadruples and an
  // output tile on a 16-byte boundary
  const bool vec4 = ((n2 & 3) == 0) && ((reinterpret_cast<uintptr_t>(dst) & 15) == 0);
  const double eps = P.eps;
  // ---- S3 + S4: Jacobi gain/loss, every sample reads the post-stream h
  if (MODE == ACC_SPLIT) {
    // two passes over the samples, one half of the nodes each; h^c of the
    // halves waits in registers, then goes over the accumulators
    constexpr int R = split_regs<BLOCK>();
    const int h2 = CollideLDS::half(nv);
    float* ovf = reinterpret_cast<float*>(reinterpret_cast<unsigned char*>(acc64) + CollideLDS::split64(nv));
    float hc0[R], hc1[R];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int lo = p * h2, n = min(nv - lo, h2);
      if (p == 1) {
        uint4* z = reinterpret_cast<uint4*>(acc64);
        const int nz = (int)(CollideLDS::acc(nv, ACC_SPLIT) / 16);
        for (int i = tid; i < nz; i += BLOCK) z[i] = make_uint4(0u, 0u, 0u, 0u);
        __syncthreads();
      }
      gain_loss<BLOCK, TABLE, ACC_SPLIT, PU, DRAW>(P, T, hs, ovf, acc64, group, step, tidx, tcoef, lo, (unsigned)n);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const int i = tid + k * BLOCK;
        float v = 0.0f;
        if (i < n) v = (float)((double)hs[lo + i] + ((double)ovf[i] + from_fixed(acc64[i])));
        if (p == 0) hc0[k] = v;
        else hc1[k] = v;
      }
      __syncthreads();
    }
    next();
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int i = tid + k * BLOCK;
      if (i < h2) accf[i] = hc0[k];
      if (i < nv - h2) accf[h2 + i] = hc1[k];
    }
    __syncthreads();
  } else {
    gain_loss<BLOCK, TABLE, MODE, PU, DRAW>(P, T, hs, accf, acc64, group, step, tidx, tcoef);
    __syncthreads();
    next();
    // ---- S5 (1): h^c = h^s + increment, stored over the FP32 accumulator;
    // the 64-bit accumulators are left cleared for the next cell
    auto hc_of = [&](float hsj, float a, unsigned long long q) {
      double dh = (double)a;
      if (MODE == ACC_FIXED) dh += from_fixed(q);
      return (float)((double)hsj + dh);
    };
    if (vec4) {
      // four nodes per thread and access
      f32x4* a4 = reinterpret_cast<f32x4*>(accf);
      const f32x4* s4 = reinterpret_cast<const f32x4*>(hs);
      u64x2* q2 = reinterpret_cast<u64x2*>(acc64);
#pragma unroll NU
      for (int i = tid; i < (nv >> 2); i += BLOCK) {
        const f32x4 hv = s4[i];
        f32x4 av = a4[i];
        u64x2 q0 = {0ull, 0ull}, q1 = {0ull, 0ull};
        if (MODE == ACC_FIXED) {
          q0 = q2[2 * i];
          q1 = q2[2 * i + 1];
          q2[2 * i] = u64x2{0ull, 0ull};
          q2[2 * i + 1] = u64x2{0ull, 0ull};
        }
        av.x = hc_of(hv.x, av.x, q0.x);
        av.y = hc_of(hv.y, av.y, q0.y);
        av.z = hc_of(hv.z, av.z, q1.x);
        av.w = hc_of(hv.w, av.w, q1.y);
        a4[i] = av;
      }
    } else {
#pragma unroll NU
      for (int j = tid; j < nv; j += BLOCK) {
        unsigned long long q = 0ull;
        if (MODE == ACC_FIXED) {
          q = acc64[j];
          acc64[j] = 0ull;
        }
        accf[j] = hc_of(hs[j], accf[j], q);
      }
    }
  }
  if (correct) {
    __syncthreads();
    // (2) FP64 sums of M and r, block-reduced
    double acc[20];
    correction_sums<BLOCK>(T, P.zmom, hs, accf, n0, n1, n2, acc);
    // wavefronts past the last velocity row hold zeros and stay out
    const int rows = n0 * n1;
    const double t = block_sum20_w0<BLOCK>(acc, red, rows >= BLOCK ? BLOCK / 64 : (rows + 63) / 64);
    // M0 through the constant address space (scalar loads): the other
    // wavefronts may be filling the LDS for the next cell meanwhile
    const const_f64* m0c = (const const_f64*)P.m0;
    if (tid < 64) {
      // wavefront 0 solves M x = r and tabulates x . psi per axis:
      // x1 v_x + x4 v_x^2, x2 v_y + x4 v_y^2, x0 + x3 v_z + x4 v_z^2
      double M[15], r[5], x[5];
#pragma unroll
      for (int k = 0; k < 15; ++k) M[k] = m0c[k] + eps * lane_value(t, k);
#pragma unroll
      for (int k = 0; k < 5; ++k) r[k] = -eps * lane_value(t, 15 + k);
      if (!solve5(M, r, x)) {
#pragma unroll
        for (int k = 0; k < 5; ++k) x[k] = 0.0;
        if (tid == 0) atomicOr(P.status, 1u);
      }
      for (int i = tid; i < n0 + n1 + n2; i += 64) {
        const double v = T.v[i];
        T.xt[i] = i < n0 ? x[1] * v + x[4] * (v * v)
                         : (i < n0 + n1 ? x[2] * v + x[4] * (v * v) : x[0] + x[3] * v + x[4] * (v * v));
      }
    }
    early();
    __syncthreads();
  }
  // ---- (3) h^{n+1} = h^c + F^c (x . psi) / eps, one coalesced store; the
  // FP32 array is left cleared for the next cell
  bool finite = true;
  auto out_of = [&](double hc, double xpsi) { return (float)fma(fma(eps, hc, 1.0) * xpsi, P.inv_eps, hc); };
  if (vec4 && !defect) {
    // four nodes (one z quadruple of a row) per thread and access
    f32x4* a4 = reinterpret_cast<f32x4*>(accf);
    f32x4* d4 = reinterpret_cast<f32x4*>(dst);
    NodeWalk nw4(4 * tid, 4 * BLOCK, n1, n2);
    if (correct) {
#pragma unroll NU
      for (int i = tid; i < (nv >> 2); i += BLOCK, nw4.next()) {
        const f32x4 c = a4[i];
        a4[i] = f32x4{0.f, 0.f, 0.f, 0.f};
        const double xa = T.xt[nw4.jx] + T.xt[n0 + nw4.jy];
        const double* xz = T.xt + n0 + n1 + nw4.jz;
        f32x4 o;
        o.x = out_of((double)c.x, xa + xz[0]);
        o.y = out_of((double)c.y, xa + xz[1]);
        o.z = out_of((double)c.z, xa + xz[2]);
        o.w = out_of((double)c.w, xa + xz[3]);
        finite = finite && isfinite(o.x) && isfinite(o.y) && isfinite(o.z) && isfinite(o.w);
        __builtin_nontemporal_store(o, &d4[i]);
      }
    } else {
#pragma unroll NU
      for (int i = tid; i < (nv >> 2); i += BLOCK) {
        const f32x4 c = a4[i];
        a4[i] = f32x4{0.f, 0.f, 0.f, 0.f};
        finite = finite && isfinite(c.x) && isfinite(c.y) && isfinite(c.z) && isfinite(c.w);
        __builtin_nontemporal_store(c, &d4[i]);
      }
    }
  } else {
    double dsum[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    NodeWalk nw2(tid, BLOCK, n1, n2);
#pragma unroll NU
    for (int j = tid; j < nv; j += BLOCK, nw2.next()) {
      const int jx = nw2.jx, jy = nw2.jy, jz = nw2.jz;
      const double hc = (double)accf[j];
      accf[j] = 0.0f;
      float out = (float)hc;
      if (correct) out = out_of(hc, (T.xt[jx] + T.xt[n0 + jy]) + T.xt[n0 + n1 + jz]);
      finite = finite && isfinite(out);
      dst[j] = out;
      if (defect) {
        const double v1 = vx[jx], v2 = vy[jy], v3 = vz[jz];
        const double vv = fma(v1, v1, fma(v2, v2, v3 * v3));
        const double w = (omx[jx] * omy[jy]) * omz[jz];
        const double diff = eps * ((double)out - (double)hs[j]) * w;
        dsum[0] += diff;
        dsum[1] += v1 * diff;
        dsum[2] += v2 * diff;
        dsum[3] += v3 * diff;
        dsum[4] += vv * diff;
      }
    }
    if (defect) {
      block_sum<5>(dsum, red);
      if (tid < 5) defect[tid] = dsum[tid];
    }
  }
  if (!finite) atomicOr(P.status, 2u);
  __syncthreads();
}

// Persistent workgroups: workgroup b collides cells b, b + gridDim.x, ...;
// the h^s tile of the next cell is loaded into registers while the node
// phases of the current one run.  TABLE: the pairs come from the records of
// sample_kernel (cells of one group share them).  MODE: accumulation of the
// increments (ACC_FIXED, ACC_SPLIT, ACC_CAS).  h_s may equal h_out.
template <int BLOCK, bool TABLE, int MODE, int DRAW = 1>
__global__ __launch_bounds__(BLOCK) void collide_kernel(Params P, const float* hs_g, float* hout_g, uint32_t step,
                                                        uint32_t flags, double* __restrict__ defect,
                                                        const uint2* __restrict__ tidx,
                                                        const float4* __restrict__ tcoef) {
  extern __shared__ __align__(16) unsigned char dsm[];
  __shared__ double red[20 * (BLOCK / 64)];
  const int nv = P.nv;
  const int64_t ncells = (int64_t)P.nx * P.ny;
  const int tid = threadIdx.x;
  float* hs = reinterpret_cast<float*>(dsm);
  if constexpr (MODE == ACC_HYBRID) {
    // tile, 64-bit accumulators of the inner slabs, FP32 ones of the outer
    // slabs, tables; no h^c array, so the next tile goes in at the start of
    // each cell (from the registers it was loaded into during the previous
    // cell's node phases)
    __shared__ unsigned hflag[2];
    const int nin = P.hyb_n;
    Hyb H;
    H.in = reinterpret_cast<unsigned long long*>(dsm + CollideLDS::tile(nv));
    H.out = reinterpret_cast<float*>(dsm + CollideLDS::tile(nv) + CollideLDS::hyb64(nin));
    H.lo = P.hyb_lo;
    H.n = (unsigned)nin;
    H.ovf = P.hyb_ovf + (int64_t)blockIdx.x * nv;
    TablesLDS T;
    load_tables(P, dsm + CollideLDS::tile(nv) + CollideLDS::hyb_acc(nv, nin), !TABLE, T);
    {
      uint4* z = reinterpret_cast<uint4*>(dsm + CollideLDS::tile(nv));
      const int nz = (int)(CollideLDS::hyb_acc(nv, nin) / 16);
      for (int i = tid; i < nz; i += BLOCK) z[i] = make_uint4(0u, 0u, 0u, 0u);
      if (tid < 2) hflag[tid] = 0u;
    }
    const int nv4 = nv >> 2;
    constexpr int NR = prefetch_regs<BLOCK, MODE>();
    const bool vec = ((nv & 3) == 0) && nv4 <= NR * BLOCK && ((reinterpret_cast<uintptr_t>(hs_g) & 15) == 0);
    Prefetch<NR> pre;
    int64_t cell = blockIdx.x;
    if (vec && cell < ncells) pre.load(hs_g + cell * nv, tid, BLOCK, nv4);
    for (int k = 0; cell < ncells; cell += gridDim.x, ++k) {
      if (vec) {
        pre.store(hs, tid, BLOCK, nv4);
      } else {
        const float* src = hs_g + cell * nv;
        for (int j = tid; j < nv; j += BLOCK) hs[j] = src[j];
      }
      H.flag = &hflag[k & 1];
      if (tid == 0) hflag[(k + 1) & 1] = 0u;
      __syncthreads();
      const uint32_t group = (P.sample_group == 0) ? 0u : (uint32_t)(cell / P.sample_group);
      const int64_t next = cell + gridDim.x;
      collide_body_hybrid<BLOCK, TABLE, DRAW>(P, T, hs, H, red, group, step, flags, hout_g + cell * nv,
                                        defect ? defect + cell * 5 : nullptr, tidx, tcoef, [&]() {
                                          if (vec && next < ncells) pre.load(hs_g + next * nv, tid, BLOCK, nv4);
                                        });
    }
    return;
  }
  if constexpr (MODE == ACC_PART) {
    // accumulators of every node, the inner tile, tables; the next cell's
    // inner tile waits in registers during the node phases
    __shared__ unsigned pflag[2];
    const int nin = P.hyb_n;
    Part Q;
    Q.acc = reinterpret_cast<unsigned long long*>(dsm);
    Q.tile = reinterpret_cast<float*>(dsm + CollideLDS::part64(nv));
    Q.lo = P.hyb_lo;
    Q.n = (unsigned)nin;
    Q.ovf = P.hyb_ovf + (int64_t)blockIdx.x * nv;
    TablesLDS T;
    load_tables(P, dsm + CollideLDS::part64(nv) + CollideLDS::tile(nin), !TABLE, T);
    {
      uint4* z = reinterpret_cast<uint4*>(dsm);
      const int nz = (int)(CollideLDS::part64(nv) / 16);
      for (int i = tid; i < nz; i += BLOCK) z[i] = make_uint4(0u, 0u, 0u, 0u);
      if (tid < 2) pflag[tid] = 0u;
    }
    // whole z quadruples (then lo and nin are multiples of 4 as well) and
    // a 16-byte aligned input
    const bool vec = ((P.n[2] & 3) == 0) && ((reinterpret_cast<uintptr_t>(hs_g) & 15) == 0);
    const int nin4 = nin >> 2;
    constexpr int NR = prefetch_regs<BLOCK, MODE>();
    const bool pvec = vec && nin4 <= NR * BLOCK;
    Prefetch<NR> pre;
    int64_t cell = blockIdx.x;
    if (pvec && cell < ncells) pre.load(hs_g + cell * nv + Q.lo, tid, BLOCK, nin4);
    for (int k = 0; cell < ncells; cell += gridDim.x, ++k) {
      if (pvec) {
        pre.store(Q.tile, tid, BLOCK, nin4);
      } else {
        const float* src = hs_g + cell * nv + Q.lo;
        for (int j = tid; j < nin; j += BLOCK) Q.tile[j] = src[j];
      }
      Q.hg = hs_g + cell * nv;
      Q.flag = &pflag[k & 1];
      if (tid == 0) pflag[(k + 1) & 1] = 0u;
      __syncthreads();
      const uint32_t group = (P.sample_group == 0) ? 0u : (uint32_t)(cell / P.sample_group);
      const int64_t next = cell + gridDim.x;
      auto next_part = [&]() {
        if (pvec && next < ncells) pre.load(hs_g + next * nv + Q.lo, tid, BLOCK, nin4);
      };
      collide_body_part<BLOCK, TABLE, decltype(next_part)&, 4, DRAW>(
          P, T, Q, red, vec, group, step, flags, hout_g + cell * nv, defect ? defect + cell * 5 : nullptr, tidx,
          tcoef, next_part);
    }
    return;
  }
  float* accf = reinterpret_cast<float*>(dsm + CollideLDS::tile(nv));
  unsigned long long* acc64 =
      reinterpret_cast<unsigned long long*>(dsm + (MODE == ACC_SPLIT ? 1 : 2) * CollideLDS::tile(nv));
  TablesLDS T;
  load_tables(P, dsm + CollideLDS::tile(nv) + CollideLDS::acc(nv, MODE), !TABLE, T);
  const int nv4 = nv >> 2;
  constexpr int NR = prefetch_regs<BLOCK>();
  const bool vec = ((nv & 3) == 0) && nv4 <= NR * BLOCK && ((reinterpret_cast<uintptr_t>(hs_g) & 15) == 0);
  Prefetch<NR> pre;
  // byte ranges of the LDS cleared per cell: the FP32 array (h^c until the
  // store) and, with ACC_SPLIT, its accumulators; the 64-bit accumulators
  // of ACC_FIXED after the FP32 array are cleared once here, then by the
  // h^c pass of every cell as it reads them
  const size_t t0 = CollideLDS::tile(nv), t1 = MODE == ACC_SPLIT ? t0 + CollideLDS::acc(nv, MODE) : 2 * t0,
               t2 = t0 + CollideLDS::acc(nv, MODE);
  auto clear = [&](size_t from, size_t to) {
    uint4* z = reinterpret_cast<uint4*>(dsm + from);
    const int nz = (int)((to - from) / 16);
    for (int i = tid; i < nz; i += BLOCK) z[i] = make_uint4(0u, 0u, 0u, 0u);
  };
  if (t2 > t1) clear(t1, t2);
  // staged: the next cell's tile was written while wavefront 0 solved for
  // the correction of this cell (h^s is no longer read then, unless the
  // defect is asked for)
  bool staged = false;
  int64_t cell = blockIdx.x;
  if (vec && cell < ncells) pre.load(hs_g + cell * nv, tid, BLOCK, nv4);
  for (; cell < ncells; cell += gridDim.x) {
    // ---- h^s tile in, accumulators cleared
    // a staged cell finds its tile in place and the FP32 array and the
    // 64-bit accumulators cleared by the previous cell's passes
    if (!staged) {
      if (vec) {
        pre.store(hs, tid, BLOCK, nv4);
      } else {
        const float* src = hs_g + cell * nv;
        for (int j = tid; j < nv; j += BLOCK) hs[j] = src[j];
      }
      clear(t0, t1);
      __syncthreads();
    }
    const uint32_t group = (P.sample_group == 0) ? 0u : (uint32_t)(cell / P.sample_group);
    const int64_t next = cell + gridDim.x;
    staged = false;
    // The next cell's tile is requested once the pair pass is over:
    // vector-memory waits retire in issue order, so loads issued before the
    // pair loop would stall its first record loads; the node phases wait on
    // no vector load.
    collide_body<BLOCK, TABLE, MODE, 4, DRAW>(
        P, T, hs, accf, acc64, red, group, step, flags, hout_g + cell * nv, defect ? defect + cell * 5 : nullptr,
        tidx, tcoef,
        [&]() {
          if (vec && next < ncells) pre.load(hs_g + next * nv, tid, BLOCK, nv4);
        },
        [&]() {
          if (MODE != ACC_SPLIT && vec && !defect && next < ncells) {
            pre.store(hs, tid, BLOCK, nv4);
            staged = true;
          }
        });
  }
}

// ------------------------------------------------------------ batches --
// One work item of the batched collision: (problem, cell).  Workgroup b
// takes items b, b + gridDim.x, ... of a list sorted by decreasing cost, so
// every workgroup receives about the same number of pair-cells; the
// problem's tables are reloaded into LDS when it changes from one item to
// the next.  The dynamic LDS is that of the largest problem; each problem
// uses its own layout (accumulation mode, drawn or shared
// samples).  The step number is read from the device (graph replays).  PU:
// shared records per thread in flight in the pair loop.  A launch covers the
// items of one class of problems (one velocity grid).
template <int BLOCK, int PU>
__global__ __launch_bounds__(BLOCK) void collide_batch_kernel(const BatchCav* __restrict__ cavs,
                                                              const int2* __restrict__ items, int nitems,
                                                              const float* hin, float* hout,
                                                              const uint32_t* __restrict__ step_dev) {
  extern __shared__ __align__(16) unsigned char dsm[];
  __shared__ double red[20 * (BLOCK / 64)];
  __shared__ unsigned pflag;
  const int tid = threadIdx.x;
  const uint32_t step = *step_dev;
  int prev = -1;
  TablesLDS T;
  for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
    const int2 it = items[i];
    const BatchCav& C = cavs[it.x];
    const Params& P = C.P;
    const int nv = P.nv;
    const int mode = C.mode;
    const bool table = P.sample_group != 1;
    if constexpr (BLOCK == 1024) {
      if (mode == ACC_PART) {
        // the partial-tile layout (grids of one class share it); the
        // launch has at most one workgroup per row of P.hyb_ovf
        Part Q;
        Q.acc = reinterpret_cast<unsigned long long*>(dsm);
        Q.tile = reinterpret_cast<float*>(dsm + CollideLDS::part64(nv));
        Q.lo = P.hyb_lo;
        Q.n = (unsigned)P.hyb_n;
        Q.ovf = P.hyb_ovf + (int64_t)blockIdx.x * nv;
        Q.flag = &pflag;
        if (it.x != prev) {
          load_tables(P, dsm + CollideLDS::part64(nv) + CollideLDS::tile(P.hyb_n), !table, T);
          prev = it.x;
        }
        const int64_t cell = it.y;
        Q.hg = hin + C.hoff + cell * nv;
        const bool vec = ((P.n[2] & 3) == 0) && ((reinterpret_cast<uintptr_t>(Q.hg) & 15) == 0);
        if (vec) {
          const float4* s4 = reinterpret_cast<const float4*>(Q.hg + Q.lo);
          float4* d4 = reinterpret_cast<float4*>(Q.tile);
          for (int j = tid; j < (P.hyb_n >> 2); j += BLOCK) d4[j] = s4[j];
        } else {
          for (int j = tid; j < P.hyb_n; j += BLOCK) Q.tile[j] = Q.hg[Q.lo + j];
        }
        {
          uint4* z = reinterpret_cast<uint4*>(dsm);
          const int nz = (int)(CollideLDS::part64(nv) / 16);
          for (int k = tid; k < nz; k += BLOCK) z[k] = make_uint4(0u, 0u, 0u, 0u);
          if (tid == 0) pflag = 0u;
        }
        __syncthreads();
        const uint32_t group = (P.sample_group == 0) ? 0u : (uint32_t)(cell / P.sample_group);
        float* dst = hout + C.hoff + cell * nv;
        auto none = []() {};
        if (table)
          collide_body_part<BLOCK, true, decltype(none)&, PU>(P, T, Q, red, vec, group, step, 0u, dst, nullptr, C.tidx,
                                                             C.tcoef, none);
        else
          collide_body_part<BLOCK, false, decltype(none)&, PU>(P, T, Q, red, vec, group, step, 0u, dst, nullptr,
                                                              C.tidx, C.tcoef, none);
        continue;
      }
    }
    float* hs = reinterpret_cast<float*>(dsm);
    float* accf = reinterpret_cast<float*>(dsm + CollideLDS::tile(nv));
    unsigned long long* acc64 =
        reinterpret_cast<unsigned long long*>(dsm + (mode == ACC_SPLIT ? 1 : 2) * CollideLDS::tile(nv));
    if (it.x != prev) {
      load_tables(P, dsm + CollideLDS::tile(nv) + CollideLDS::acc(nv, mode), !table, T);
      prev = it.x;
    }
    const int64_t cell = it.y;
    const float* src = hin + C.hoff + cell * nv;
    if ((nv & 3) == 0) {
      const float4* s4 = reinterpret_cast<const float4*>(src);
      float4* d4 = reinterpret_cast<float4*>(hs);
      for (int j = tid; j < (nv >> 2); j += BLOCK) d4[j] = s4[j];
    } else {
      for (int j = tid; j < nv; j += BLOCK) hs[j] = src[j];
    }
    {
      uint4* z = reinterpret_cast<uint4*>(accf);
      const int nz = (int)(CollideLDS::acc(nv, mode) / 16);
      for (int k = tid; k < nz; k += BLOCK) z[k] = make_uint4(0u, 0u, 0u, 0u);
    }
    __syncthreads();
    const uint32_t group = (P.sample_group == 0) ? 0u : (uint32_t)(cell / P.sample_group);
    float* dst = hout + C.hoff + cell * nv;
    auto none = []() {};
#define BOLTZ_BODY(TB, MD)                                                                                      \
  collide_body<BLOCK, TB, MD, PU>(P, T, hs, accf, acc64, red, group, step, 0u, dst, nullptr, C.tidx, C.tcoef, none, \
                                  none)
    if (table) {
      if (mode == ACC_FIXED) BOLTZ_BODY(true, ACC_FIXED);
      else if (mode == ACC_SPLIT) BOLTZ_BODY(true, ACC_SPLIT);
      else BOLTZ_BODY(true, ACC_CAS);
    } else {
      if (mode == ACC_FIXED) BOLTZ_BODY(false, ACC_FIXED);
      else if (mode == ACC_SPLIT) BOLTZ_BODY(false, ACC_SPLIT);
      else BOLTZ_BODY(false, ACC_CAS);
    }
#undef BOLTZ_BODY
  }
}

// ------------------------------------------------ faces with samples --
// wall_kernel<PHASE> in blocks [0, 8 per_xcd) and, in the blocks after
// them, the shared pair records of the step (sample_kernel's work, dealt to
// lanes unless deal = 0; nb blocks per sample group): the records do not
// depend on h, so they are drawn while the face reductions (one workgroup
// per face) leave most of the GPU idle.  Dynamic LDS: the sampler tables.
static_assert(kWallBlock == kSampleBlock, "one block shape for faces and samples");

template <int PHASE>
__global__ __launch_bounds__(kWallBlock) void wall_sample_kernel(Params P, const float* __restrict__ h, int nface,
                                                                 int per_xcd, int nb, uint32_t step,
                                                                 uint2* __restrict__ tidx,
                                                                 float4* __restrict__ tcoef, int deal) {
  const int nwb = 8 * per_xcd;
  if ((int)blockIdx.x < nwb) {
    __shared__ double red[kWallBlock / 64];
    int f = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (f >= nface) return;
    if (PHASE == 1) f += 2 * P.ny;
    wall_face<PHASE>(P, h, f, red);
    return;
  }
  extern __shared__ __align__(16) unsigned char dsm[];
  __shared__ unsigned sh[1280];
  TablesLDS T;
  load_tables(P, dsm, true, T);
  __syncthreads();
  const int b = (int)blockIdx.x - nwb, group = b / nb;
  sample_block(P, T, step, (uint32_t)group, (int64_t)(b - group * nb) * kSampleBlock, deal != 0, tidx, tcoef, sh);
}

}  // namespace boltz
