// sequential.hpp -- the in-place sequential collision of Alg. 3 on gfx950.
//
// In Alg. 3 the samples of a cell update its h one after another: sample m
// reads the current h at its nodes a and b, forms g, and changes h at a*,
// b*, a and b before sample m + 1 reads anything.  (Eq. collision_step, the
// Jacobi form the other collision kernels implement, evaluates every sample
// at the post-stream h.)  Shared-sample mode only: the N_t records of a
// sample group are read by every cell of the group, so the order
// constraints between them are worked out once per step.
//
// Two schedules of the records, chosen per problem (boltz_create):
//   steps (seq_level_kernel, seq_steps_kernel; SCHED 1)
//                       groups of 1024 consecutive records, one workgroup
//                       each: the level of a record is 1 + the largest level
//                       among the earlier records of its group that share a
//                       node with it.  Records of one level share no node,
//                       so they can be applied together; the group is
//                       rewritten in level order and cut into steps of up to
//                       64 records, and the steps of all groups listed in
//                       order.  Applying the steps in order gives every node
//                       its updates in record order, hence the result of the
//                       sequential loop.  Where a record's nodes coincide its
//                       coefficients are merged (each slot then carries the
//                       sum over the slots of its node, signed: gain at a*,
//                       b*, loss at a, b), so the collision writes whole
//                       values.
//   groups (seq_level64_kernel; SCHED 0)
//                       the same levels within groups of 64 records, one per
//                       lane, kept in registers while the wavefront applies
//                       the group's levels one after another: more levels
//                       (a new group starts at level 1) but no loads per
//                       level.  Faster where the levels are short (many
//                       pairs per velocity node: 2383 levels against 1981
//                       steps for 20 000 pairs on 20^3), slower where long
//                       chains span groups (6144 pairs on 20^3: 370 against
//                       206).
//   seq_collide_kernel  one workgroup per cell, the cell's h in LDS (FP32,
//                       4 B per node, five cells per CU on a 20^3 grid):
//                       moments of h^s, the steps in order (one wavefront),
//                       then the conservation correction (S5) and the store.
#pragma once

namespace boltz {

constexpr int kSeqGroup = 1024;  // records per level group (one workgroup of the level kernel)
constexpr int kSeqAhead = 8;     // steps of records loaded ahead of the one applied
constexpr int kSeqBlock = 256;   // threads per cell: the node phases use all, the pair loop one wavefront
constexpr int kSeqGroup64 = 64;  // records per level group of the in-register schedule
constexpr int kSeqAhead64 = 4;   // groups of records loaded ahead in that schedule

// Dynamic LDS of seq_collide_kernel: the h tile (FP32), one spare word per
// lane, then the per-axis parts of x . psi of the correction (FP64); the
// block reductions (at most 20 doubles per wavefront) use the region after
// the tile before x . psi is written.
struct SeqLDS {
  static constexpr size_t kSpare = 64 * 4;
  static __host__ __device__ size_t tile(int nv) { return ((size_t)nv * 4 + 15) & ~(size_t)15; }
  static __host__ __device__ size_t bytes(int nv, int ns) {
    const size_t tail = kSpare + (size_t)ns * 8, red = (size_t)20 * (kSeqBlock / 64) * 8;
    return tile(nv) + (tail > red ? tail : red);
  }
};

// The schedule of the records of every sample group (table), ngr = ceil(N_t
// / kSeqGroup) level groups per table: a step is up to 64 records of one
// level of one group, contiguous in the table once seq_level_kernel has
// sorted each group by level.
//   gstep[tab][g][s]  offset within the group | count << 16, s < gcount
//   gcount[tab][g]    steps of group g
//   step[tab][t]      first record (index into the table) and count of
//                     step t of the table, t < total[tab]
struct SeqSched {
  uint32_t* gstep;
  int* gcount;
  uint2* step;
  int* total;
  static __host__ __device__ size_t bytes(int64_t ngr, int64_t ntab) {
    const int64_t slots = ngr * kSeqGroup * ntab;
    return (size_t)slots * 4 + (size_t)(ngr * ntab) * 4 + (size_t)slots * 8 + (size_t)ntab * 4 + 64;
  }
  static __host__ __device__ SeqSched carve(unsigned char* base, int64_t ngr, int64_t ntab) {
    const int64_t slots = ngr * kSeqGroup * ntab;
    SeqSched S;
    S.step = reinterpret_cast<uint2*>(base);
    S.gstep = reinterpret_cast<uint32_t*>(base + (size_t)slots * 8);
    S.gcount = reinterpret_cast<int*>(base + (size_t)slots * 12);
    S.total = reinterpret_cast<int*>(base + (size_t)slots * 12 + (size_t)(ngr * ntab) * 4);
    return S;
  }
};

// The groups schedule.  Grid: (ceil(N_t / 64), sample groups); 64 threads.  A record's nodes are
// a = id.x & 0xFFFF, b = id.x >> 16, a* = id.y & 0xFFFF, b* = id.y >> 16 and
// its coefficients {q/w_a*, q/w_b*, q/w_a, q/w_b} (all zero: a discarded
// pair, which takes level 0 and changes nothing).  Writes lev[m] = level
// (0..64) | (the group's largest level << 8) and the merged signed
// coefficients over tcoef.
__global__ __launch_bounds__(64) void seq_level64_kernel(const uint2* __restrict__ tidx, float4* __restrict__ tcoef,
                                                       int64_t nt, uint16_t* __restrict__ lev) {
  const int lane = threadIdx.x;
  const int64_t tab = blockIdx.y;
  const int64_t m = (int64_t)blockIdx.x * kSeqGroup64 + lane;
  const bool in = m < nt;
  uint2 id = make_uint2(0u, 0u);
  float4 k = make_float4(0.f, 0.f, 0.f, 0.f);
  if (in) {
    id = tidx[tab * nt + m];
    k = tcoef[tab * nt + m];
  }
  const bool act = in && (k.x != 0.f || k.y != 0.f || k.z != 0.f || k.w != 0.f);
  // slots in coefficient order: a*, b*, a, b
  const unsigned n0 = id.y & 0xFFFFu, n1 = id.y >> 16, n2 = id.x & 0xFFFFu, n3 = id.x >> 16;
  // records of lower lanes sharing a node: bit (lane - d) for distance d
  unsigned long long conf = 0ull;
  for (int d = 1; d < kSeqGroup64; ++d) {
    const unsigned ox = (unsigned)__shfl_up((int)id.x, d, 64), oy = (unsigned)__shfl_up((int)id.y, d, 64);
    const int oact = __shfl_up(act ? 1 : 0, d, 64);
    const unsigned o0 = oy & 0xFFFFu, o1 = oy >> 16, o2 = ox & 0xFFFFu, o3 = ox >> 16;
    const bool hit = n0 == o0 || n0 == o1 || n0 == o2 || n0 == o3 || n1 == o0 || n1 == o1 || n1 == o2 ||
                     n1 == o3 || n2 == o0 || n2 == o1 || n2 == o2 || n2 == o3 || n3 == o0 || n3 == o1 ||
                     n3 == o2 || n3 == o3;
    if (lane >= d && act && oact && hit) conf |= 1ull << (lane - d);
  }
  // levels in lane order: lane j's level is final once the lanes below it
  // have been taken into account
  int level = act ? 1 : 0;
  for (int j = 0; j < kSeqGroup64 - 1; ++j) {
    const int lj = __builtin_amdgcn_readlane(level, j);
    if ((conf >> j) & 1ull) level = max(level, lj + 1);
  }
  int top = level;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) top = max(top, __shfl_xor(top, off, 64));
  if (in) {
    lev[tab * nt + m] = (uint16_t)(level | (top << 8));
    // every slot carries the signed sum over the slots of its node, summed
    // in slot order (equal for all slots of one node)
    const float s[4] = {k.x, k.y, -k.z, -k.w};
    const unsigned nn[4] = {n0, n1, n2, n3};
    float c[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      float v = 0.0f;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (nn[u] == nn[t]) v += s[u];
      c[t] = v;
    }
    tcoef[tab * nt + m] = make_float4(c[0], c[1], c[2], c[3]);
  }
}

// The steps schedule.  Grid: (ceil(N_t / 1024), sample groups); 1024
// threads, one record each.
// A record's nodes are a = id.x & 0xFFFF, b = id.x >> 16, a* = id.y & 0xFFFF,
// b* = id.y >> 16 and its coefficients {q/w_a*, q/w_b*, q/w_a, q/w_b} (all
// zero: a discarded pair, which changes nothing and is left out).
//   1. The 4096 (node, record, slot) keys of the group are sorted (bitonic
//      sort in LDS); a record's predecessor at one of its nodes is the
//      latest earlier record of the group with that node.
//   2. Levels: 1 + the largest level of the record's predecessors, relaxed
//      in place until nothing changes (values only grow, so the fixed point
//      is the longest chain).  Records of one level share no node.
//   3. The group's records are rewritten in level order (positions within a
//      level are arbitrary: they commute), with the four coefficients of a
//      record merged where its nodes coincide (each slot then carries the
//      signed sum over the slots of its node: gain at a*, b*, loss at a, b);
//      each level is cut into steps of up to 64 records.
// Applying the groups in order, the steps of a group in order, gives every
// node its updates in record order: the result of the sequential loop.
__global__ __launch_bounds__(kSeqGroup) void seq_level_kernel(uint2* __restrict__ tidx, float4* __restrict__ tcoef,
                                                              int64_t nt, SeqSched S) {
  __shared__ uint32_t key[4 * kSeqGroup];
  __shared__ uint16_t pred[4 * kSeqGroup];
  __shared__ int lvl[kSeqGroup + 1];
  __shared__ int hist[kSeqGroup + 1];
  __shared__ int nstep[kSeqGroup + 1];
  const int t = threadIdx.x;
  const int64_t ngr = (nt + kSeqGroup - 1) / kSeqGroup;
  const int64_t tab = blockIdx.y, g = blockIdx.x;
  const int64_t m = g * kSeqGroup + t;
  const bool in = m < nt;
  uint2 id = make_uint2(0u, 0u);
  float4 k = make_float4(0.f, 0.f, 0.f, 0.f);
  if (in) {
    id = tidx[tab * nt + m];
    k = tcoef[tab * nt + m];
  }
  const bool act = in && (k.x != 0.f || k.y != 0.f || k.z != 0.f || k.w != 0.f);
  // slots in coefficient order: a*, b*, a, b
  const unsigned nn[4] = {id.y & 0xFFFFu, id.y >> 16, id.x & 0xFFFFu, id.x >> 16};
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    key[4 * t + s] = act ? ((nn[s] << 12) | ((unsigned)t << 2) | (unsigned)s) : 0xFFFFFFFFu;
    pred[4 * t + s] = 0xFFFFu;
  }
  lvl[t] = act ? 1 : 0;
  hist[t] = 0;
  if (t == 0) hist[kSeqGroup] = 0;
  __syncthreads();
  // ---- 1. bitonic sort of the 4096 keys, ascending
  for (int kk = 2; kk <= 4 * kSeqGroup; kk <<= 1) {
    for (int j = kk >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int p = t + e * kSeqGroup, q = p ^ j;
        if (q > p) {
          const uint32_t x = key[p], y = key[q];
          const bool up = (p & kk) == 0;
          if ((x > y) == up) {
            key[p] = y;
            key[q] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  // the element before the first key of (node, record) holds, if its node
  // is the same, the latest earlier record with that node
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int p = 4 * t + e;
    const uint32_t x = key[p];
    if (x != 0xFFFFFFFFu && p > 0) {
      int q = p - 1;
      // skip the other slots of the same record at the same node
      while (q >= 0 && (key[q] >> 2) == (x >> 2)) --q;
      if (q >= 0 && (key[q] >> 12) == (x >> 12)) pred[((x >> 2) & 0x3FFu) * 4 + (x & 3u)] = (uint16_t)((key[q] >> 2) & 0x3FFu);
    }
  }
  __syncthreads();
  // ---- 2. levels by relaxation
  bool more = true;
  while (more) {
    bool changed = false;
    if (act) {
      int L = lvl[t];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const unsigned p = pred[4 * t + s];
        if (p != 0xFFFFu) L = max(L, lvl[p] + 1);
      }
      if (L != lvl[t]) {
        lvl[t] = L;
        changed = true;
      }
    }
    more = __syncthreads_or(changed);
  }
  // ---- 3. level histogram, positions, steps
  const int L = lvl[t];
  if (act) atomicAdd(&hist[L], 1);
  __syncthreads();
  // exclusive prefix of the counts (record offsets) and of the steps per
  // level, over levels 1 .. kSeqGroup (one per thread, Hillis-Steele)
  {
    const int c = t + 1 <= kSeqGroup ? hist[t + 1] : 0;
    int off = c, ns = (c + 63) / 64;
    nstep[t] = ns;
    lvl[t] = off;  // reuse: inclusive counts
    __syncthreads();
    for (int d = 1; d < kSeqGroup; d <<= 1) {
      int a = 0, b = 0;
      if (t >= d) {
        a = lvl[t - d];
        b = nstep[t - d];
      }
      __syncthreads();
      off += a;
      ns += b;
      lvl[t] = off;
      nstep[t] = ns;
      __syncthreads();
    }
    // thread t describes level t + 1: records [off - c, off), steps
    // [ns - ceil(c / 64), ns)
    const int r0 = off - c, s0 = ns - (c + 63) / 64;
    uint32_t* gs = S.gstep + (tab * ngr + g) * kSeqGroup;
    for (int q = 0; 64 * q < c; ++q) gs[s0 + q] = (uint32_t)(r0 + 64 * q) | ((uint32_t)min(64, c - 64 * q) << 16);
    if (t == kSeqGroup - 1) S.gcount[tab * ngr + g] = ns;
    __syncthreads();
    // record offsets of each level: reuse hist as a cursor
    hist[t + 1 <= kSeqGroup ? t + 1 : 0] = r0;
  }
  __syncthreads();
  if (act) {
    const int pos = atomicAdd(&hist[L], 1);
    const float sv[4] = {k.x, k.y, -k.z, -k.w};
    float c[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      float v = 0.0f;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (nn[u] == nn[s]) v += sv[u];
      c[s] = v;
    }
    // in place: every thread of the group has read its record above
    tidx[tab * nt + g * kSeqGroup + pos] = id;
    tcoef[tab * nt + g * kSeqGroup + pos] = make_float4(c[0], c[1], c[2], c[3]);
  }
}

// Grid: sample groups; 1024 threads.  The steps of all level groups of a
// table in one list (first record as an index into the table, count).
__global__ __launch_bounds__(kSeqGroup) void seq_steps_kernel(int64_t nt, SeqSched S) {
  const int64_t ngr = (nt + kSeqGroup - 1) / kSeqGroup;
  const int64_t tab = blockIdx.x;
  int64_t base = 0;
  for (int64_t g = 0; g < ngr; ++g) {
    const int n = S.gcount[tab * ngr + g];
    const uint32_t* gs = S.gstep + (tab * ngr + g) * kSeqGroup;
    for (int s = threadIdx.x; s < n; s += blockDim.x) {
      const uint32_t d = gs[s];
      S.step[tab * ngr * kSeqGroup + base + s] = make_uint2((uint32_t)(g * kSeqGroup) + (d & 0xFFFFu), d >> 16);
    }
    base += n;
  }
  if (threadIdx.x == 0) S.total[tab] = (int)base;
}

// Sums over the cell of w_j psi_k(j) h_j, psi = (1, v_x, v_y, v_z, |v|^2),
// by velocity rows (jx, jy): per row the z sums with the factors
// omega_z v_z^p (four z nodes per scalar load batch), then the row weight
// omega_x omega_y.  Block-reduced over kSeqBlock threads (red: 5 * kSeqBlock
// / 64 doubles of LDS; ends with a barrier); h in LDS.
__device__ __forceinline__ void seq_moments(const double* vx, const double* vy, const double* omx,
                                            const double* omy, const double* zmom, const float* h, int n0, int n1,
                                            int n2, double* red, double (&s)[5]) {
  typedef __attribute__((address_space(4))) const double cf64;
  const cf64* zc = (const cf64*)zmom;
#pragma unroll
  for (int i = 0; i < 5; ++i) s[i] = 0.0;
  for (int row = threadIdx.x; row < n0 * n1; row += kSeqBlock) {
    const int jx = row / n1, jy = row - (row / n1) * n1;
    double S0 = 0.0, S1 = 0.0, S2 = 0.0;
    int jz = 0;
    for (; jz + 4 <= n2; jz += 4) {
      double z[4][3];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int p = 0; p < 3; ++p) z[k][p] = zc[8 * (jz + k) + p];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double v = (double)h[row * n2 + jz + k];
        S0 = fma(z[k][0], v, S0);
        S1 = fma(z[k][1], v, S1);
        S2 = fma(z[k][2], v, S2);
      }
    }
    for (; jz < n2; ++jz) {
      const double v = (double)h[row * n2 + jz];
      S0 = fma(zc[8 * jz], v, S0);
      S1 = fma(zc[8 * jz + 1], v, S1);
      S2 = fma(zc[8 * jz + 2], v, S2);
    }
    const double W = omx[jx] * omy[jy], a = vx[jx], b = vy[jy];
    const double T0 = W * S0;
    s[0] += T0;
    s[1] += a * T0;
    s[2] += b * T0;
    s[3] += W * S1;
    s[4] += (a * a + b * b) * T0 + W * S2;
  }
  block_sum<5, kSeqBlock>(s, red);
}

// Grid: one workgroup of kSeqBlock threads per cell.  vom: node velocities
// of the three axes, then their weights omega (n0 + n1 + n2 each, FP64).
// Records of the cell's sample group as left by seq_level_kernel (SCHED 1,
// schedule S) or seq_level64_kernel (SCHED 0, levels lev).  The node
// phases use the whole workgroup; the pair loop, a chain of dependent LDS
// accesses, runs on wavefront 0 while the others wait at a barrier.
template <int SCHED>
__global__ __launch_bounds__(kSeqBlock, 5) void seq_collide_kernel(
    Params P, const double* __restrict__ vom, const float* __restrict__ hs_all, float* __restrict__ hout_all,
    uint32_t flags, double* __restrict__ defect, const uint2* __restrict__ tidx, const float4* __restrict__ tcoef,
    SeqSched S, const uint16_t* __restrict__ lev) {
  extern __shared__ __align__(16) unsigned char dsm[];
  const int tid = threadIdx.x, lane = tid & 63;
  const int nv = P.nv, n0 = P.n[0], n1 = P.n[1], n2 = P.n[2], ns = n0 + n1 + n2;
  const int64_t cell = blockIdx.x;
  float* tile = reinterpret_cast<float*>(dsm);
  // after the tile: one spare word per lane (the accesses of the lanes
  // without a record in a level), then x . psi per axis; the block sums use
  // the same region before x . psi is written
  double* red = reinterpret_cast<double*>(dsm + SeqLDS::tile(nv));
  double* xt = reinterpret_cast<double*>(dsm + SeqLDS::tile(nv) + SeqLDS::kSpare);
  const float* hs = hs_all + cell * (int64_t)nv;
  float* dst = hout_all + cell * (int64_t)nv;
  const double* vx = vom;
  const double* vy = vom + n0;
  const double* vz = vom + n0 + n1;
  const double* omx = vom + ns;
  const double* omy = vom + ns + n0;
  const double* omz = vom + ns + n0 + n1;
  const double eps = P.eps;
  const bool vec4 = ((nv & 3) == 0) && ((reinterpret_cast<uintptr_t>(hs) & 15) == 0) &&
                    ((reinterpret_cast<uintptr_t>(dst) & 15) == 0);
  // ---- h^s into LDS (read once), and its moments: the targets of S5
  if (vec4) {
    const f32x4* s4 = reinterpret_cast<const f32x4*>(hs);
    f32x4* t4 = reinterpret_cast<f32x4*>(tile);
    for (int i = tid; i < (nv >> 2); i += kSeqBlock) t4[i] = __builtin_nontemporal_load(&s4[i]);
  } else {
    for (int j = tid; j < nv; j += kSeqBlock) tile[j] = hs[j];
  }
  __syncthreads();
  double ms[5];
  seq_moments(vx, vy, omx, omy, P.zmom, tile, n0, n1, n2, red, ms);
  // ---- S3 + S4: the records in order, one level of a group at a time
  if (SCHED == 0 && tid < 64) {
    const int64_t nt = P.n_pairs, ngr = (nt + kSeqGroup64 - 1) / kSeqGroup64;
    const int64_t tab = P.sample_group == 0 ? 0 : cell / P.sample_group;
    const uint2* T = tidx + tab * nt;
    const float4* C = tcoef + tab * nt;
    const uint16_t* L = lev + tab * nt;
    const float epsf = (float)eps;
    const int spare = (int)(SeqLDS::tile(nv) / 4) + lane;
    // the records of the next kSeqAhead64 groups are in flight in registers
    // (a group's levels take less time than a load from L2).  The loads are
    // unconditional (indices clamped into the table) and their values are
    // not touched before the group is applied, so each group waits only
    // for its own records.
    uint2 qid[kSeqAhead64];
    float4 qco[kSeqAhead64];
    unsigned qlt[kSeqAhead64];
    bool qok[kSeqAhead64];
    auto fetch = [&](int64_t g, int s) {
      const int64_t gc = g < ngr ? g : ngr - 1;
      const int64_t m = gc * kSeqGroup64 + lane;
      const int64_t mc = m < nt ? m : nt - 1;
      qid[s] = T[mc];
      qco[s] = C[mc];
      qlt[s] = L[mc];
      qok[s] = m < nt;
    };
    if (ngr > 0) {
#pragma unroll
      for (int s = 0; s < kSeqAhead64; ++s) fetch(s, s);
    }
    for (int64_t g0 = 0; g0 < ngr; g0 += kSeqAhead64) {
#pragma unroll
      for (int s = 0; s < kSeqAhead64; ++s) {
        const int64_t g = g0 + s;
        const uint2 id = qid[s];
        const float4 co = qco[s];
        const unsigned lt = qlt[s];
        const bool ok = qok[s];
        fetch(g + kSeqAhead64, s);
        if (g < ngr) {
          // level of the lane's record and the group's last level (lane 0
          // always holds a record of the group)
          const int lv = ok ? (int)(lt & 0xFFu) : 0;
          const int top = __builtin_amdgcn_readfirstlane((int)(lt >> 8));
          const int ia = (int)(id.x & 0xFFFFu), ib = (int)(id.x >> 16);
          const int ias = (int)(id.y & 0xFFFFu), ibs = (int)(id.y >> 16);
          for (int k = 1; k <= top; ++k) {
            // every lane reads and writes four words; a lane whose record
            // is not of this level uses its spare word for all four
            const bool on = lv == k;
            const int pa = on ? ia : spare, pb = on ? ib : spare;
            const int pas = on ? ias : spare, pbs = on ? ibs : spare;
            // the four current values, then the four new ones: slots of one
            // node read the same value and carry the same merged coefficient
            const float va = tile[pa], vb = tile[pb], vas = tile[pas], vbs = tile[pbs];
            const float gg = (va + vb) + (epsf * va) * vb;
            tile[pas] = fmaf(co.x, gg, vas);
            tile[pbs] = fmaf(co.y, gg, vbs);
            tile[pa] = fmaf(co.z, gg, va);
            tile[pb] = fmaf(co.w, gg, vb);
          }
        }
      }
    }
  }
  // ---- S3 + S4: the steps of the cell's table in order (up to 64
  // records of one level each, contiguous in the table)
  if (SCHED == 1 && tid < 64) {
    const int64_t nt = P.n_pairs, ngr = (nt + kSeqGroup - 1) / kSeqGroup;
    const int64_t tab = P.sample_group == 0 ? 0 : cell / P.sample_group;
    const uint2* T = tidx + tab * nt;
    const float4* C = tcoef + tab * nt;
    const uint2* ST = S.step + tab * ngr * kSeqGroup;
    const int nsteps = ngr > 0 ? __builtin_amdgcn_readfirstlane(S.total[tab]) : 0;
    const float epsf = (float)eps;
    const int spare = (int)(SeqLDS::tile(nv) / 4) + lane;
    // The records of the next kSeqAhead steps and the descriptors of the
    // kSeqAhead steps after those are in flight in registers, one slot per
    // step of the unrolled loop: a step's slot is applied, then refilled
    // with the records of the step kSeqAhead later (whose descriptor
    // arrived kSeqAhead steps ago) and the descriptor kSeqAhead beyond.
    // The loads are unconditional (indices clamped into the tables), so
    // each step waits only for its own loads.
    // descriptors through the scalar path (uniform addresses, read-only)
    typedef __attribute__((address_space(4))) const unsigned cu32;
    const cu32* STc = (const cu32*)ST;
    auto dload = [&](int st) {
      const int i = min(st, max(nsteps - 1, 0));
      return make_uint2(STc[2 * i], STc[2 * i + 1]);
    };
    uint2 qid[kSeqAhead], qd[kSeqAhead];
    float4 qco[kSeqAhead];
    bool qok[kSeqAhead];
    auto fetch = [&](uint2 d, int st, int sl) {
      const uint32_t start = d.x;
      const int cnt = (int)d.y;
      const bool ok = st < nsteps && lane < cnt;
      const int64_t mrec = (int64_t)start + (ok ? lane : 0);
      qid[sl] = T[mrec];
      qco[sl] = C[mrec];
      qok[sl] = ok;
    };
    if (nsteps > 0) {
#pragma unroll
      for (int sl = 0; sl < kSeqAhead; ++sl) fetch(dload(sl), sl, sl);
#pragma unroll
      for (int sl = 0; sl < kSeqAhead; ++sl) qd[sl] = dload(sl + kSeqAhead);
    }
    for (int st0 = 0; st0 < nsteps; st0 += kSeqAhead) {
#pragma unroll
      for (int sl = 0; sl < kSeqAhead; ++sl) {
        const int st = st0 + sl;
        if (st < nsteps) {
          // every lane reads and writes four words; a lane without a record
          // in this step uses its spare word for all four
          const uint2 id = qid[sl];
          const float4 co = qco[sl];
          const bool on = qok[sl];
          const int pa = on ? (int)(id.x & 0xFFFFu) : spare, pb = on ? (int)(id.x >> 16) : spare;
          const int pas = on ? (int)(id.y & 0xFFFFu) : spare, pbs = on ? (int)(id.y >> 16) : spare;
          // the four current values, then the four new ones: slots of one
          // node read the same value and carry the same merged coefficient
          const float va = tile[pa], vb = tile[pb], vas = tile[pas], vbs = tile[pbs];
          const float gg = (va + vb) + (epsf * va) * vb;
          tile[pas] = fmaf(co.x, gg, vas);
          tile[pbs] = fmaf(co.y, gg, vbs);
          tile[pa] = fmaf(co.z, gg, va);
          tile[pb] = fmaf(co.w, gg, vb);
        }
        fetch(qd[sl], st + kSeqAhead, sl);
        qd[sl] = dload(st + 2 * kSeqAhead);
      }
    }
  }
  __syncthreads();
  // ---- S5: M x = r with M_kl = sum w F^c psi_k psi_l and r = eps (moments
  // of h^s - moments of h^c), the moments of h^c being row 0 of the sums
  const bool correct = !(flags & 1u);
  if (correct) {
    TablesLDS Tb;
    Tb.v = const_cast<double*>(vom);
    Tb.om = const_cast<double*>(vom + ns);
    Tb.xt = xt;
    double acc[20];
    correction_sums<kSeqBlock>(Tb, P.zmom, tile, tile, n0, n1, n2, acc);
    const int rows = n0 * n1;
    const double t = block_sum20_w0<kSeqBlock>(acc, red, rows >= kSeqBlock ? kSeqBlock / 64 : (rows + 63) / 64);
    if (tid < 64) {
      // wavefront 0: thread k < 20 holds total k; it has read red before
      // x . psi overwrites the region
      const const_f64* m0c = (const const_f64*)P.m0;
      double M[15], r[5], x[5];
#pragma unroll
      for (int k = 0; k < 15; ++k) M[k] = m0c[k] + eps * lane_value(t, k);
#pragma unroll
      for (int k = 0; k < 5; ++k) r[k] = eps * (ms[k] - lane_value(t, k));
      if (!solve5(M, r, x)) {
#pragma unroll
        for (int k = 0; k < 5; ++k) x[k] = 0.0;
        if (tid == 0) atomicOr(P.status, 1u);
      }
      for (int i = tid; i < ns; i += 64) {
        const double v = vom[i];
        xt[i] = i < n0 ? x[1] * v + x[4] * (v * v)
                       : (i < n0 + n1 ? x[2] * v + x[4] * (v * v) : x[0] + x[3] * v + x[4] * (v * v));
      }
    }
    __syncthreads();
  }
  // ---- h^{n+1} = h^c + F^c (x . psi) / eps; moments of the output for the
  // defect
  bool finite = true;
  auto out_of = [&](double hc, double xpsi) { return (float)fma(fma(eps, hc, 1.0) * xpsi, P.inv_eps, hc); };
  if (vec4 && !defect) {
    const f32x4* a4 = reinterpret_cast<const f32x4*>(tile);
    f32x4* d4 = reinterpret_cast<f32x4*>(dst);
    NodeWalk nw4(4 * tid, 4 * kSeqBlock, n1, n2);
    for (int i = tid; i < (nv >> 2); i += kSeqBlock, nw4.next()) {
      const f32x4 c = a4[i];
      f32x4 o = c;
      if (correct) {
        const double xa = xt[nw4.jx] + xt[n0 + nw4.jy];
        const double* xz = xt + n0 + n1 + nw4.jz;
        o.x = out_of((double)c.x, xa + xz[0]);
        o.y = out_of((double)c.y, xa + xz[1]);
        o.z = out_of((double)c.z, xa + xz[2]);
        o.w = out_of((double)c.w, xa + xz[3]);
      }
      finite = finite && isfinite(o.x) && isfinite(o.y) && isfinite(o.z) && isfinite(o.w);
      __builtin_nontemporal_store(o, &d4[i]);
    }
  } else {
    NodeWalk nw1(tid, kSeqBlock, n1, n2);
    for (int j = tid; j < nv; j += kSeqBlock, nw1.next()) {
      const double hc = (double)tile[j];
      float out = (float)hc;
      if (correct) out = out_of(hc, (xt[nw1.jx] + xt[n0 + nw1.jy]) + xt[n0 + n1 + nw1.jz]);
      finite = finite && isfinite(out);
      dst[j] = out;
      tile[j] = out;
    }
    if (defect) {
      // the output's moments against those of h^s, times eps (red is free:
      // x . psi has been used)
      __syncthreads();
      double mo[5];
      seq_moments(vx, vy, omx, omy, P.zmom, tile, n0, n1, n2, red, mo);
      if (tid < 5) {
        double d = 0.0;
#pragma unroll
        for (int k = 0; k < 5; ++k)
          if (tid == k) d = eps * (mo[k] - ms[k]);
        defect[cell * 5 + tid] = d;
      }
    }
  }
  (void)vz;
  (void)omz;
  if (!finite) atomicOr(P.status, 2u);
}

}  // namespace boltz
