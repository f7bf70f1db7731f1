// device_math.hpp -- device-side building blocks shared by the kernels of
// libboltz: the counter-based generator, the direction map, the node-law
// lookup, the Beam-Warming update and FP64 wavefront reductions.
//
// Everything that decides an integer (a node index) is evaluated in FP64 with
// the compiler's floating-point contraction disabled (-ffp-contract=off), so
// the result depends only on IEEE-rounded add/mul/div/sqrt and is reproducible
// bit for bit by any other IEEE implementation of the same formulas.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace boltz {

constexpr int kMaxAxis = 255;          // velocity cells per axis
constexpr int kFieldBits = 12;         // bits of a Philox word selecting one node index
constexpr int kFieldSize = 1 << kFieldBits;
constexpr double kPiOver4 = 0.78539816339744830961566084581988;

// ---------------------------------------------------------------- Philox --
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 products; the key advances by the Weyl constants between rounds.
struct u32x4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
    u32x4 n;
    n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
    n.y = (uint32_t)p1;
    n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
    n.w = (uint32_t)p0;
    c = n;
  }
  return c;
}

// ------------------------------------------------------- direction map --
// (cos 2 pi u, sin 2 pi u) for u in (0,1): exact octant reduction of 8u, fold
// to z in [0, pi/4], Taylor polynomials in z^2 of degree 13 (sin) and 12
// (cos) evaluated in a fixed order (truncation below 4e-13).
__device__ __forceinline__ void cos_sin_2pi(double u, double& cs, double& sn) {
  const double t = u * 8.0;
  const double o = floor(t);
  const double f = t - o;
  const int oct = ((int)o) & 7;
  const double z = ((oct & 1) ? (1.0 - f) : f) * kPiOver4;
  const double z2 = z * z;
  double ps = 1.0 / 6227020800.0;
  ps = -1.0 / 39916800.0 + z2 * ps;
  ps = 1.0 / 362880.0 + z2 * ps;
  ps = -1.0 / 5040.0 + z2 * ps;
  ps = 1.0 / 120.0 + z2 * ps;
  ps = -1.0 / 6.0 + z2 * ps;
  ps = 1.0 + z2 * ps;
  const double S = z * ps;
  double pc = 1.0 / 479001600.0;
  pc = -1.0 / 3628800.0 + z2 * pc;
  pc = 1.0 / 40320.0 + z2 * pc;
  pc = -1.0 / 720.0 + z2 * pc;
  pc = 1.0 / 24.0 + z2 * pc;
  pc = -1.0 / 2.0 + z2 * pc;
  const double C = 1.0 + z2 * pc;
  // octant o covers [o pi/4, (o+1) pi/4)
  const double c0 = (oct == 0 || oct == 7) ? C : (oct == 3 || oct == 4) ? -C : (oct == 1 || oct == 6) ? S : -S;
  const double s0 = (oct == 1 || oct == 2) ? C : (oct == 5 || oct == 6) ? -C : (oct == 0 || oct == 3) ? S : -S;
  cs = c0;
  sn = s0;
}

// ------------------------------------------------------------ node law --
// A node index comes from a 12-bit field f of a Philox word: the Maxwellian
// law is a direct inverse-CDF table icdf[f] = #{i >= 1 : T_i <= f}; the
// uniform law is floor(f n / 2^12) (a 24-bit product).
__device__ __forceinline__ int uniform_draw(uint32_t f, int n) {
  return (int)((f * (uint32_t)n) >> kFieldBits);
}

// ------------------------------------------------------------ streaming --
// Second-order upwind (Beam-Warming) update along one axis:
//   h0 - C (h0 - h1) - C (1 - C)/2 ((h0 - 2 h1) + h2),  h1, h2 = one and two
// cells upwind; c2 = C (1 - C)/2.  A uniform state is reproduced exactly.
__device__ __forceinline__ float bw_update(float h0, float h1, float h2, float C, float c2) {
  return h0 - C * (h0 - h1) - c2 * ((h0 - 2.0f * h1) + h2);
}

// ------------------------------------------------------- LDS float add --
// Float accumulation into LDS as a read plus a 32-bit compare-and-swap,
// retried when another lane changed the word.  On gfx950 the native LDS
// float atomic add completes about one lane every three clocks per CU
// whatever the address pattern, while integer LDS atomics run ~28x faster;
// the compare-and-swap form keeps exact FP32 addition semantics.
__device__ __forceinline__ void lds_add(float* p, float v) {
  unsigned* u = reinterpret_cast<unsigned*>(p);
  unsigned old = *u;
  while (true) {
    const unsigned nw = __float_as_uint(__uint_as_float(old) + v);
    const unsigned prev = atomicCAS(u, old, nw);
    if (prev == old) break;
    old = prev;
  }
}

// Per-thread walk over j = j0, j0 + step, ... of the velocity index with the
// components (jx, jy, jz) updated by carries instead of integer divisions
// (step < n1 * n2 * n0 arbitrary; each carry is at most one).
struct NodeWalk {
  int jx, jy, jz, dx, dy, dz, n1, n2;
  __device__ NodeWalk(int j0, int step, int n1_, int n2_) : n1(n1_), n2(n2_) {
    jz = j0 % n2;
    jy = (j0 / n2) % n1;
    jx = j0 / (n2 * n1);
    dz = step % n2;
    dy = (step / n2) % n1;
    dx = step / (n2 * n1);
  }
  __device__ __forceinline__ void next() {
    jz += dz;
    int cy = 0;
    if (jz >= n2) { jz -= n2; cy = 1; }
    jy += dy + cy;
    int cx = 0;
    if (jy >= n1) { jy -= n1; cx = 1; }
    jx += dx + cx;
  }
};

// ---------------------------------------------------------- reductions --
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of N values per thread over the whole block (blockDim.x a multiple of
// 64); every thread receives the totals.  red: LDS scratch of
// N * (blockDim.x / 64) doubles.  Deterministic order.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) red[i * nw + wid] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[i * nw + w];
    v[i] = s;
  }
  __syncthreads();
}

}  // namespace boltz
