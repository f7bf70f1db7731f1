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

// -ln u for u in (0, 1] (the radii of the Box-Muller pairs): u = 2^e m with
// m in [sqrt(1/2), sqrt(2)) taken from the bits, ln m = ln(1 + t), t = m - 1
// (exact), by its alternating series to 40 terms (|t|^40 / 40 < 2e-17) in
// Horner form from the last term, with coefficients folded at compile time;
// IEEE adds and multiplies only, so the host reproduces every bit.
__device__ __forceinline__ double neg_ln_unit(double u) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(u);
  int e = (int)((bits >> 52) & 0x7FFull) - 1023;
  double m = __longlong_as_double((long long)((bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
  if (m > 1.4142135623730951) {
    m = m * 0.5;
    e += 1;
  }
  const double t = m - 1.0;
  double p = 0.0;
#pragma unroll
  for (int n = 40; n >= 1; --n) p = ((n & 1) ? 1.0 : -1.0) / (double)n + t * p;
  return -((double)e * 0.6931471805599453094172321 + t * p);
}

// A 16-byte store that does not keep its line in L2 (outputs read by the
// next launch only): the halo rows and shared tables that are read again
// stay cached.
__device__ __forceinline__ void nt_store4(float* p, float4 v) {
  typedef float f4v __attribute__((ext_vector_type(4)));
  __builtin_nontemporal_store(f4v{v.x, v.y, v.z, v.w}, reinterpret_cast<f4v*>(p));
}

// ------------------------------------------------ fixed-point LDS sums --
// Increments of h are accumulated as signed 64-bit integers in units of
// 2^-32 with the integer LDS atomic add, which on gfx950 runs an order of
// magnitude faster than any float accumulation in LDS and is associative,
// so the sums do not depend on the order of the lanes.  A value c with
// |c| < 2^18 is rounded to the 2^-32 grid by adding 1.5 * 2^20 (whose FP64
// ulp is 2^-32, round to nearest even); the difference of the two bit
// patterns is then round(c 2^32) (the low word of 1.5 * 2^20 is zero).  Larger contributions (deviations in the
// far tail of the velocity grid, where Phi0 is tiny and |h| can grow by many
// orders of magnitude) and non-finite ones go to an FP32 accumulator
// instead, so no value is clipped.
constexpr double kFixMagic = 1572864.0;               // 1.5 * 2^20
constexpr double kFixLimit = 262144.0;                // 2^18
constexpr double kFixScale = 2.3283064365386963e-10;  // 2^-32

// Value of a 64-bit fixed-point sum: hi + lo 2^-32 of its signed high and
// unsigned low words with the single rounding of the FMA, which is the
// correctly rounded (double)(int64) v times 2^-32.
__device__ __forceinline__ double from_fixed(unsigned long long v) {
  return fma((double)(unsigned)v, kFixScale, (double)(int)(v >> 32));
}

// ------------------------------------------------------- LDS float add --
// Float accumulation into LDS as a read plus a 32-bit compare-and-swap,
// retried when another lane changed the word.  On gfx950 the native LDS
// float atomic add completes about one lane every three clocks per CU
// whatever the address pattern, while integer LDS atomics run ~28x faster;
// the compare-and-swap form keeps exact FP32 addition semantics.  Used when
// the 64-bit accumulators of a large velocity grid do not fit in LDS.
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

// FP64 accumulation into LDS as a read plus a 64-bit compare-and-swap (the
// adjoint sums, whose scale is not known in advance).
__device__ __forceinline__ void lds_add_f64(double* p, double v) {
  unsigned long long* u = reinterpret_cast<unsigned long long*>(p);
  unsigned long long old = *u;
  while (true) {
    const unsigned long long nw = (unsigned long long)__double_as_longlong(__longlong_as_double((long long)old) + v);
    const unsigned long long prev = atomicCAS(u, old, nw);
    if (prev == old) break;
    old = prev;
  }
}

// One contribution k g to node j: 64-bit fixed point when |k g| < 2^18,
// else the FP32 accumulator ovf[j].  fma(k, g, 1.5 * 2^20) rounds the exact
// product once onto the 2^-32 grid; the high word of the bit difference
// then lies in [-2^18, 2^18) exactly for the values kept in fixed point
// (the bit patterns of positive doubles are ordered like their values;
// negative, infinite and NaN sums fall outside that window).
__device__ __forceinline__ void lds_add_hybrid(unsigned long long* acc, float* ovf, int j, double k, double g) {
  const long long d = __double_as_longlong(fma(k, g, kFixMagic)) - __double_as_longlong(kFixMagic);
  const int hi = (int)(d >> 32);
  if ((unsigned)(hi + (1 << 18)) < (1u << 19)) {
    __hip_atomic_fetch_add(&acc[j], (unsigned long long)d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  } else {
    lds_add(&ovf[j], (float)(k * g));
  }
}

// Fixed-point value of k g (units of 2^-32, see lds_add_hybrid) and whether it
// lies in the fixed-point window.
__device__ __forceinline__ long long fixed_of(double k, double g) {
  return __double_as_longlong(fma(k, g, kFixMagic)) - __double_as_longlong(kFixMagic);
}

__device__ __forceinline__ bool in_fixed_window(long long d) {
  return (unsigned)((int)(d >> 32) + (1 << 18)) < (1u << 19);
}

// A contribution whose fixed-point value d was computed by fixed_of: the
// 64-bit accumulator when d is in the window, else the FP32 array.
__device__ __forceinline__ void lds_add_fixed_or(unsigned long long* acc, float* ovf, int j, long long d, double k,
                                                 double g) {
  if (in_fixed_window(d)) {
    __hip_atomic_fetch_add(&acc[j], (unsigned long long)d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  } else {
    lds_add(&ovf[j], (float)(k * g));
  }
}

// round(x 2^32) as a 64-bit two's complement integer for |x| < 2^26, the
// range the magic-number form (|x| < 2^18) does not reach: t = rint(x 2^32)
// is an integer below 2^58, its high word floor(t 2^-32) and low word
// t - 2^32 floor(t 2^-32) are exact in FP64.  false (nothing written) beyond
// that range or for a non-finite x.
constexpr double kFixWide = 67108864.0;  // 2^26
__device__ __forceinline__ bool fixed_exact(double x, unsigned long long& v) {
  if (!(fabs(x) < kFixWide)) return false;
  const double t = rint(x * 4294967296.0);
  const double hi = floor(t * kFixScale);
  const double lo = fma(-hi, 4294967296.0, t);
  v = ((unsigned long long)(unsigned)(int)hi << 32) | (unsigned long long)(unsigned)lo;
  return true;
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
// 64; BLOCK, when given, is blockDim.x known at compile time); every thread
// receives the totals.  red: LDS scratch of N * (blockDim.x / 64) doubles.
// Deterministic order.
template <int N, int BLOCK = 0>
__device__ __forceinline__ void block_sum(double (&v)[N], double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = BLOCK ? BLOCK / 64 : (int)(blockDim.x >> 6);
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
#pragma unroll 2
    for (int w = 0; w < nw; ++w) s += red[i * nw + w];
    v[i] = s;
  }
  __syncthreads();
}

// ----------------------------------------- 20-value block reduction --
// Lane exchanges of gfx950 without the LDS: v_permlane32_swap and
// v_permlane16_swap (swap two registers' halves between lanes l and l ^ 32,
// resp. l ^ 16), and DPP reads of lane l ^ 15 (row_mirror), l ^ 7
// (row_half_mirror), l ^ 2 and l ^ 1 (quad permutations).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
constexpr int kDppMirror = 0x140, kDppHalfMirror = 0x141, kDppXor2 = 0x4E, kDppXor1 = 0xB1;

// Halving step with a lane swap: lanes with (lane & OFF) == 0 end with
// lo + partner's lo, the others with hi + partner's hi (OFF = 32 or 16).
template <int OFF>
__device__ __forceinline__ double swap_sum(double lo, double hi) {
  const unsigned a0 = (unsigned)__double2loint(lo), a1 = (unsigned)__double2hiint(lo);
  const unsigned b0 = (unsigned)__double2loint(hi), b1 = (unsigned)__double2hiint(hi);
  if (OFF == 32) {
    const auto l = __builtin_amdgcn_permlane32_swap(a0, b0, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(a1, b1, false, false);
    return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
  } else {
    const auto l = __builtin_amdgcn_permlane16_swap(a0, b0, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(a1, b1, false, false);
    return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
  }
}

// Halving step of a multi-value wavefront reduction: v[0..N) becomes
// v[0..H), H = (N + 1) / 2; lanes without bit OFF keep the sums of the lower
// half (v[i] + partner's v[i]), the others those of the upper half
// (v[H + i], zero-padded when N is odd).  The partner differs in bit OFF
// (and in lower bits only, for the DPP partners).
template <int N, int OFF, int CTRL>
__device__ __forceinline__ void fold_half(double* v, int lane) {
  constexpr int H = (N + 1) / 2;
  const bool upper = lane & OFF;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const double lo = v[i];
    const double hi = (H + i < N) ? v[H + i] : 0.0;
    if (OFF >= 16) {
      v[i] = swap_sum<OFF>(lo, hi);
    } else {
      const double send = upper ? lo : hi;
      const double keep = upper ? hi : lo;
      v[i] = keep + dpp_f64<CTRL>(send);
    }
  }
}

// Sum of 20 values per thread over a block of BLOCK threads (a multiple of
// 64).  Within a wavefront the values are halved at every exchange (lane
// bits 5, 4, 3, 2, 1, then a plain pairwise sum), 22 exchanges instead of
// 120; lane l then holds value 10 b5 + 5 b4 + 3 b3 + 2 b2 + b1 of its bits
// b_k (or a zero pad).  The wavefront sums are added in wavefront order;
// on return lane k < 20 of wavefront 0 holds total k (the value returned;
// other lanes: unspecified).  Deterministic order.  Only the first nwd
// wavefronts take part (the values of the others must be zero).  red: LDS
// scratch of 20 * (BLOCK / 64) doubles.  v is consumed.  Ends without a
// barrier after the reads of red: the caller synchronises before red is
// written again.
// The wavefront part: returns, in lane 32 b5 + 16 b4 + 8 b3 + 4 b2 + 2 b1
// with k = 10 b5 + 5 b4 + 3 b3 + 2 b2 + b1 (b3 = 1 only with b2 = 0), the
// wavefront's sum of value k (other lanes: partial sums or pads).  v is
// consumed.
__device__ __forceinline__ double wave_fold20(double (&v)[20], int lane) {
  fold_half<20, 32, 0>(v, lane);
  fold_half<10, 16, 0>(v, lane);
  fold_half<5, 8, kDppMirror>(v, lane);
  fold_half<3, 4, kDppHalfMirror>(v, lane);
  fold_half<2, 2, kDppXor2>(v, lane);
  return v[0] + dpp_f64<kDppXor1>(v[0]);
}

template <int BLOCK>
__device__ __forceinline__ double block_sum20_w0(double (&v)[20], double* red, int nwd = BLOCK / 64) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = BLOCK / 64;
  if (wid < nwd) {
    const double s = wave_fold20(v, lane);
    const int b5 = (lane >> 5) & 1, b4 = (lane >> 4) & 1, b3 = (lane >> 3) & 1, b2 = (lane >> 2) & 1,
              b1 = (lane >> 1) & 1;
    // positions within the last group of five: b3 b2 b1 -> 0,1,2,pad,3,4,pad,pad
    const int pos = 3 * b3 + 2 * b2 + b1;
    const bool valid = ((lane & 1) == 0) && (b3 ? (b2 == 0) : (pos < 3));
    if (valid) red[(10 * b5 + 5 * b4 + pos) * nw + wid] = s;
  }
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x < 20) {
#pragma unroll 4
    for (int w = 0; w < nwd; ++w) t += red[threadIdx.x * nw + w];
  }
  return t;
}

// Value of lane k of a wavefront (k uniform), in every lane.
__device__ __forceinline__ double lane_value(double t, int k) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(t), k),
                          __builtin_amdgcn_readlane(__double2loint(t), k));
}

// block_sum20_w0 with the totals stored to tot[0..20) in LDS for the whole
// block (ends with a barrier).
template <int BLOCK>
__device__ __forceinline__ void block_sum20_lds(double (&v)[20], double* red, double* tot) {
  const double t = block_sum20_w0<BLOCK>(v, red);
  if (threadIdx.x < 20) tot[threadIdx.x] = t;
  __syncthreads();
}

}  // namespace boltz
