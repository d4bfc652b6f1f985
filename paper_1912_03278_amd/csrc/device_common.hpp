// Device-side building blocks shared by the lattice and dense HMC kernels.
//
//  * Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11),
//    53-bit uniforms and FP64 Box-Muller: the momentum distribution of Sec. 3,
//    eq. momentum distribution.
//  * Exact fixed-point accumulation of FP64 terms in 128-bit two's complement
//    (unit 2^-64).  Integer addition is associative, so every reduction order,
//    atomics included, gives the same bits: the Hamiltonian of Sec. 3 and the
//    estimator sums of Sec. 4 are independent of tiling, batching and launch
//    shape.
//  * tanh in the state precision and FP64 log cosh / tanh for the action.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ihmc_internal.hpp"

namespace ihmc {

// ---------------------------------------------------------------- Philox ---

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

__device__ __forceinline__ double unit53(uint32_t a, uint32_t b) {
  const uint64_t k = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
  return ((double)k + 0.5) * 0x1p-53;
}

__device__ __forceinline__ uint4 draw(const ChainDev& cd, uint32_t i, uint32_t traj, uint32_t tag) {
  return philox4x32_10(make_uint4(i, traj, cd.chain_id, tag), cd.seed_lo, cd.seed_hi);
}

// Standard normal for `site`: pair site/2 gives (r cos th, r sin th) to sites 2i, 2i+1.
__device__ __forceinline__ double normal_at(const ChainDev& cd, uint32_t traj, uint32_t tag, int64_t site) {
  const uint4 w = draw(cd, (uint32_t)(site >> 1), traj, tag);
  const double u1 = unit53(w.x, w.y), u2 = unit53(w.z, w.w);
  const double r = sqrt(-2.0 * log(u1));
  const double th = 6.283185307179586 * u2;
  return (site & 1) ? r * sin(th) : r * cos(th);
}

// Both normals of pair i.  FP64 state: FP64 Box-Muller (matches an FP64
// reference to a few ulp).  FP32 state: the same 53-bit uniforms, Box-Muller
// in FP32 with the hardware log2 / sin / cos (absolute error ~1e-6).
template <typename T>
__device__ __forceinline__ void normal_pair(const ChainDev& cd, uint32_t traj, uint32_t tag, int64_t pair,
                                            T& z0, T& z1);
template <>
__device__ __forceinline__ void normal_pair<double>(const ChainDev& cd, uint32_t traj, uint32_t tag,
                                                    int64_t pair, double& z0, double& z1) {
  const uint4 w = draw(cd, (uint32_t)pair, traj, tag);
  const double u1 = unit53(w.x, w.y), u2 = unit53(w.z, w.w);
  const double r = sqrt(-2.0 * log(u1));
  const double th = 6.283185307179586 * u2;
  z0 = r * cos(th);
  z1 = r * sin(th);
}
template <>
__device__ __forceinline__ void normal_pair<float>(const ChainDev& cd, uint32_t traj, uint32_t tag,
                                                   int64_t pair, float& z0, float& z1) {
  const uint4 w = draw(cd, (uint32_t)pair, traj, tag);
  const float u1 = (float)unit53(w.x, w.y);
  const float u2 = (float)unit53(w.z, w.w);
  // -2 ln u1 = -2 ln2 log2(u1); the hardware sine/cosine take revolutions,
  // so sin(2 pi u2) needs no range reduction for u2 in (0, 1)
  const float r = __builtin_sqrtf(-1.38629436111989061f * __builtin_amdgcn_logf(u1));
  z0 = r * __builtin_amdgcn_cosf(u2);
  z1 = r * __builtin_amdgcn_sinf(u2);
}

__device__ __forceinline__ double uniform_at(const ChainDev& cd, uint32_t traj, uint32_t tag) {
  const uint4 w = draw(cd, 0u, traj, tag);
  return unit53(w.x, w.y);
}

// ----------------------------------------------------- exact fixed point ---

struct u128 {
  uint64_t lo, hi;
};

__host__ __device__ __forceinline__ u128 add128(u128 a, u128 b) {
  u128 r;
  r.lo = a.lo + b.lo;
  r.hi = a.hi + b.hi + (r.lo < a.lo ? 1ull : 0ull);
  return r;
}

__host__ __device__ __forceinline__ u128 neg128(u128 a) {
  u128 r;
  r.lo = ~a.lo + 1ull;
  r.hi = ~a.hi + (r.lo == 0ull ? 1ull : 0ull);
  return r;
}

__host__ __device__ __forceinline__ u128 sub128(u128 a, u128 b) { return add128(a, neg128(b)); }


// round(x * 2^64) (ties away from zero) as a signed 128-bit integer, from the
// bit pattern: |x| = m 2^e with a 53-bit integer m, so |x| 2^64 = m 2^(e+64)
// is m shifted left or right.  |x| < 2^28 keeps any sum of up to 2^34 terms
// inside the 128-bit range; larger or non-finite terms set `bad`.
__device__ __forceinline__ u128 to_fixed(double x, uint32_t& bad) {
  // branch-free: every case is computed and selected, so the conversions of a
  // wave never split into divergent paths
  const uint64_t bits = (uint64_t)__double_as_longlong(x);
  const int ex = (int)((bits >> 52) & 0x7ffu);
  const bool too_big = (ex >= 1023 + 28);  // |x| >= 2^28, inf or nan
  bad |= too_big ? 1u : 0u;
  const uint64_t m = (ex == 0 || too_big) ? 0ull : ((bits & 0x000fffffffffffffull) | 0x0010000000000000ull);
  const int sh = ex - 1011;  // |x| 2^64 = m 2^sh, sh <= 39
  const int k = -sh;
  const uint64_t left_lo = m << (sh & 63);
  const uint64_t left_hi = m >> ((64 - sh) & 63);
  const uint64_t rnd = 1ull << ((k - 1) & 63);
  const uint64_t right = (m + rnd) >> (k & 63);
  u128 r;
  r.lo = (sh >= 0) ? left_lo : ((k < 64) ? right : 0ull);
  r.hi = (sh > 0) ? left_hi : 0ull;
  const u128 n = neg128(r);
  const bool neg = (bits >> 63) != 0ull;
  r.lo = neg ? n.lo : r.lo;
  r.hi = neg ? n.hi : r.hi;
  return r;
}

__host__ __device__ __forceinline__ double fixed_to_double(u128 v) {
  const bool neg = (int64_t)v.hi < 0;
  if (neg) v = neg128(v);
  const double m = (double)v.hi + (double)v.lo * 0x1p-64;
  return neg ? -m : m;
}

__device__ __forceinline__ u128 wave_sum128(u128 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    u128 o;
    o.lo = __shfl_xor(v.lo, off, 64);
    o.hi = __shfl_xor(v.hi, off, 64);
    v = add128(v, o);
  }
  return v;
}

// Workgroup barrier that orders LDS accesses only.  The full __syncthreads
// fence also waits for every global load in flight, which would expose the
// latency of loads issued early to overlap work across the barrier.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ------------------------------------------------------------- functions ---

// tanh in FP32: tanh|x| = 1 - 2 / (1 + e^{2|x|}) with the hardware base-2
// exponential and reciprocal, extended as an odd function.  Absolute error
// about 1e-7, ample against the FP32 state.
__device__ __forceinline__ float tanh_state(float x) {
  const float ax = fabsf(x);
  const float e = __builtin_amdgcn_exp2f(ax * 2.88539008177792681f);
  const float t = fmaf(-2.0f, __builtin_amdgcn_rcpf(1.0f + e), 1.0f);
  return copysignf(t, x);
}

__device__ __forceinline__ double tanh_state(double x) { return tanh(x); }

// log cosh(y) = |y| + log1p(e) - ln 2 and tanh(y) = sign(y) (1 - e)/(1 + e)
// with e = exp(-2|y|) in [0, 1], in FP64:
//   exp: Cody-Waite reduction x = k ln2 + r, |r| <= ln2/2, Taylor polynomial of
//        degree 13 (truncation < 5e-18), then 2^k;
//   log1p(e) = 2 atanh(s), s = e/(2+e) (e <= sqrt2 - 1) or
//        ln 2 + 2 atanh((e-1)/(e+3)) (e > sqrt2 - 1), so |s| <= 0.1716 and the
//        odd series to s^23 is below 1e-18 relative.
// Agrees with correctly rounded log cosh / tanh to a few ulp.
__device__ __forceinline__ double exp_nonpos(double x) {
  const bool under = (x < -745.0);
  x = under ? 0.0 : x;
  const double k = rint(x * 1.4426950408889634);
  double r = __builtin_fma(-k, 6.93147180369123816490e-01, x);
  r = __builtin_fma(-k, 1.90821492927058770002e-10, r);
  double p = 1.6059043836821614e-10;  // 1/13!
  p = __builtin_fma(p, r, 2.0876756987868099e-09);
  p = __builtin_fma(p, r, 2.5052108385441720e-08);
  p = __builtin_fma(p, r, 2.7557319223985893e-07);
  p = __builtin_fma(p, r, 2.7557319223985888e-06);
  p = __builtin_fma(p, r, 2.4801587301587302e-05);
  p = __builtin_fma(p, r, 1.9841269841269841e-04);
  p = __builtin_fma(p, r, 1.3888888888888889e-03);
  p = __builtin_fma(p, r, 8.3333333333333332e-03);
  p = __builtin_fma(p, r, 4.1666666666666664e-02);
  p = __builtin_fma(p, r, 1.6666666666666666e-01);
  p = __builtin_fma(p, r, 0.5);
  p = __builtin_fma(p, r, 1.0);
  p = __builtin_fma(p, r, 1.0);
  return under ? 0.0 : ldexp(p, (int)k);
}

__device__ __forceinline__ double log1p_unit(double e) {
  const bool hi = (e > 0.41421356237309503);
  const double s = (hi ? e - 1.0 : e) / (hi ? e + 3.0 : 2.0 + e);
  const double off = hi ? 0.6931471805599453 : 0.0;
  const double z = s * s;
  double q = 1.0 / 23.0;
  q = __builtin_fma(q, z, 1.0 / 21.0);
  q = __builtin_fma(q, z, 1.0 / 19.0);
  q = __builtin_fma(q, z, 1.0 / 17.0);
  q = __builtin_fma(q, z, 1.0 / 15.0);
  q = __builtin_fma(q, z, 1.0 / 13.0);
  q = __builtin_fma(q, z, 1.0 / 11.0);
  q = __builtin_fma(q, z, 1.0 / 9.0);
  q = __builtin_fma(q, z, 1.0 / 7.0);
  q = __builtin_fma(q, z, 1.0 / 5.0);
  q = __builtin_fma(q, z, 1.0 / 3.0);
  q = q * z;  // atanh(s)/s - 1
  return off + 2.0 * __builtin_fma(s, q, s);
}

__device__ __forceinline__ void logcosh_tanh(double y, double& lc, double& t) {
  const double a = fabs(y);
  const double e = exp_nonpos(-2.0 * a);
  lc = (a - 0.6931471805599453) + log1p_unit(e);
  t = copysign((1.0 - e) / (1.0 + e), y);
}

template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c);
template <>
__device__ __forceinline__ float fma_t<float>(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}
template <>
__device__ __forceinline__ double fma_t<double>(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}

}  // namespace ihmc
