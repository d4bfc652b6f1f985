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
    // each 32 x 32 -> 64-bit product in one multiply (both halves)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
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

// ln 2 as head + tail: the head is ln 2 with its low 21 significand bits
// cleared, so e * head is exact for |e| < 2^21; the tail is the rounded rest.
constexpr double kLn2Head = 6.93147180369123816490e-01;
constexpr double kLn2Tail = 1.90821492927058770002e-10;

// ln u for u in (0, 1) (a 53-bit uniform): u = m 2^e with m in [sqrt(1/2),
// sqrt 2), ln u = e ln 2 + 2 atanh(s), s = (m - 1)/(m + 1), |s| <= 0.1716, with
// the odd Taylor series of atanh to s^23 (truncation below 1e-19 relative).
__device__ __forceinline__ double ln_unit(double u) {
  int e;
  double m = frexp(u, &e);  // u = m 2^e, m in [1/2, 1)
  const bool lo = m < 0.70710678118654752;
  m = lo ? 2.0 * m : m;
  e = lo ? e - 1 : e;
  const double s = (m - 1.0) / (m + 1.0);
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
  const double ls = 2.0 * __builtin_fma(s, q, s);
  const double de = (double)e;
  return __builtin_fma(de, kLn2Head, __builtin_fma(de, kLn2Tail, ls));
}

// sin and cos of the angle 2 pi u, u in [0, 1] (a fraction of a turn): u is
// reduced exactly to t = u - k/4, k = round(4u), |t| <= 1/8 turn; x = 2 pi t
// (|x| <= pi/4, one rounding) goes into the Taylor series of sin (to x^17) and
// cos (to x^18), truncation below 1e-19; quarter turn k mod 4 rotates the pair.
__device__ __forceinline__ void sincos_turn(double u, double& sn, double& cs) {
  const double k = rint(4.0 * u);
  const double t = __builtin_fma(k, -0.25, u);  // exact
  const double x = 6.283185307179586 * t;
  const double z = x * x;
  // sin x = x + x z P(z), cos x = 1 + z Q(z), z = x^2, coefficients +-1/n!
  double ps = 1.0 / 355687428096000.0;
  ps = __builtin_fma(ps, z, -1.0 / 1307674368000.0);
  ps = __builtin_fma(ps, z, 1.0 / 6227020800.0);
  ps = __builtin_fma(ps, z, -1.0 / 39916800.0);
  ps = __builtin_fma(ps, z, 1.0 / 362880.0);
  ps = __builtin_fma(ps, z, -1.0 / 5040.0);
  ps = __builtin_fma(ps, z, 1.0 / 120.0);
  ps = __builtin_fma(ps, z, -1.0 / 6.0);
  const double sx = __builtin_fma(x * z, ps, x);
  double pc = -1.0 / 6402373705728000.0;
  pc = __builtin_fma(pc, z, 1.0 / 20922789888000.0);
  pc = __builtin_fma(pc, z, -1.0 / 87178291200.0);
  pc = __builtin_fma(pc, z, 1.0 / 479001600.0);
  pc = __builtin_fma(pc, z, -1.0 / 3628800.0);
  pc = __builtin_fma(pc, z, 1.0 / 40320.0);
  pc = __builtin_fma(pc, z, -1.0 / 720.0);
  pc = __builtin_fma(pc, z, 1.0 / 24.0);
  pc = __builtin_fma(pc, z, -0.5);
  const double cx = __builtin_fma(pc, z, 1.0);
  const int q = (int)k & 3;
  const double s0 = (q & 1) ? cx : sx, c0 = (q & 1) ? sx : cx;
  sn = (q & 2) ? -s0 : s0;
  cs = ((q + 1) & 2) ? -c0 : c0;
}

// Box-Muller in FP64 on a Philox output: two 53-bit uniforms u1, u2 give
// r cos(2 pi u2) and r sin(2 pi u2), r = sqrt(-2 ln u1).
__device__ __forceinline__ void box_muller(uint4 w, double& z0, double& z1) {
  const double u1 = unit53(w.x, w.y), u2 = unit53(w.z, w.w);
  const double r = sqrt(-2.0 * ln_unit(u1));
  double sn, cs;
  sincos_turn(u2, sn, cs);
  z0 = r * cs;
  z1 = r * sn;
}

// Standard normal for `site`: pair site/2 gives (r cos th, r sin th) to sites 2i, 2i+1.
__device__ __forceinline__ double normal_at(const ChainDev& cd, uint32_t traj, uint32_t tag, int64_t site) {
  double z0, z1;
  box_muller(draw(cd, (uint32_t)(site >> 1), traj, tag), z0, z1);
  return (site & 1) ? z1 : z0;
}

// Both normals of pair i, Box-Muller in FP64.  An FP32 state takes these FP64
// normals rounded to nearest, so its momenta are the FP64 normals to within
// one rounding (FP64 values of another log / sin / cos implementation lie a
// few ulp away, which changes the FP32 rounding only when a value sits that
// close to a rounding boundary).
template <typename T>
__device__ __forceinline__ void normal_pair(const ChainDev& cd, uint32_t traj, uint32_t tag, int64_t pair,
                                            T& z0, T& z1) {
  double a, b;
  box_muller(draw(cd, (uint32_t)pair, traj, tag), a, b);
  z0 = (T)a;
  z1 = (T)b;
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

// round(x 2^64) (ties away from zero, as to_fixed) for any |x| < 2^62, the
// range of the 128-bit sums; false (and zero) for larger or non-finite x.  For
// single values of any size, such as the action change of the sign flip.
__host__ __device__ inline bool to_fixed_wide(double x, u128& out) {
  const uint64_t bits = __builtin_bit_cast(uint64_t, x);
  const int ex = (int)((bits >> 52) & 0x7ffu);
  out = u128{0ull, 0ull};
  if (ex >= 1023 + 62) return false;  // |x| >= 2^62, inf or nan
  if (ex == 0) return true;                   // zero or subnormal: rounds to 0
  const uint64_t m = (bits & 0x000fffffffffffffull) | 0x0010000000000000ull;
  const int sh = ex - 1011;  // |x| 2^64 = m 2^sh, sh <= 73
  u128 r{0ull, 0ull};
  if (sh >= 64) {
    r.hi = m << (sh - 64);
  } else if (sh > 0) {
    r.lo = m << sh;
    r.hi = m >> (64 - sh);
  } else if (sh == 0) {
    r.lo = m;
  } else if (sh > -64) {
    const int k = -sh;
    r.lo = (m + (1ull << (k - 1))) >> k;
  }
  out = ((bits >> 63) != 0ull) ? neg128(r) : r;
  return true;
}

__host__ __device__ __forceinline__ double fixed_to_double(u128 v) {
  const bool neg = (int64_t)v.hi < 0;
  if (neg) v = neg128(v);
  const double m = (double)v.hi + (double)v.lo * 0x1p-64;
  return neg ? -m : m;
}

// Cross-lane moves within rows of 16 lanes by DPP (a modifier of a VALU
// operation: no LDS round trip, unlike a shuffle).  CTRL is the DPP control
// word; every source lane named below lies in the destination's row.
constexpr int DPP_QUAD_XOR1 = 0xB1;         // quad_perm [1,0,3,2]: lane l ^ 1
constexpr int DPP_QUAD_XOR2 = 0x4E;         // quad_perm [2,3,0,1]: lane l ^ 2
constexpr int DPP_ROW_MIRROR = 0x140;       // lane 15 - l of the row
constexpr int DPP_ROW_HALF_MIRROR = 0x141;  // lane 7 - l of the half-row
constexpr int DPP_ROW_ROR4 = 0x124;         // lane l - 4 of the row, rotating
constexpr int DPP_ROW_ROR8 = 0x128;         // lane l - 8 of the row, rotating

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
  return (uint64_t)dpp_u32<CTRL>((uint32_t)v) | ((uint64_t)dpp_u32<CTRL>((uint32_t)(v >> 32)) << 32);
}
template <int CTRL>
__device__ __forceinline__ u128 dpp_u128(u128 v) {
  return u128{dpp_u64<CTRL>(v.lo), dpp_u64<CTRL>(v.hi)};
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  return __longlong_as_double((long long)dpp_u64<CTRL>((uint64_t)__double_as_longlong(v)));
}
__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
  return (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l) |
         ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l) << 32);
}

// Sum over the 64 lanes of the wave, the same value in every lane; the whole
// wave must be active.  Within each row by DPP (quads, half-rows, rows), then
// the four row sums read out.  Integer sums: the order does not matter.
__device__ __forceinline__ u128 wave_sum128(u128 v) {
  v = add128(v, dpp_u128<DPP_QUAD_XOR1>(v));
  v = add128(v, dpp_u128<DPP_QUAD_XOR2>(v));
  v = add128(v, dpp_u128<DPP_ROW_HALF_MIRROR>(v));
  v = add128(v, dpp_u128<DPP_ROW_MIRROR>(v));  // every lane holds its row's sum
  u128 r[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) r[q] = u128{readlane_u64(v.lo, 16 * q), readlane_u64(v.hi, 16 * q)};
  return add128(add128(r[0], r[1]), add128(r[2], r[3]));
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
  double r = __builtin_fma(-k, kLn2Head, x);
  r = __builtin_fma(-k, kLn2Tail, r);
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

// Both quotients, s = num/den of the log1p series and (1 - e)/(1 + e), come
// from the one reciprocal q = 1/((1 + e) den): s = num (1 + e) q and
// 1/(1 + e) = den q (a few ulp each, instead of two divisions).
__device__ __forceinline__ void logcosh_tanh(double y, double& lc, double& t) {
  const double a = fabs(y);
  const double e = exp_nonpos(-2.0 * a);
  const bool hi = (e > 0.41421356237309503);
  const double num = hi ? e - 1.0 : e;
  const double den = hi ? e + 3.0 : 2.0 + e;
  const double g = 1.0 + e;
  const double q = 1.0 / (g * den);
  const double s = (num * g) * q;
  const double z = s * s;
  double p = 1.0 / 23.0;
  p = __builtin_fma(p, z, 1.0 / 21.0);
  p = __builtin_fma(p, z, 1.0 / 19.0);
  p = __builtin_fma(p, z, 1.0 / 17.0);
  p = __builtin_fma(p, z, 1.0 / 15.0);
  p = __builtin_fma(p, z, 1.0 / 13.0);
  p = __builtin_fma(p, z, 1.0 / 11.0);
  p = __builtin_fma(p, z, 1.0 / 9.0);
  p = __builtin_fma(p, z, 1.0 / 7.0);
  p = __builtin_fma(p, z, 1.0 / 5.0);
  p = __builtin_fma(p, z, 1.0 / 3.0);
  p = p * z;  // atanh(s)/s - 1
  const double l1p = (hi ? 0.6931471805599453 : 0.0) + 2.0 * __builtin_fma(s, p, s);
  lc = (a - 0.6931471805599453) + l1p;
  t = copysign((1.0 - e) * (den * q), y);
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
