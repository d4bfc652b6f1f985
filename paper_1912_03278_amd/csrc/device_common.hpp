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
// in FP32 (sqrt(-2 log u1) and sincospi(2 u2)), accurate to about 2 FP32 ulp.
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
  const float r = sqrtf(-2.0f * logf(u1));
  float sn, cs;
  sincospif(2.0f * u2, &sn, &cs);
  z0 = r * cs;
  z1 = r * sn;
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

// Magnitude limit of one term; larger or non-finite terms set `bad`.
constexpr double kFixedLimit = 268435456.0;  // 2^28

// round(x * 2^64) as a signed 128-bit integer.  |x| < 2^28: the integer part
// goes to `hi`, the fraction times 2^64 (exact: a power-of-two scaling of an
// exactly computed fraction) to `lo`.
__device__ __forceinline__ u128 to_fixed(double x, uint32_t& bad) {
  const double ax = fabs(x);
  if (!(ax < kFixedLimit)) {
    bad = 1u;
    return u128{0ull, 0ull};
  }
  const double ip = floor(ax);
  const double fr = (ax - ip) * 18446744073709551616.0;
  u128 r;
  r.hi = (uint64_t)ip;
  r.lo = (uint64_t)rint(fr);
  return x < 0.0 ? neg128(r) : r;
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

// Order-independent 128-bit atomic accumulation from two 64-bit atomics: the
// number of carries out of the low word equals floor(sum of low words / 2^64)
// whatever the order, so the high word ends up exact.
// Both RMWs return, so the caller can wait for them to be performed before it
// publishes completion (see publish_done).
__device__ __forceinline__ void atomic_add128(uint64_t* slot, u128 v) {
  const uint64_t old = __hip_atomic_fetch_add(&slot[0], v.lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint64_t carry = (old + v.lo < old) ? 1ull : 0ull;
  (void)__hip_atomic_fetch_add(&slot[1], v.hi + carry, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store128_agent(uint64_t* slot, u128 v) {
  __hip_atomic_store(&slot[0], v.lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&slot[1], v.hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Count one finished block of a chain and tell whether it was the last one.
// The accumulators are only ever touched by device-scope atomics, so ordering
// needs no cache write-back: the caller's atomics are made to complete
// (workgroup-scope release = wait for this wave's outstanding memory
// operations) before the counter increments.
__device__ __forceinline__ bool publish_done(uint32_t* done, uint32_t n_blocks) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  const uint32_t prev = __hip_atomic_fetch_add(done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return prev == n_blocks - 1u;
}

__device__ __forceinline__ u128 load128_agent(const uint64_t* slot) {
  u128 r;
  r.lo = __hip_atomic_load(&slot[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  r.hi = __hip_atomic_load(&slot[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return r;
}

// ------------------------------------------------------------- functions ---

// tanh in FP32: tanh|x| = 1 - 2 / (1 + e^{2|x|}) with the hardware base-2
// exponential and reciprocal, extended as an odd function.  Absolute error
// about 1e-7, ample against the FP32 state.
__device__ __forceinline__ float tanh_state(float x) {
  const float ax = fabsf(x);
  const float e = __builtin_amdgcn_exp2f(ax * 2.88539008177792681f);
  const float t = 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + e);
  return copysignf(t, x);
}

__device__ __forceinline__ double tanh_state(double x) { return tanh(x); }

// log cosh(y) = |y| + log1p(e^{-2|y|}) - ln 2 and tanh(y), sharing one exponential.
__device__ __forceinline__ void logcosh_tanh(double y, double& lc, double& t) {
  const double a = fabs(y);
  const double e = exp(-2.0 * a);
  lc = a + log1p(e) - 0.6931471805599453;
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
