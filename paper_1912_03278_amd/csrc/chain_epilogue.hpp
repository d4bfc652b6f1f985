// Trajectory epilogue shared by the lattice kernels: block reduction of the
// exact fixed-point sums, accumulation into the chain, and the work of the
// block that finishes last -- the Metropolis test of Sec. 3 on
// dH = H_new - H_old in FP64 (exact integer difference of the fixed-point
// Hamiltonians), the optional global sign flip, and the Sec. 4 estimators.
#pragma once

#include "device_common.hpp"
#include "lattice_kernels.hpp"

namespace ihmc {

// Metropolis decision and record, run by one thread of the last block of a LAST
// pass once the block has gathered the chain's accumulators (`sum`, `bad`).
__device__ __forceinline__ void finalize_trajectory(const ChainDev& cd, ChainState* st, int last_buf,
                                                    const u128* sum, uint32_t bad) {
  const int t = st->traj;
  const u128 S_old{st->S_lo, st->S_hi};
  const u128 H_old = add128(sum[T_K0], S_old);
  const u128 H_new = add128(sum[T_K1], sum[T_S]);
  double dH = fixed_to_double(sub128(H_new, H_old));
  uint32_t flags = 0u;
  bool finite = (bad == 0u);
  if (!finite) {
    dH = __builtin_nan("");
    flags |= REC_NONFINITE;
    st->n_nonfinite += 1;
  }
  if (finite && st->cur_bad) dH = -__builtin_inf();  // leaving a state of zero weight
  bool accept;
  if (cd.replay && t < cd.cap) {
    accept = cd.replay[t] != 0;
  } else {
    const double r = uniform_at(cd, (uint32_t)t, TAG_ACC);
    accept = finite && (dH <= 0.0 || r < exp(-dH));
  }
  if (finite && !st->cur_bad) st->sum_exp_mdh += exp(-dH);
  if (accept) {
    st->cur_bad = 0;
    st->S_lo = sum[T_S].lo;
    st->S_hi = sum[T_S].hi;
    st->sum_psi = fixed_to_double(sum[T_PSI]);
    st->sum_psih = fixed_to_double(sum[T_PSIH]);
    st->sum_ut = fixed_to_double(sum[T_UT]);
    st->cur = last_buf;
    st->sign = 1;
    st->n_acc += 1;
    flags |= REC_ACCEPT;
  }
  if (cd.flip_every > 0 && (t + 1) % cd.flip_every == 0) {
    // S(-psi) - S(psi) = 2 psi.h'/sqrt(J'): only the linear field term changes.
    const double dS = 2.0 * st->sum_psih / cd.sqJ;
    const double r2 = uniform_at(cd, (uint32_t)t, TAG_FLIP);
    if (dS <= 0.0 || r2 < exp(-dS)) {
      uint32_t b2 = 0u;
      const u128 S = add128(u128{st->S_lo, st->S_hi}, to_fixed(dS, b2));
      st->S_lo = S.lo;
      st->S_hi = S.hi;
      st->sign = -st->sign;
      st->sum_psi = -st->sum_psi;
      st->sum_psih = -st->sum_psih;
      flags |= REC_FLIP;
    }
  }
  if (t < cd.cap) {
    const double N = (double)cd.N;
    TrajRecord rec;
    rec.dH = dH;
    rec.H_old = fixed_to_double(H_old);
    rec.H_new = fixed_to_double(H_new);
    rec.m = (st->sum_psi / cd.sqJ - cd.c_m / cd.Jp) / N;
    rec.abs_m = fabs(rec.m);
    rec.m2c = rec.m * rec.m - cd.c_v / (N * N * cd.Jp);
    rec.beta_eps = 0.5 * cd.C * cd.Jp + cd.c_e / (2.0 * N * cd.Jp) - st->sum_psih / (2.0 * N * cd.sqJ) -
                   cd.sqJ / (2.0 * N) * st->sum_ut;
    rec.flags = flags;
    rec.pad = 0u;
    cd.rec[t] = rec;
  }
  st->traj = t + 1;
  __hip_atomic_store(&st->bad, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&st->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void finalize_measure(ChainState* st, const u128* sum, uint32_t bad) {
  st->cur_bad = bad ? 1 : 0;
  st->S_lo = sum[T_S].lo;
  st->S_hi = sum[T_S].hi;
  st->sum_psi = fixed_to_double(sum[T_PSI]);
  st->sum_psih = fixed_to_double(sum[T_PSIH]);
  st->sum_ut = fixed_to_double(sum[T_UT]);
  __hip_atomic_store(&st->bad, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&st->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Last-block epilogue shared by every kernel that closes a trajectory or a
// measurement: gather the NTERM x NSLOT accumulators with one load per thread,
// clear them for the next trajectory, and let thread 0 finish.
template <bool kTraj>
__device__ __forceinline__ void close_chain(const ChainDev& cd, ChainState* st, int last_buf) {
  __shared__ u128 sAcc[NTERM][NSLOT];
  __shared__ uint32_t sBad;
  for (int k = threadIdx.x; k < NTERM * NSLOT; k += blockDim.x) {
    const int a = k / NSLOT, sl = k % NSLOT;
    sAcc[a][sl] = load_limbs_agent(st->acc[a][sl]);
  }
  if (threadIdx.x == 0) sBad = __hip_atomic_load(&st->bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  for (int k = threadIdx.x; k < NTERM * NSLOT; k += blockDim.x) {
    const int a = k / NSLOT, sl = k % NSLOT;
    clear_limbs_agent(st->acc[a][sl]);
  }
  if (threadIdx.x == 0) {
    u128 sum[NTERM];
#pragma unroll
    for (int a = 0; a < NTERM; ++a) {
      sum[a] = u128{0ull, 0ull};
#pragma unroll 1
      for (int sl = 0; sl < NSLOT; ++sl) sum[a] = add128(sum[a], sAcc[a][sl]);
    }
    if (kTraj) finalize_trajectory(cd, st, last_buf, sum, sBad);
    else finalize_measure(st, sum, sBad);
  }
}

// Block reduction of the per-thread fixed-point sums, order-independent
// accumulation into the chain, and the last block's epilogue.  NW = waves per
// block; `slot` spreads blocks over the NSLOT atomic slots of every term.
template <int MODE, int NW>
__device__ __forceinline__ void block_accumulate(const ChainDev& cd, ChainState* st, const u128* acc,
                                                 uint32_t bad, int cur, int j, int slot) {
  __shared__ u128 sRed[NW][NTERM];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int t_lo = (MODE == PASS_FIRST) ? T_K0 : ((MODE == PASS_MEASURE) ? T_S : T_K1);
  constexpr int t_hi = (MODE == PASS_FIRST) ? T_K0 : T_UT;
#pragma unroll
  for (int a = t_lo; a <= t_hi; ++a) {
    const u128 v = wave_sum128(acc[a]);
    if (lane == 0) sRed[wave][a] = v;
  }
  // non-finite flags: any lane of any wave
  __shared__ uint32_t sBadW[NW];
  const unsigned long long any_bad = __ballot(bad != 0u);
  if (lane == 0) sBadW[wave] = any_bad ? 1u : 0u;
  __shared__ int sLast;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int a = t_lo; a <= t_hi; ++a) {
      u128 v = sRed[0][a];
      for (int w = 1; w < NW; ++w) v = add128(v, sRed[w][a]);
      atomic_add_limbs(st->acc[a][slot], v);
    }
    uint32_t anyb = 0u;
    for (int w = 0; w < NW; ++w) anyb |= sBadW[w];
    if (anyb) (void)__hip_atomic_fetch_or(&st->bad, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (MODE != PASS_FIRST) sLast = publish_done(&st->done, cd.n_tiles) ? 1 : 0;
  }
  if (MODE == PASS_FIRST) return;
  __syncthreads();
  if (!sLast) return;
  close_chain<MODE == PASS_LAST>(cd, st, pass_in_buf(cur, j));
}


// Terms of four x-aligned sites held by four consecutive lanes, summed as
// (t0 + t1) + (t2 + t3) in FP64 (FP addition is commutative, so every lane of
// the quad forms the identical value; lane 4q keeps it, the other three give 0).
__device__ __forceinline__ double quad_sum_lanes(double t) {
  t = t + __shfl_xor(t, 1, 64);
  t = t + __shfl_xor(t, 2, 64);
  return ((threadIdx.x & 3) == 0) ? t : 0.0;
}

// Block reduction of the terms [a_lo, a_hi] and their accumulation into the
// chain, without counting the block as finished (used where another kernel
// closes the trajectory).
template <int NW>
__device__ __forceinline__ void block_add_terms(ChainState* st, const u128* acc, uint32_t bad, int a_lo, int a_hi,
                                                int slot) {
  __shared__ u128 sRedA[NW][NTERM];
  __shared__ uint32_t sBadA[NW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int a = a_lo; a <= a_hi; ++a) {
    const u128 v = wave_sum128(acc[a]);
    if (lane == 0) sRedA[wave][a] = v;
  }
  const unsigned long long any_bad = __ballot(bad != 0u);
  if (lane == 0) sBadA[wave] = any_bad ? 1u : 0u;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int a = a_lo; a <= a_hi; ++a) {
      u128 v = sRedA[0][a];
      for (int w = 1; w < NW; ++w) v = add128(v, sRedA[w][a]);
      atomic_add_limbs(st->acc[a][slot], v);
    }
    uint32_t anyb = 0u;
    for (int w = 0; w < NW; ++w) anyb |= sBadA[w];
    if (anyb) (void)__hip_atomic_fetch_or(&st->bad, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace ihmc
