// Trajectory epilogue shared by the lattice and dense kernels: block reduction
// of the exact fixed-point sums, their store into per-tile entries, and the
// work of the block that finishes last -- the Metropolis test of Sec. 3 on
// dH = H_new - H_old in FP64 (exact integer difference of the fixed-point
// Hamiltonians), the optional global sign flip, and the Sec. 4 estimators.
#pragma once

#include "device_common.hpp"
#include "lattice_kernels.hpp"

namespace ihmc {

// Metropolis decision and record, run by one thread of the last block of a LAST
// pass once the block has gathered the chain's accumulators (`sum`, `bad`).
// Returns the record's flags (REC_ACCEPT, REC_FLIP, REC_NONFINITE).
//
// In the phi form the estimator slots hold the sums of t = tanh(h' + phi):
// T_PSI sum t, T_PSIH sum h' t, T_UT t.K t, and `t2` is sum t^2 of the
// proposal; the records then hold the spin expectations given phi.
__device__ __forceinline__ uint32_t finalize_trajectory(const ChainDev& cd, ChainState* st, int last_buf,
                                                        const u128* sum, uint32_t bad, double t2 = 0.0) {
  // Every field of the state that the step reads is loaded up front (one round
  // trip of independent loads rather than a chain of dependent ones) and the
  // changed ones are stored at the end.
  const int t = st->traj;
  u128 S{st->S_lo, st->S_hi};
  int cur_bad = st->cur_bad;
  int cur = st->cur, sign = st->sign;
  double sum_psi = st->sum_psi, sum_psih = st->sum_psih, sum_ut = st->sum_ut, sum_t2 = st->sum_t2;
  int64_t n_acc = st->n_acc, n_nonfinite = st->n_nonfinite;
  double sum_exp_mdh = st->sum_exp_mdh;

  const u128 H_old = add128(sum[T_K0], S);
  const u128 H_new = add128(sum[T_K1], sum[T_S]);
  double dH = fixed_to_double(sub128(H_new, H_old));
  uint32_t flags = 0u;
  bool finite = (bad == 0u);
  const bool counted = (t >= cd.n_therm);  // past thermalisation: enters the summary
  if (!finite) {
    dH = __builtin_nan("");
    flags |= REC_NONFINITE;
    if (counted) n_nonfinite += 1;
  }
  if (finite && cur_bad) dH = -__builtin_inf();  // leaving a state of zero weight
  bool accept;
  if (cd.replay && t < cd.cap) {
    accept = cd.replay[t] != 0;
  } else {
    const double r = uniform_at(cd, (uint32_t)t, TAG_ACC);
    accept = finite && (dH <= 0.0 || r < exp(-dH));
  }
  if (finite && !cur_bad && counted) sum_exp_mdh += exp(-dH);
  if (accept) {
    cur_bad = 0;
    S = sum[T_S];
    sum_psi = fixed_to_double(sum[T_PSI]);
    sum_psih = fixed_to_double(sum[T_PSIH]);
    sum_ut = fixed_to_double(sum[T_UT]);
    sum_t2 = t2;
    cur = last_buf;
    sign = 1;
    if (counted) n_acc += 1;
    flags |= REC_ACCEPT;
  }
  if (cd.flip_every > 0 && (t + 1) % cd.flip_every == 0) {
    // S(-psi) - S(psi) = 2 psi.h'/sqrt(J'): only the linear field term changes.
    // A change that the fixed-point action cannot hold (non-finite, or
    // |dS| >= 2^62) rejects the flip and marks the record.
    const double dS = 2.0 * sum_psih / cd.sqJ;
    const double r2 = uniform_at(cd, (uint32_t)t, TAG_FLIP);
    u128 dSf;
    if (!to_fixed_wide(dS, dSf)) {
      if (finite && counted) n_nonfinite += 1;
      flags |= REC_NONFINITE;
    } else if (dS <= 0.0 || r2 < exp(-dS)) {
      S = add128(S, dSf);
      sign = -sign;
      sum_psi = -sum_psi;
      sum_psih = -sum_psih;
      flags |= REC_FLIP;
    }
  }
  if (t < cd.cap) {
    const double N = (double)cd.N;
    TrajRecord rec;
    rec.dH = dH;
    rec.H_old = fixed_to_double(H_old);
    rec.H_new = fixed_to_double(H_new);
    if (cd.form == FORM_PHI) {
      // E[s_i | phi] = t_i, spins independent given phi
      rec.m = sum_psi / N;
      rec.abs_m = fabs(rec.m);
      rec.m2c = (sum_psi * sum_psi - sum_t2 + N) / (N * N);
      rec.beta_eps = (-0.5 * cd.Jp * sum_ut - sum_psih) / N;
    } else if (cd.form == FORM_SHIFTED) {
      // the paper's estimators at psi + Kt^-1 h'/sqrt(J'): no Kt^-1 terms;
      // sum_ut holds sum y tanh(y), y = sqrt(J') u + h'
      rec.m = sum_psi / cd.sqJ / N;
      rec.abs_m = fabs(rec.m);
      rec.m2c = rec.m * rec.m - cd.c_v / (N * N * cd.Jp);
      rec.beta_eps = 0.5 * cd.C * cd.Jp - sum_psih / (2.0 * N * cd.sqJ) - sum_ut / (2.0 * N);
    } else {
      rec.m = (sum_psi / cd.sqJ - cd.c_m / cd.Jp) / N;
      rec.abs_m = fabs(rec.m);
      rec.m2c = rec.m * rec.m - cd.c_v / (N * N * cd.Jp);
      rec.beta_eps = 0.5 * cd.C * cd.Jp + cd.c_e / (2.0 * N * cd.Jp) - sum_psih / (2.0 * N * cd.sqJ) -
                     cd.sqJ / (2.0 * N) * sum_ut;
    }
    rec.flags = flags;
    rec.pad = 0u;
    cd.rec[t] = rec;
  }
  st->S_lo = S.lo;
  st->S_hi = S.hi;
  st->cur_bad = cur_bad;
  st->cur = cur;
  st->sign = sign;
  st->sum_psi = sum_psi;
  st->sum_psih = sum_psih;
  st->sum_ut = sum_ut;
  st->sum_t2 = sum_t2;
  st->n_acc = n_acc;
  st->n_nonfinite = n_nonfinite;
  st->sum_exp_mdh = sum_exp_mdh;
  st->traj = t + 1;
  __hip_atomic_store(&st->bad, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&st->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return flags;
}

__device__ __forceinline__ void finalize_measure(ChainState* st, const u128* sum, uint32_t bad, double t2 = 0.0) {
  st->cur_bad = bad ? 1 : 0;
  st->sum_t2 = t2;
  st->S_lo = sum[T_S].lo;
  st->S_hi = sum[T_S].hi;
  st->sum_psi = fixed_to_double(sum[T_PSI]);
  st->sum_psih = fixed_to_double(sum[T_PSIH]);
  st->sum_ut = fixed_to_double(sum[T_UT]);
  __hip_atomic_store(&st->bad, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&st->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------- partial sums ---
//
// Every block of a pass that contributes FP64 terms stores its exact
// fixed-point block sums in its own entries of the chain's partial table
// (part[tile][NPART] of 128-bit values; the last entry holds non-finite flags
// as 32-bit words: 0 the momenta of the first pass, 1 the final momenta, 2 the
// action terms).  Stores and loads of the table are agent-scope (coherent across
// the XCDs' L2 caches); a full wait for outstanding memory operations precedes
// every counter increment, so a closer that sees the final count also sees every
// entry counted.  Tiles are counted in groups (part_group): the block that completes
// a group sums the group's entries (integer sums: exact, in any order), and the
// block that completes the last group closes the chain.  No two blocks ever add
// into the same memory, so large chains do not serialise on a few cache lines.

__device__ __forceinline__ uint64_t* part_entry(uint64_t* base, int64_t idx, int a) {
  return base + (idx * NPART + a) * 2;
}
__device__ __forceinline__ void store_u128_agent(uint64_t* p, u128 v) {
  __hip_atomic_store(&p[0], v.lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&p[1], v.hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u128 load_u128_agent(const uint64_t* p) {
  return u128{__hip_atomic_load(&p[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
              __hip_atomic_load(&p[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)};
}
__device__ __forceinline__ void store_flag_agent(uint64_t* entry, int word, uint32_t v) {
  __hip_atomic_store((uint32_t*)entry + word, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t load_flag_agent(const uint64_t* entry, int word) {
  return __hip_atomic_load((const uint32_t*)entry + word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Count one finished unit at `counter`; true for the unit that completes `n`.
//
// Ordering: the entries are agent-scope atomic stores, which write through to
// the memory that all XCDs share, and the counter is an agent-scope atomic.
// The compiler barriers keep the entry stores above the wait and the counter
// update below it; the wait for every outstanding memory operation makes the
// entries complete (visible to every agent-scope load) before the counter
// moves.  After the update, a compiler barrier keeps the caller's gathers of
// the entries below it, and they are issued only once its return value has
// arrived (they depend on it).  A release/acquire pair at agent scope would
// say the same in the language's model, but on this GPU an agent-scope
// release writes back the whole L2 of the XCD, including the field and momenta
// the pass has just written, which the next launch does not need early.
__device__ __forceinline__ bool count_done(uint32_t* counter, uint32_t n) {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);  // the entries stored above have completed
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  const uint32_t prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  return prev == n - 1u;
}

// Sums over `count` consecutive entries of terms [a_lo, a_hi] and the OR of
// the flag words in `wmask`: one wave per term, lanes striding over entries.
// Results in sum[] / *flags (LDS) for thread 0 after the closing barrier.
template <int NW>
__device__ __forceinline__ void gather_entries(const uint64_t* base, int count, int a_lo, int a_hi, uint32_t wmask,
                                               u128* sum, uint32_t* flags) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int a = a_lo + wave; a <= a_hi; a += NW) {
    u128 v{0ull, 0ull};
    for (int i = lane; i < count; i += 64) v = add128(v, load_u128_agent(part_entry((uint64_t*)base, i, a)));
    v = wave_sum128(v);
    if (lane == 0) sum[a] = v;
  }
  if (wave == NW - 1) {
    uint32_t f = 0u;
    for (int i = lane; i < count; i += 64) {
      const uint64_t* e = part_entry((uint64_t*)base, i, NTERM);
#pragma unroll
      for (int w = 0; w < 3; ++w)
        if (wmask & (1u << w)) f |= load_flag_agent(e, w);
    }
    const unsigned long long any = __ballot(f != 0u);
    if (lane == 0) *flags = any ? 1u : 0u;
  }
  __syncthreads();
}

// Terms of four x-aligned sites held by four consecutive lanes, summed as
// (t0 + t1) + (t2 + t3) in FP64; every lane of the quad gets the identical value.
__device__ __forceinline__ double quad_sum_all(double t) {
  t = t + dpp_f64<DPP_QUAD_XOR1>(t);
  return t + dpp_f64<DPP_QUAD_XOR2>(t);
}

// Flag words a pass stores, by kind of contribution.
enum : int { CONTRIB_FIRST = 0, CONTRIB_FINAL_KIN = 1, CONTRIB_ACTION = 2, CONTRIB_LAST = 3 };

// Block reduction of the per-thread fixed-point sums of terms [a_lo, a_hi] and
// their store into the chain's entries of tile `tix`; flag words per `kind`.
template <int NW>
__device__ __forceinline__ void block_store_terms(const ChainDev& cd, const u128* acc, uint32_t bad, int a_lo,
                                                  int a_hi, int kind, int tix) {
  __shared__ u128 sRedA[NW][NTERM];
  __shared__ uint32_t sBadA[NW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < NTERM; ++a) {
    if (a < a_lo || a > a_hi) continue;
    const u128 v = wave_sum128(acc[a]);
    if (lane == 0) sRedA[wave][a] = v;
  }
  const unsigned long long any_bad = __ballot(bad != 0u);
  if (lane == 0) sBadA[wave] = any_bad ? 1u : 0u;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t* base = cd.part;
    for (int a = a_lo; a <= a_hi; ++a) {
      u128 v = sRedA[0][a];
      for (int w = 1; w < NW; ++w) v = add128(v, sRedA[w][a]);
      store_u128_agent(part_entry(base, tix, a), v);
    }
    uint32_t anyb = 0u;
    for (int w = 0; w < NW; ++w) anyb |= sBadA[w];
    uint64_t* fe = part_entry(base, tix, NTERM);
    if (kind == CONTRIB_FIRST) store_flag_agent(fe, 0, anyb);
    if (kind == CONTRIB_FINAL_KIN || kind == CONTRIB_LAST) store_flag_agent(fe, 1, anyb);
    if (kind == CONTRIB_ACTION || kind == CONTRIB_LAST) store_flag_agent(fe, 2, anyb);
  }
}

// As block_store_terms, for accumulators dealt over the lanes of each quad:
// the pass's terms t0 .. t0 + nterms - 1 in rank order, rank 4k + j held by
// lane j (mod 4) of every quad in accR[k] (the quad's four lanes hold the same
// FP64 sums, so each converts a different term to fixed point).  The sums over
// the lanes of one residue are the terms' block sums, as before.
template <int NW, int NR>
__device__ __forceinline__ void block_store_ranks(const ChainDev& cd, const u128 (&accR)[NR], uint32_t bad, int t0,
                                                  int nterms, int kind, int tix) {
  __shared__ u128 sRedR[NW][NTERM];
  __shared__ uint32_t sBadR[NW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    u128 v = accR[k];
    // the four lanes of each residue within a row (DPP), then across rows
    v = add128(v, dpp_u128<DPP_ROW_ROR4>(v));
    v = add128(v, dpp_u128<DPP_ROW_ROR8>(v));
#pragma unroll
    for (int off = 16; off < 64; off <<= 1) {
      u128 o;
      o.lo = __shfl_xor(v.lo, off, 64);
      o.hi = __shfl_xor(v.hi, off, 64);
      v = add128(v, o);
    }
    const int r = 4 * k + lane;
    if (lane < 4 && r < nterms) sRedR[wave][t0 + r] = v;
  }
  const unsigned long long any_bad = __ballot(bad != 0u);
  if (lane == 0) sBadR[wave] = any_bad ? 1u : 0u;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t* base = cd.part;
    for (int a = t0; a < t0 + nterms; ++a) {
      u128 v = sRedR[0][a];
      for (int w = 1; w < NW; ++w) v = add128(v, sRedR[w][a]);
      store_u128_agent(part_entry(base, tix, a), v);
    }
    uint32_t anyb = 0u;
    for (int w = 0; w < NW; ++w) anyb |= sBadR[w];
    uint64_t* fe = part_entry(base, tix, NTERM);
    if (kind == CONTRIB_FIRST) store_flag_agent(fe, 0, anyb);
    if (kind == CONTRIB_FINAL_KIN || kind == CONTRIB_LAST) store_flag_agent(fe, 1, anyb);
    if (kind == CONTRIB_ACTION || kind == CONTRIB_LAST) store_flag_agent(fe, 2, anyb);
  }
}

// After block_store_terms of a closing pass (LAST or MEASURE): count the tile,
// and in the block completing its group / the chain, sum the entries and run
// the Metropolis step (kTraj) or the measurement of the accepted field.
template <bool kTraj, int NW>
__device__ __forceinline__ void block_close(const ChainDev& cd, ChainState* st, int last_buf, int tix) {
  __shared__ u128 sSum[NTERM];
  __shared__ uint32_t sFlag, sLast;
  const int a_lo = kTraj ? T_K0 : T_S;
  const uint32_t wmask = kTraj ? 7u : 4u;
  const int pg = part_group(cd.n_tiles);
  const int g = tix / pg;
  const int ng = (int)part_groups(cd.n_tiles);
  const int gs = min(pg, (int)cd.n_tiles - g * pg);
  if (threadIdx.x == 0) sLast = count_done(&cd.gcnt[g], (uint32_t)gs) ? 1u : 0u;
  __syncthreads();
  if (!sLast) return;
  // this block completed group g
  gather_entries<NW>(cd.part + (int64_t)g * pg * NPART * 2, gs, a_lo, T_UT, wmask, sSum, &sFlag);
  if (ng > 1) {
    if (threadIdx.x == 0) {
      __hip_atomic_store(&cd.gcnt[g], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      for (int a = a_lo; a <= T_UT; ++a) store_u128_agent(part_entry(cd.gsum, g, a), sSum[a]);
      store_flag_agent(part_entry(cd.gsum, g, NTERM), 0, sFlag);
      sLast = count_done(&st->done, (uint32_t)ng) ? 1u : 0u;
    }
    __syncthreads();
    if (!sLast) return;
    // this block completed the chain: sum the group sums (flags in word 0)
    gather_entries<NW>(cd.gsum, ng, a_lo, T_UT, 1u, sSum, &sFlag);
  }
  if (threadIdx.x == 0) {
    if (ng == 1) __hip_atomic_store(&cd.gcnt[g], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    u128 sum[NTERM];
#pragma unroll
    for (int a = 0; a < NTERM; ++a) sum[a] = (a >= a_lo) ? sSum[a] : u128{0ull, 0ull};
    if (kTraj) finalize_trajectory(cd, st, last_buf, sum, sFlag);
    else finalize_measure(st, sum, sFlag);
  }
}

// Site terms are summed per quad of four x-aligned sites (x = 4q .. 4q+3; in the dense
// path, site indices 4q .. 4q+3) as (t0 + t1) + (t2 + t3) in FP64; 2D lattice
// passes then sum four consecutive quads (16 x-aligned sites) the same way, 3D
// ones the quads of a column's 4-plane slab, before one conversion to fixed
// point.  The groups are the same in every tiling, so the totals stay
// tile-independent.
__device__ __forceinline__ double quad_sum(double t0, double t1, double t2, double t3) {
  return (t0 + t1) + (t2 + t3);
}

// Epilogue of a lattice pass: store the block's terms (FIRST: kinetic energy of
// the fresh momenta; LAST: final kinetic energy and the action terms; MEASURE:
// the action terms) and close the chain where this block completes it;
// last_buf is the buffer holding the proposal (LAST).
template <int MODE, int NW>
__device__ __forceinline__ void block_accumulate(const ChainDev& cd, ChainState* st, const u128* acc, uint32_t bad,
                                                 int last_buf, int tix) {
  constexpr int t_lo = (MODE == PASS_FIRST) ? T_K0 : ((MODE == PASS_MEASURE) ? T_S : T_K1);
  constexpr int t_hi = (MODE == PASS_FIRST) ? T_K0 : T_UT;
  constexpr int kind = (MODE == PASS_FIRST) ? CONTRIB_FIRST : ((MODE == PASS_MEASURE) ? CONTRIB_ACTION : CONTRIB_LAST);
  block_store_terms<NW>(cd, acc, bad, t_lo, t_hi, kind, tix);
  if (MODE == PASS_FIRST) return;
  block_close<MODE == PASS_LAST, NW>(cd, st, last_buf, tix);
}

// The same with accumulators dealt over the lanes of each quad (block_store_ranks).
template <int MODE, int NW, int NR>
__device__ __forceinline__ void block_accumulate_ranks(const ChainDev& cd, ChainState* st, const u128 (&accR)[NR],
                                                       uint32_t bad, int last_buf, int tix) {
  constexpr int t_lo = (MODE == PASS_FIRST) ? T_K0 : ((MODE == PASS_MEASURE) ? T_S : T_K1);
  constexpr int t_hi = (MODE == PASS_FIRST) ? T_K0 : T_UT;
  constexpr int kind = (MODE == PASS_FIRST) ? CONTRIB_FIRST : ((MODE == PASS_MEASURE) ? CONTRIB_ACTION : CONTRIB_LAST);
  block_store_ranks<NW, NR>(cd, accR, bad, t_lo, t_hi - t_lo + 1, kind, tix);
  if (MODE == PASS_FIRST) return;
  block_close<MODE == PASS_LAST, NW>(cd, st, last_buf, tix);
}

}  // namespace ihmc
