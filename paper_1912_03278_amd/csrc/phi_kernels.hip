// HMC in the inverse formulation of Sec. 2 (eq. cosh_in_exponent): the field
// phi with the action
//     S(phi) = 1/(2J') phi.Kt^-1 phi - sum_i log cosh(h'_i + phi_i)
// and the force -Kt^-1 phi / J' + tanh(h' + phi).  The paper recommends the
// substitution phi = sqrt(J') Kt psi - h' instead, because this form needs a
// linear solve at every force evaluation; this kernel runs it as the A/B
// baseline of that claim, on the same chains and the same GPU.
//
// One 256-thread workgroup runs whole trajectories of one chain (FP64 state)
// with every array in LDS in site order: the accepted and working field, the
// momenta, and the conjugate-gradient vectors x, r, d, q (plus h' for a
// per-site field).  Kt x = phi is solved by CG from x = 0 to a relative
// residual of 1e-14 (rr <= 1e-28 rr0, at most 20000 iterations), with the
// inner products reduced in a fixed order, so the force is a deterministic
// function of phi (leap-frog stays reversible).  The last force evaluation of
// a trajectory is at the proposal itself, so its solution also gives the
// proposal's phi.Kt^-1 phi.  Sums for H and the estimators are exact fixed
// point, as in the psi form, and the Metropolis step and the records are the
// shared epilogue's (estimators: E[s_i | phi] = tanh(h'_i + phi_i)).
#include "chain_epilogue.hpp"
#include "device_common.hpp"
#include "lattice_kernels.hpp"

namespace ihmc {

constexpr int PHI_THREADS = 256;
constexpr int PHI_LDS_BYTES = 81408;  // as the psi form's resident kernel: two chains per CU
constexpr double kCgTol2 = 1e-28;
constexpr int kCgMaxIter = 20000;

int resident_phi_max_sites(bool site_field) { return PHI_LDS_BYTES / ((site_field ? 8 : 7) * 8); }

template <int NDIM>
__global__ __launch_bounds__(PHI_THREADS) void lattice_resident_phi(const ChainDev* __restrict__ chains,
                                                                    const Tile* __restrict__ tiles, int n_traj) {
  __shared__ __align__(16) double lds[PHI_LDS_BYTES / 8];
  __shared__ double sDot[PHI_THREADS / 64];
  __shared__ u128 sRed[PHI_THREADS / 64][NTERM];
  __shared__ uint32_t sBad[PHI_THREADS / 64];
  __shared__ double sT2[PHI_THREADS / 64];
  __shared__ int sTraj;
  __shared__ uint32_t sFlags;
  const ChainDev& cd = chains[tiles[blockIdx.x].chain];
  ChainState* st = cd.st;
  const int L0 = cd.L0, L1 = cd.L1, L2 = (NDIM == 3) ? cd.L2 : 1;
  const int N = (int)cd.N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool site_field = (cd.h_kind == 2);
  double* sA = lds;       // accepted field
  double* sP = sA + N;    // working field
  double* sM = sP + N;    // momenta
  double* sX = sM + N;    // CG solution
  double* sR = sX + N;    // CG residual
  double* sD = sR + N;    // CG direction
  double* sQ = sD + N;    // Kt d
  double* sH = sQ + N;    // h' per site (site field only)
  const int pitch = cd.pitch, plane = L0 * L1;
  const int cur = st->cur;
  double* gphi = (double*)cd.psi + (int64_t)cur * cd.NP;
  for (int i = tid; i < N; i += PHI_THREADS) {
    const int64_t g = (i % L0) + (int64_t)pitch * (i / L0);
    sA[i] = gphi[g];
    if (site_field) sH[i] = cd.hp[g];
  }
  const double hp0 = cd.hp0, C = cd.C, Jp = cd.Jp;

  // periodic neighbour sum of field v at site i = x + L0 (y + L1 z)
  auto nb_sum = [&](const double* v, int i) {
    const int x = i % L0, r = i / L0, y = r % L1, z = r / L1;
    double s = (v[i + (x == 0 ? L0 - 1 : -1)] + v[i + (x == L0 - 1 ? 1 - L0 : 1)]) +
               (v[i + (y == 0 ? (L1 - 1) * L0 : -L0)] + v[i + (y == L1 - 1 ? -(L1 - 1) * L0 : L0)]);
    if (NDIM == 3)
      s = s + (v[i + (z == 0 ? (L2 - 1) * plane : -plane)] + v[i + (z == L2 - 1 ? -(L2 - 1) * plane : plane)]);
    return s;
  };
  // a.b over the sites in a fixed order (per thread in site order, the waves'
  // lane 0 sums, then the four waves), the same value in every thread
  auto block_dot = [&](const double* a, const double* b) {
    double s = 0.0;
    for (int i = tid; i < N; i += PHI_THREADS) s = __builtin_fma(a[i], b[i], s);
    for (int off = 32; off > 0; off >>= 1) s = s + __shfl_xor(s, off, 64);
    __syncthreads();  // earlier readers of sDot are done
    if (lane == 0) sDot[wave] = s;
    __syncthreads();
    return (sDot[0] + sDot[1]) + (sDot[2] + sDot[3]);
  };
  // x = Kt^-1 sP by CG from x = 0; returns the iterations
  auto solve = [&]() {
    for (int i = tid; i < N; i += PHI_THREADS) {
      sX[i] = 0.0;
      sR[i] = sP[i];
      sD[i] = sP[i];
    }
    __syncthreads();
    double rr = block_dot(sR, sR);
    const double stop = kCgTol2 * rr;
    int it = 0;
    while (rr > stop && it < kCgMaxIter) {
      for (int i = tid; i < N; i += PHI_THREADS) sQ[i] = __builtin_fma(C, sD[i], nb_sum(sD, i));
      __syncthreads();
      const double alpha = rr / block_dot(sD, sQ);
      for (int i = tid; i < N; i += PHI_THREADS) {
        sX[i] = __builtin_fma(alpha, sD[i], sX[i]);
        sR[i] = __builtin_fma(-alpha, sQ[i], sR[i]);
      }
      __syncthreads();
      const double rn = block_dot(sR, sR);
      const double beta = rn / rr;
      rr = rn;
      for (int i = tid; i < N; i += PHI_THREADS) sD[i] = __builtin_fma(beta, sD[i], sR[i]);
      __syncthreads();
      ++it;
    }
    return it;
  };
  auto hprime = [&](int i) { return site_field ? sH[i] : hp0; };
  // The block's fixed-point totals of the per-thread sums (thread 0 gets them).
  auto block_total = [&](const u128* acc, uint32_t bad, double t2, u128* sum, double* t2_out) {
#pragma unroll
    for (int a = 0; a < NTERM; ++a) {
      const u128 v = wave_sum128(acc[a]);
      if (lane == 0) sRed[wave][a] = v;
    }
    double w = t2;
    for (int off = 32; off > 0; off >>= 1) w = w + __shfl_xor(w, off, 64);
    const unsigned long long any = __ballot(bad != 0u);
    if (lane == 0) {
      sBad[wave] = any ? 1u : 0u;
      sT2[wave] = w;
    }
    __syncthreads();
    uint32_t b = 0u;
    if (tid == 0) {
      for (int a = 0; a < NTERM; ++a) {
        u128 v = sRed[0][a];
        for (int k = 1; k < PHI_THREADS / 64; ++k) v = add128(v, sRed[k][a]);
        sum[a] = v;
      }
      for (int k = 0; k < PHI_THREADS / 64; ++k) b |= sBad[k];
      *t2_out = (sT2[0] + sT2[1]) + (sT2[2] + sT2[3]);
    }
    return b;
  };
  // Action and estimator terms of the field in sP with sX = Kt^-1 sP, into the
  // thread's accumulators; returns the thread's sum of t^2.
  auto action_terms = [&](u128* acc, uint32_t& bad) {
    double s = 0.0, ts = 0.0, hts = 0.0, tkt = 0.0, t2 = 0.0;
    // t = tanh(h' + phi) into sR (free after the solve)
    for (int i = tid; i < N; i += PHI_THREADS) {
      double lc, t;
      logcosh_tanh(sP[i] + hprime(i), lc, t);
      sR[i] = t;
    }
    __syncthreads();
    for (int i = tid; i < N; i += PHI_THREADS) {
      double lc, t;
      logcosh_tanh(sP[i] + hprime(i), lc, t);
      s = s + (0.5 * sP[i] * sX[i] / Jp - lc);
      ts = ts + t;
      hts = hts + hprime(i) * t;
      tkt = tkt + t * nb_sum(sR, i);
      t2 = t2 + t * t;
    }
    acc[T_S] = add128(acc[T_S], to_fixed(s, bad));
    acc[T_PSI] = add128(acc[T_PSI], to_fixed(ts, bad));
    acc[T_PSIH] = add128(acc[T_PSIH], to_fixed(hts, bad));
    acc[T_UT] = add128(acc[T_UT], to_fixed(tkt, bad));
    __syncthreads();  // sR is a CG vector again afterwards
    return t2;
  };

  int64_t cg_iters = 0;
  if (n_traj == 0) {  // set-up: S and the estimator sums of the accepted field
    for (int i = tid; i < N; i += PHI_THREADS) sP[i] = sA[i];
    __syncthreads();
    cg_iters += solve();
    u128 acc[NTERM];
    for (int a = 0; a < NTERM; ++a) acc[a] = u128{0ull, 0ull};
    uint32_t bad = 0u;
    const double t2 = action_terms(acc, bad);
    u128 sum[NTERM];
    double t2s = 0.0;
    const uint32_t b = block_total(acc, bad, t2, sum, &t2s);
    if (tid == 0) {
      finalize_measure(st, sum, b, t2s);
      st->n_cg += cg_iters;
    }
    return;
  }

  for (int t = 0; t < n_traj; ++t) {
    if (tid == 0) sTraj = st->traj;
    __syncthreads();
    const uint32_t traj = (uint32_t)sTraj;
    for (int i = tid; i < N; i += PHI_THREADS) sP[i] = sA[i];
    for (int pr = tid; 2 * pr < N; pr += PHI_THREADS) {
      double z0, z1;
      normal_pair<double>(cd, traj, TAG_MOM, pr, z0, z1);
      sM[2 * pr] = z0;
      if (2 * pr + 1 < N) sM[2 * pr + 1] = z1;
    }
    __syncthreads();
    u128 acc[NTERM];
    for (int a = 0; a < NTERM; ++a) acc[a] = u128{0ull, 0ull};
    uint32_t bad = 0u;
    {
      double k0 = 0.0;
      for (int i = tid; i < N; i += PHI_THREADS) k0 = k0 + 0.5 * sM[i] * sM[i];
      acc[T_K0] = to_fixed(k0, bad);
    }
    // leap-frog: kick at phi, then drift (the last pass kicks only)
    for (int j = 0; j < cd.n_pass; ++j) {
      cg_iters += solve();
      double kick = 0.0, drift = 0.0;
      pass_coeffs(cd, j, kick, drift);
      const bool last = (j == cd.n_pass - 1);
      for (int i = tid; i < N; i += PHI_THREADS) {
        double lc, th;
        logcosh_tanh(sP[i] + hprime(i), lc, th);
        const double F = th - sX[i] / Jp;
        const double p = __builtin_fma(kick, F, sM[i]);
        sM[i] = p;
        if (!last) sP[i] = __builtin_fma(drift, p, sP[i]);
      }
      __syncthreads();
    }
    // the last solve was at the proposal: its action and estimator terms
    {
      double k1 = 0.0;
      for (int i = tid; i < N; i += PHI_THREADS) k1 = k1 + 0.5 * sM[i] * sM[i];
      acc[T_K1] = to_fixed(k1, bad);
    }
    const double t2 = action_terms(acc, bad);
    u128 sum[NTERM];
    double t2s = 0.0;
    const uint32_t b = block_total(acc, bad, t2, sum, &t2s);
    if (tid == 0) sFlags = finalize_trajectory(cd, st, cur, sum, b, t2s);
    __syncthreads();
    if (sFlags & REC_ACCEPT)
      for (int i = tid; i < N; i += PHI_THREADS) sA[i] = sP[i];
    __syncthreads();
  }
  if (tid == 0) st->n_cg += cg_iters;
  // the accepted field back to its buffer (finalize kept st->cur = cur)
  for (int i = tid; i < N; i += PHI_THREADS) gphi[(i % L0) + (int64_t)pitch * (i / L0)] = sA[i];
}

hipError_t launch_lattice_resident_phi(int ndim, const ChainDev* chains, const Tile* tiles, int n_chains, int n_traj,
                                       hipStream_t s) {
  if (n_chains <= 0) return hipSuccess;
  if (ndim == 2) lattice_resident_phi<2><<<n_chains, PHI_THREADS, 0, s>>>(chains, tiles, n_traj);
  else lattice_resident_phi<3><<<n_chains, PHI_THREADS, 0, s>>>(chains, tiles, n_traj);
  return hipGetLastError();
}

}  // namespace ihmc
