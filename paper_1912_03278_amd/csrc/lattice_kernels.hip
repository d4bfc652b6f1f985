// Fused leap-frog passes for HMC on periodic 2D / 3D nearest-neighbour lattices.
//
// One pass = one force evaluation of the equations of motion (Sec. 3):
//     u = Kt psi,  w = sqrt(J') tanh(sqrt(J') u) - psi,  F = Kt w + h'/sqrt(J'),
// followed by the kick p += c_j F and the drift psi' = psi + d_j p.  Because F
// at a site needs psi on the radius-2 diamond around it, a workgroup stages its
// tile plus a 2-wide halo of psi in LDS, computes w on the tile plus a 1-wide
// halo, and then F, p and psi' on the tile: every pass reads psi (and p) once
// and writes p and psi' once from HBM.
//
// Pass kinds (template MODE):
//   FIRST   - momenta from Philox (Sec. 3, eq. momentum distribution), 1/2 p^2
//             accumulated for H_old, first kick and drift;
//   MIDDLE  - kick and drift;
//   LAST    - final kick, then the FP64 Hamiltonian and estimator sums of the
//             proposal; the last block to finish takes the Metropolis decision
//             (Sec. 3) and writes the trajectory record (Sec. 4 estimators);
//   MEASURE - FP64 action and estimator sums of the accepted field (set-up);
//   FORCE   - writes F itself (diagnostic; same arithmetic as the other passes).
//
// Sums are exact 128-bit fixed point (device_common.hpp), so every result is
// independent of the tile shape and of which chains share a launch.
#include "device_common.hpp"
#include "lattice_kernels.hpp"

namespace ihmc {

template <int NDIM, int BX, int BY, int BZ>
struct Geom {
  static constexpr int Z3 = (NDIM == 3) ? 1 : 0;
  static constexpr int PX = BX + 4, PY = BY + 4, PZ = Z3 ? BZ + 4 : 1;
  static constexpr int WX = BX + 2, WY = BY + 2, WZ = Z3 ? BZ + 2 : 1;
  static constexpr int NP = PX * PY * PZ;
  static constexpr int NW = WX * WY * WZ;
  static constexpr int BZE = Z3 ? BZ : 1;
  static constexpr int NO = BX * BY * BZE;
};

__device__ __forceinline__ int wrap_near(int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }
__device__ __forceinline__ int wrap_any(int v, int L) {
  const int r = v % L;
  return r < 0 ? r + L : r;
}

template <typename T>
__device__ __forceinline__ T neg_if(T v, int sign) {
  return sign < 0 ? -v : v;
}

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
  const int k = threadIdx.x;
  if (k < NTERM * NSLOT) {
    const int a = k / NSLOT, sl = k % NSLOT;
    sAcc[a][sl] = load128_agent(st->acc[a][sl]);
  }
  if (k == 0) sBad = __hip_atomic_load(&st->bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  if (k < NTERM * NSLOT) {
    const int a = k / NSLOT, sl = k % NSLOT;
    store128_agent(st->acc[a][sl], u128{0ull, 0ull});
  }
  if (k == 0) {
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
// accumulation into the chain, and the last block's epilogue.
template <int MODE>
__device__ __forceinline__ void block_accumulate(const ChainDev& cd, ChainState* st, const u128* acc,
                                                 uint32_t bad, u128 (*sRed)[NTERM], int cur, int j) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int t_lo = (MODE == PASS_FIRST) ? T_K0 : ((MODE == PASS_MEASURE) ? T_S : T_K1);
  constexpr int t_hi = (MODE == PASS_FIRST) ? T_K0 : T_UT;
#pragma unroll
  for (int a = t_lo; a <= t_hi; ++a) {
    const u128 v = wave_sum128(acc[a]);
    if (lane == 0) sRed[wave][a] = v;
  }
  // non-finite flags: any lane of any wave
  __shared__ uint32_t sBadW[4];
  const unsigned long long any_bad = __ballot(bad != 0u);
  if (lane == 0) sBadW[wave] = any_bad ? 1u : 0u;
  __shared__ int sLast;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int slot = blockIdx.x % NSLOT;
    for (int a = t_lo; a <= t_hi; ++a) {
      u128 v = add128(add128(sRed[0][a], sRed[1][a]), add128(sRed[2][a], sRed[3][a]));
      atomic_add128(st->acc[a][slot], v);
    }
    if (sBadW[0] | sBadW[1] | sBadW[2] | sBadW[3])
      (void)__hip_atomic_fetch_or(&st->bad, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (MODE != PASS_FIRST) sLast = publish_done(&st->done, cd.n_tiles) ? 1 : 0;
  }
  if (MODE == PASS_FIRST) return;
  __syncthreads();
  if (!sLast) return;
  close_chain<MODE == PASS_LAST>(cd, st, pass_in_buf(cur, j));
}

template <typename T, int NDIM, int BX, int BY, int BZ, int MODE>
__global__ __launch_bounds__(256) void lattice_pass(const ChainDev* __restrict__ chains,
                                                    const Tile* __restrict__ tiles, int j) {
  using G = Geom<NDIM, BX, BY, BZ>;
  constexpr bool kHasW = (MODE != PASS_MEASURE);
  constexpr bool kH64 = (MODE == PASS_LAST || MODE == PASS_MEASURE);
  __shared__ T sP[G::NP];
  __shared__ T sW[kHasW ? G::NW : 1];
  __shared__ u128 sRed[4][NTERM];

  const Tile tl = tiles[blockIdx.x];
  const ChainDev& cd = chains[tl.chain];
  ChainState* st = cd.st;
  const int L0 = cd.L0, L1 = cd.L1, L2 = cd.L2;
  const int64_t N = cd.N;
  const int cur = st->cur;
  const int sign = st->sign;
  const int traj = st->traj;
  const bool from_cur = (MODE == PASS_FIRST || MODE == PASS_MEASURE || MODE == PASS_FORCE);
  const int in_buf = from_cur ? cur : pass_in_buf(cur, j);
  const int out_buf = pass_out_buf(cur, j);
  const T* __restrict__ pin = (const T*)cd.psi + (int64_t)in_buf * N;
  T* __restrict__ pout = (T*)cd.psi + (int64_t)out_buf * N;
  T* __restrict__ pmom = (T*)cd.p;

  // ---- stage psi on the tile plus a 2-wide halo (periodic wrap)
  const bool near = (L0 > BX) && (L1 > BY) && (NDIM == 2 || L2 > BZ);
  for (int i = threadIdx.x; i < G::NP; i += 256) {
    const int lx = i % G::PX;
    const int r = i / G::PX;
    const int ly = r % G::PY;
    const int lz = r / G::PY;
    int gx = tl.x0 + lx - 2, gy = tl.y0 + ly - 2, gz = G::Z3 ? tl.z0 + lz - 2 : 0;
    if (near) {
      gx = wrap_near(gx, L0);
      gy = wrap_near(gy, L1);
      if (G::Z3) gz = wrap_near(gz, L2);
    } else {
      gx = wrap_any(gx, L0);
      gy = wrap_any(gy, L1);
      if (G::Z3) gz = wrap_any(gz, L2);
    }
    const int64_t g = gx + (int64_t)L0 * (gy + (int64_t)L1 * gz);
    T v = pin[g];
    if (from_cur) v = neg_if(v, sign);
    sP[i] = v;
  }
  __syncthreads();

  const T Ct = (T)cd.C;
  const T at = (T)cd.sqJ;
  constexpr int SP = G::PX * G::PY;
  constexpr int SW = G::WX * G::WY;

  // ---- w = sqrt(J') tanh(sqrt(J') Kt psi) - psi on the tile plus a 1-wide halo
  if (kHasW) {
    for (int i = threadIdx.x; i < G::NW; i += 256) {
      const int wx = i % G::WX;
      const int r = i / G::WX;
      const int wy = r % G::WY;
      const int wz = r / G::WY;
      const int pc = (wx + 1) + G::PX * ((wy + 1) + G::PY * (wz + G::Z3));
      const T c = sP[pc];
      T s = (sP[pc - 1] + sP[pc + 1]) + (sP[pc - G::PX] + sP[pc + G::PX]);
      if (G::Z3) s = s + (sP[pc - SP] + sP[pc + SP]);
      const T u = fma_t(Ct, c, s);
      sW[i] = fma_t(at, tanh_state(at * u), -c);
    }
    __syncthreads();
  }

  // Momenta of the first pass: one Philox draw feeds the two sites of a pair.
  // With an even row length a pair never straddles a row, so the tile draws
  // each pair once and stages both normals in LDS.
  constexpr bool kMom = (MODE == PASS_FIRST);
  __shared__ T sMom[kMom ? G::NO : 1];
  const bool pair_rows = ((L0 & 1) == 0);
  if (kMom && !cd.p_given && pair_rows) {
    for (int q = threadIdx.x; q < G::NO / 2; q += 256) {
      const int o = 2 * q;
      const int lx = o % BX;
      const int r = o / BX;
      const int ly = r % BY;
      const int lz = r / BY;
      const int gx = tl.x0 + lx, gy = tl.y0 + ly, gz = tl.z0 + lz;
      if (gx >= L0 || gy >= L1 || (G::Z3 && gz >= L2)) continue;
      const int64_t site = gx + (int64_t)L0 * (gy + (int64_t)L1 * gz);
      T z0, z1;
      normal_pair<T>(cd, (uint32_t)traj, TAG_MOM, site >> 1, z0, z1);
      sMom[o] = z0;
      sMom[o + 1] = z1;
    }
    __syncthreads();
  }

  double kick_d = 0.0, drift_d = 0.0;
  pass_coeffs(cd, j, kick_d, drift_d);
  const T kick = (MODE == PASS_FORCE) ? (T)1 : (T)kick_d;
  const T drift = (T)drift_d;
  const T b_uniform = (T)cd.b0;
  const T* __restrict__ bsite = (const T*)cd.b;
  const bool site_field = (cd.h_kind == 2);

  uint32_t bad = 0u;
  u128 acc[NTERM];
#pragma unroll
  for (int a = 0; a < NTERM; ++a) acc[a] = u128{0ull, 0ull};

  auto site_body = [&](int o) {
    const int lx = o % BX;
    const int r = o / BX;
    const int ly = r % BY;
    const int lz = r / BY;
    const int gx = tl.x0 + lx, gy = tl.y0 + ly, gz = tl.z0 + lz;
    if (gx >= L0 || gy >= L1 || (G::Z3 && gz >= L2)) return;
    const int64_t site = gx + (int64_t)L0 * (gy + (int64_t)L1 * gz);
    const int pc = (lx + 2) + G::PX * ((ly + 2) + G::PY * (lz + 2 * G::Z3));
    const T c = sP[pc];
    T pn = (T)0;
    if (kHasW) {
      const int wc = (lx + 1) + G::WX * ((ly + 1) + G::WY * (lz + G::Z3));
      T sw = (sW[wc - 1] + sW[wc + 1]) + (sW[wc - G::WX] + sW[wc + G::WX]);
      if (G::Z3) sw = sw + (sW[wc - SW] + sW[wc + SW]);
      T F = fma_t(Ct, sW[wc], sw);
      F = F + (site_field ? bsite[site] : b_uniform);
      T p;
      if (MODE == PASS_FIRST) {
        if (cd.p_given) {
          p = pmom[site];
        } else if (pair_rows) {
          p = sMom[o];
        } else {
          T z0, z1;
          normal_pair<T>(cd, (uint32_t)traj, TAG_MOM, site >> 1, z0, z1);
          p = (site & 1) ? z1 : z0;
        }
        const double pd = (double)p;
        acc[T_K0] = add128(acc[T_K0], to_fixed(0.5 * pd * pd, bad));
      } else if (MODE == PASS_FORCE) {
        p = (T)0;
      } else {
        p = pmom[site];
      }
      pn = fma_t(kick, F, p);
      if (MODE == PASS_FIRST || MODE == PASS_MIDDLE) {
        pmom[site] = pn;
        pout[site] = fma_t(drift, pn, c);
      } else if (MODE == PASS_FORCE) {
        pmom[site] = pn;
      } else if (MODE == PASS_LAST) {
        if (cd.write_p_last) pmom[site] = pn;
        const double pd = (double)pn;
        acc[T_K1] = add128(acc[T_K1], to_fixed(0.5 * pd * pd, bad));
      }
    }
    if (kH64) {
      // FP64 action terms of the field as stored: the integer stencil weights
      // are exact, C and sqrt(J') are the true FP64 constants.
      const double cdv = (double)c;
      double nb = ((double)sP[pc - 1] + (double)sP[pc + 1]) + ((double)sP[pc - G::PX] + (double)sP[pc + G::PX]);
      if (G::Z3) nb = nb + ((double)sP[pc - SP] + (double)sP[pc + SP]);
      const double u = cd.C * cdv + nb;
      double lc, th;
      logcosh_tanh(cd.sqJ * u, lc, th);
      double hpx = cd.hp0, bx = cd.b0;
      if (site_field) {
        hpx = cd.hp[site];
        bx = hpx / cd.sqJ;
      }
      acc[T_S] = add128(acc[T_S], to_fixed(0.5 * cdv * u - cdv * bx - lc, bad));
      acc[T_PSI] = add128(acc[T_PSI], to_fixed(cdv, bad));
      acc[T_PSIH] = add128(acc[T_PSIH], to_fixed(cdv * hpx, bad));
      acc[T_UT] = add128(acc[T_UT], to_fixed(u * th, bad));
    }
  };
  if constexpr (MODE == PASS_MIDDLE || MODE == PASS_FORCE) {
#pragma unroll
    for (int o = threadIdx.x; o < G::NO; o += 256) site_body(o);
  } else {
#pragma unroll 1
    for (int o = threadIdx.x; o < G::NO; o += 256) site_body(o);
  }

  if (MODE == PASS_MIDDLE || MODE == PASS_FORCE) return;
  block_accumulate<MODE>(cd, st, acc, bad, sRed, cur, j);
}


// 3D passes as a 2.5D stream: a block owns a BX x BY column of the xy plane
// and walks z over [z0, z0 + ZR).  A ring of five psi planes (2-wide xy halo)
// and three w planes (1-wide halo) stays in LDS, so each psi value is read
// from memory (ZR + 4) / ZR times and each w is computed (BX+2)(BY+2)/(BX BY)
// times, instead of staging a full 3D halo box per tile.  Step z computes
// w(z+1) and the update of plane z while the loads of plane z+3 are in flight.
template <typename T, int BX, int BY, int ZR, int MODE>
__global__ __launch_bounds__(256) void lattice_pass3s(const ChainDev* __restrict__ chains,
                                                      const Tile* __restrict__ tiles, int j) {
  constexpr int PX = BX + 4, PY = BY + 4, PP = PX * PY;
  constexpr int WX = BX + 2, WY = BY + 2, WP = WX * WY;
  constexpr int NO = BX * BY;
  constexpr bool kHasW = (MODE != PASS_MEASURE);
  constexpr bool kH64 = (MODE == PASS_LAST || MODE == PASS_MEASURE);
  __shared__ T sP[5][PP];
  __shared__ T sW[kHasW ? 3 : 1][kHasW ? WP : 1];
  __shared__ u128 sRed[4][NTERM];

  const Tile tl = tiles[blockIdx.x];
  const ChainDev& cd = chains[tl.chain];
  ChainState* st = cd.st;
  const int L0 = cd.L0, L1 = cd.L1, L2 = cd.L2;
  const int64_t N = cd.N;
  const int64_t plane = (int64_t)L0 * L1;
  const int cur = st->cur;
  const int sign = st->sign;
  const int traj = st->traj;
  const bool from_cur = (MODE == PASS_FIRST || MODE == PASS_MEASURE || MODE == PASS_FORCE);
  const int in_buf = from_cur ? cur : pass_in_buf(cur, j);
  const int out_buf = pass_out_buf(cur, j);
  const T* __restrict__ pin = (const T*)cd.psi + (int64_t)in_buf * N;
  T* __restrict__ pout = (T*)cd.psi + (int64_t)out_buf * N;
  T* __restrict__ pmom = (T*)cd.p;
  const int z_end = min(tl.z0 + ZR, L2);
  const bool near_xy = (L0 > BX) && (L1 > BY);

  const T Ct = (T)cd.C;
  const T at = (T)cd.sqJ;
  double kick_d = 0.0, drift_d = 0.0;
  pass_coeffs(cd, j, kick_d, drift_d);
  const T kick = (MODE == PASS_FORCE) ? (T)1 : (T)kick_d;
  const T drift = (T)drift_d;
  const T b_uniform = (T)cd.b0;
  const T* __restrict__ bsite = (const T*)cd.b;
  const bool site_field = (cd.h_kind == 2);

  // Plane z (any integer in [z0-2, z_end+2]) of psi: fetch_plane issues the
  // global loads into registers, store_plane moves them to ring slot
  // (z - z0 + 2) % 5.  Splitting the two lets the loads of plane z+3 overlap
  // the compute of plane z.
  constexpr int NPRE = (PP + 255) / 256;
  auto fetch_plane = [&](int z, T (&pre)[NPRE]) {
    int gz = z;
    if (gz < 0) gz += L2;
    else if (gz >= L2) gz -= L2;
    if (gz < 0 || gz >= L2) gz = wrap_any(z, L2);
    const T* src = pin + (int64_t)gz * plane;
#pragma unroll
    for (int k = 0; k < NPRE; ++k) {
      const int i = threadIdx.x + 256 * k;
      if (i < PP) {
        const int lx = i % PX, ly = i / PX;
        int gx = tl.x0 + lx - 2, gy = tl.y0 + ly - 2;
        if (near_xy) {
          gx = wrap_near(gx, L0);
          gy = wrap_near(gy, L1);
        } else {
          gx = wrap_any(gx, L0);
          gy = wrap_any(gy, L1);
        }
        T v = src[gx + (int64_t)L0 * gy];
        if (from_cur) v = neg_if(v, sign);
        pre[k] = v;
      }
    }
  };
  auto store_plane = [&](int z, const T (&pre)[NPRE]) {
    T* dst = sP[(z - tl.z0 + 2) % 5];
#pragma unroll
    for (int k = 0; k < NPRE; ++k) {
      const int i = threadIdx.x + 256 * k;
      if (i < PP) dst[i] = pre[k];
    }
  };
  // w on plane z from psi planes z-1, z, z+1
  auto compute_w = [&](int z) {
    const T* __restrict__ pm = sP[(z - 1 - tl.z0 + 2) % 5];
    const T* __restrict__ pc = sP[(z - tl.z0 + 2) % 5];
    const T* __restrict__ pp = sP[(z + 1 - tl.z0 + 2) % 5];
    T* __restrict__ w = sW[(z - tl.z0 + 3) % 3];
    for (int i = threadIdx.x; i < WP; i += 256) {
      const int wx = i % WX, wy = i / WX;
      const int c = (wx + 1) + PX * (wy + 1);
      const T v = pc[c];
      T sum = (pc[c - 1] + pc[c + 1]) + (pc[c - PX] + pc[c + PX]);
      sum = sum + (pm[c] + pp[c]);
      const T u = fma_t(Ct, v, sum);
      w[i] = fma_t(at, tanh_state(at * u), -v);
    }
  };

  uint32_t bad = 0u;
  u128 acc[NTERM];
#pragma unroll
  for (int a = 0; a < NTERM; ++a) acc[a] = u128{0ull, 0ull};

  // prologue: psi planes z0-2 .. z0+2 in LDS, w planes z0-1, z0
  {
    T pre[5][NPRE];
#pragma unroll
    for (int q = 0; q < 5; ++q) fetch_plane(tl.z0 - 2 + q, pre[q]);
#pragma unroll
    for (int q = 0; q < 5; ++q) store_plane(tl.z0 - 2 + q, pre[q]);
  }
  __syncthreads();
  if (kHasW) {
    compute_w(tl.z0 - 1);
    compute_w(tl.z0);
  }

  for (int z = tl.z0; z < z_end; ++z) {
    // w(z+1) needs psi planes z .. z+2 (in LDS); plane z+3 is fetched meanwhile
    T pre[NPRE];
    const bool more = (z + 1 < z_end);
    if (more) fetch_plane(z + 3, pre);
    if (kHasW) compute_w(z + 1);
    __syncthreads();
    const T* __restrict__ pm = sP[(z - 1 - tl.z0 + 2) % 5];
    const T* __restrict__ pc = sP[(z - tl.z0 + 2) % 5];
    const T* __restrict__ pp = sP[(z + 1 - tl.z0 + 2) % 5];
    const T* __restrict__ wm = sW[kHasW ? (z - 1 - tl.z0 + 3) % 3 : 0];
    const T* __restrict__ wc = sW[kHasW ? (z - tl.z0 + 3) % 3 : 0];
    const T* __restrict__ wp = sW[kHasW ? (z + 1 - tl.z0 + 3) % 3 : 0];
    for (int o = threadIdx.x; o < NO; o += 256) {
      const int lx = o % BX, ly = o / BX;
      const int gx = tl.x0 + lx, gy = tl.y0 + ly;
      if (gx >= L0 || gy >= L1) continue;
      const int64_t site = gx + (int64_t)L0 * (gy + (int64_t)L1 * z);
      const int c = (lx + 2) + PX * (ly + 2);
      const T v = pc[c];
      if (kHasW) {
        const int q = (lx + 1) + WX * (ly + 1);
        T sw = (wc[q - 1] + wc[q + 1]) + (wc[q - WX] + wc[q + WX]);
        sw = sw + (wm[q] + wp[q]);
        T F = fma_t(Ct, wc[q], sw);
        F = F + (site_field ? bsite[site] : b_uniform);
        T p;
        if (MODE == PASS_FIRST) {
          if (cd.p_given) {
            p = pmom[site];
          } else {
            T z0, z1;
            normal_pair<T>(cd, (uint32_t)traj, TAG_MOM, site >> 1, z0, z1);
            p = (site & 1) ? z1 : z0;
          }
          const double pd = (double)p;
          acc[T_K0] = add128(acc[T_K0], to_fixed(0.5 * pd * pd, bad));
        } else if (MODE == PASS_FORCE) {
          p = (T)0;
        } else {
          p = pmom[site];
        }
        const T pn = fma_t(kick, F, p);
        if (MODE == PASS_FIRST || MODE == PASS_MIDDLE) {
          pmom[site] = pn;
          pout[site] = fma_t(drift, pn, v);
        } else if (MODE == PASS_FORCE) {
          pmom[site] = pn;
        } else if (MODE == PASS_LAST) {
          if (cd.write_p_last) pmom[site] = pn;
          const double pd = (double)pn;
          acc[T_K1] = add128(acc[T_K1], to_fixed(0.5 * pd * pd, bad));
        }
      }
      if (kH64) {
        const double cdv = (double)v;
        double nb = ((double)pc[c - 1] + (double)pc[c + 1]) + ((double)pc[c - PX] + (double)pc[c + PX]);
        nb = nb + ((double)pm[c] + (double)pp[c]);
        const double u = cd.C * cdv + nb;
        double lc, th;
        logcosh_tanh(cd.sqJ * u, lc, th);
        double hpx = cd.hp0, bx = cd.b0;
        if (site_field) {
          hpx = cd.hp[site];
          bx = hpx / cd.sqJ;
        }
        acc[T_S] = add128(acc[T_S], to_fixed(0.5 * cdv * u - cdv * bx - lc, bad));
        acc[T_PSI] = add128(acc[T_PSI], to_fixed(cdv, bad));
        acc[T_PSIH] = add128(acc[T_PSIH], to_fixed(cdv * hpx, bad));
        acc[T_UT] = add128(acc[T_UT], to_fixed(u * th, bad));
      }
    }
    // plane z+3 replaces plane z-2, which no later step reads
    if (more) store_plane(z + 3, pre);
    __syncthreads();
  }

  if (MODE == PASS_MIDDLE || MODE == PASS_FORCE) return;
  block_accumulate<MODE>(cd, st, acc, bad, sRed, cur, j);
}

// ------------------------------------------------------------------ launch ---

template <typename T, int BX, int BY, int ZR>
static hipError_t launch_mode3s(int mode, const ChainDev* chains, const Tile* tiles, int n_tiles, int j,
                                hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  dim3 grid(n_tiles), block(256);
  switch (mode) {
    case PASS_FIRST:
      lattice_pass3s<T, BX, BY, ZR, PASS_FIRST><<<grid, block, 0, s>>>(chains, tiles, j);
      break;
    case PASS_MIDDLE:
      lattice_pass3s<T, BX, BY, ZR, PASS_MIDDLE><<<grid, block, 0, s>>>(chains, tiles, j);
      break;
    case PASS_LAST:
      lattice_pass3s<T, BX, BY, ZR, PASS_LAST><<<grid, block, 0, s>>>(chains, tiles, j);
      break;
    case PASS_MEASURE:
      lattice_pass3s<T, BX, BY, ZR, PASS_MEASURE><<<grid, block, 0, s>>>(chains, tiles, j);
      break;
    case PASS_FORCE:
      lattice_pass3s<T, BX, BY, ZR, PASS_FORCE><<<grid, block, 0, s>>>(chains, tiles, j);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int NDIM, int BX, int BY, int BZ>
static hipError_t launch_mode(int mode, const ChainDev* chains, const Tile* tiles, int n_tiles, int j,
                              hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  dim3 grid(n_tiles), block(256);
  switch (mode) {
    case PASS_FIRST:
      lattice_pass<T, NDIM, BX, BY, BZ, PASS_FIRST><<<grid, block, 0, s>>>(chains, tiles, j);
      break;
    case PASS_MIDDLE:
      lattice_pass<T, NDIM, BX, BY, BZ, PASS_MIDDLE><<<grid, block, 0, s>>>(chains, tiles, j);
      break;
    case PASS_LAST:
      lattice_pass<T, NDIM, BX, BY, BZ, PASS_LAST><<<grid, block, 0, s>>>(chains, tiles, j);
      break;
    case PASS_MEASURE:
      lattice_pass<T, NDIM, BX, BY, BZ, PASS_MEASURE><<<grid, block, 0, s>>>(chains, tiles, j);
      break;
    case PASS_FORCE:
      lattice_pass<T, NDIM, BX, BY, BZ, PASS_FORCE><<<grid, block, 0, s>>>(chains, tiles, j);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// 3D column tiles: BX x BY in the plane, streamed over ZR planes.
#ifndef IHMC_3D_BX
#define IHMC_3D_BX 32
#define IHMC_3D_BY 8
#define IHMC_3D_ZR 4
#endif

int tile_class(int ndim, int L0) {
  if (ndim == 2) return L0 < 48 ? 1 : 0;
  return 0;
}

TileShape tile_shape(int precision, int ndim, int cls) {
  (void)precision;
  if (ndim == 2) return cls == 1 ? TileShape{16, 16, 1} : TileShape{64, 16, 1};
  return TileShape{IHMC_3D_BX, IHMC_3D_BY, IHMC_3D_ZR};
}

hipError_t launch_lattice_pass(int precision, int ndim, int cls, int mode, const ChainDev* chains,
                               const Tile* tiles, int n_tiles, int j, hipStream_t s) {
  if (precision == 4) {
    if (ndim == 2) {
      if (cls == 1) return launch_mode<float, 2, 16, 16, 1>(mode, chains, tiles, n_tiles, j, s);
      return launch_mode<float, 2, 64, 16, 1>(mode, chains, tiles, n_tiles, j, s);
    }
    return launch_mode3s<float, IHMC_3D_BX, IHMC_3D_BY, IHMC_3D_ZR>(mode, chains, tiles, n_tiles, j, s);
  }
  if (ndim == 2) {
    if (cls == 1) return launch_mode<double, 2, 16, 16, 1>(mode, chains, tiles, n_tiles, j, s);
    return launch_mode<double, 2, 64, 16, 1>(mode, chains, tiles, n_tiles, j, s);
  }
  return launch_mode3s<double, IHMC_3D_BX, IHMC_3D_BY, IHMC_3D_ZR>(mode, chains, tiles, n_tiles, j, s);
}

}  // namespace ihmc
