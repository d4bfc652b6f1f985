// Local Metropolis-Hastings on the spins: the comparison method of Sec. 4
// (T_HMC ~ 4 N_step T_MH there), run on the same GPU as the HMC path.
//
// A sweep proposes every spin once, in checkerboard order: the sites of even
// parity x + y + z, then the odd ones.  On a periodic lattice of even extents
// no two sites of one parity are neighbours, so each half-sweep is one launch
// of independent single-site updates (one thread per site of the colour):
// dE = 2 s_i (J sum_nb s_j + h), accepted iff dE <= 0 or u < exp(-beta dE),
// u the 53-bit uniform of Philox counter (i, sweep, chain, TAG_MH).  The
// acceptance probabilities take 2 (2d + 1) values; they are computed once on
// the host and passed in, so every decision is exactly the oracle's.  The two
// half-sweeps also sum the final spins and the bonds (integers, exact in any
// order) per block, and a one-block launch adds the blocks' sums into the
// sweep's slot.  Spins are int8 in site order.  One sweep's three launches are
// captured into a HIP graph and replayed; the sweep index lives in device
// memory.
//
// With an explicit coupling matrix (the all-to-all models of Sec. 2 and
// App. A) every spin couples to every other, so the spins of a chain are
// proposed one after another in site order.  A chain is one workgroup that
// keeps the local fields f_j = sum_{k != j} K_jk s_k of its sites in
// registers; a flip of s_i adds 2 s_i K_ij to every f_j.  The proposals run in
// blocks of 64 sites on the wave that holds the block (no barrier between
// them), and the block's flips reach the other fields afterwards, from the
// flipped rows of K only (delayed updates).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "device_common.hpp"
#include "runtime_internal.hpp"

namespace ihmc {

constexpr uint32_t TAG_MH = 5u, TAG_MH_INIT = 6u;

struct MhParams {
  int32_t ndim, L0, L1, L2;
  int64_t N;
  uint32_t seed_lo, seed_hi, chain;
  double J, h;
  double p[2][13];  // exp(-beta dE) by spin (0: -1, 1: +1) and neighbour sum + 2d
};

__device__ __forceinline__ double mh_uniform(const MhParams& q, uint32_t i, uint32_t t, uint32_t tag) {
  const uint4 w = philox4x32_10(make_uint4(i, t, q.chain, tag), q.seed_lo, q.seed_hi);
  return unit53(w.x, w.y);
}

__global__ void k_mh_init(MhParams q, int8_t* __restrict__ s, const int8_t* __restrict__ s0) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= q.N) return;
  s[i] = s0 ? (s0[i] > 0 ? 1 : -1) : (mh_uniform(q, (uint32_t)i, 0u, TAG_MH_INIT) < 0.5 ? 1 : -1);
}

// Sum of one int64 per thread over the block (wave shuffles, then the four
// waves in order); thread 0 gets it.
__device__ __forceinline__ long long block_sum_i64(long long v, long long* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  long long t = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
  __syncthreads();
  return t;
}

// One half-sweep: every site of parity `color`.  Thread k -> row r = k / (L0/2)
// (y = r % L1, z = r / L1), x = 2 (k % (L0/2)) + ((y + z + color) & 1), the
// threads striding over the colour's sites.  The measurement of the sweep
// rides along: every bond has exactly one odd endpoint, and when the odd
// sites are updated all their neighbours (even) are final, so the odd half
// adds s_i times its neighbour sum over its sites, which is the sum of
// s_i s_{i+mu} over all sites and axes; each half adds its sites' final spins.
// Per block: part[3 b] accepted flips, part[3 b + 1] spin sum, part[3 b + 2]
// bond sum.
__global__ __launch_bounds__(256) void k_mh_half(MhParams q, int8_t* __restrict__ s, const int* __restrict__ sweep,
                                                 int color, long long* __restrict__ part) {
  __shared__ long long sh[4];
  const int half = q.L0 >> 1;
  const uint32_t t_sweep = (uint32_t)*sweep;
  long long acc = 0, ss = 0, bs = 0;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < q.N / 2;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = k / half;
    const int y = (int)(r % q.L1), z = (int)(r / q.L1);
    const int x = 2 * (int)(k % half) + ((y + z + color) & 1);
    const int64_t row = (int64_t)q.L0 * (y + (int64_t)q.L1 * z);
    const int64_t i = x + row;
    int sum = (int)s[row + (x + 1 == q.L0 ? 0 : x + 1)] + (int)s[row + (x == 0 ? q.L0 - 1 : x - 1)];
    const int64_t plane = (int64_t)q.L0 * q.L1;
    const int64_t yp = (y + 1 == q.L1 ? -(int64_t)(q.L1 - 1) : 1) * q.L0;
    const int64_t ym = (y == 0 ? (int64_t)(q.L1 - 1) : -1) * q.L0;
    sum += (int)s[i + yp] + (int)s[i + ym];
    if (q.ndim == 3) {
      const int64_t zp = (z + 1 == q.L2 ? -(int64_t)(q.L2 - 1) : 1) * plane;
      const int64_t zm = (z == 0 ? (int64_t)(q.L2 - 1) : -1) * plane;
      sum += (int)s[i + zp] + (int)s[i + zm];
    }
    int si = s[i];
    const double dE = 2.0 * si * (q.J * sum + q.h);
    const double u = mh_uniform(q, (uint32_t)i, t_sweep, TAG_MH);
    if (dE <= 0.0 || u < q.p[si > 0 ? 1 : 0][sum + 2 * q.ndim]) {
      si = -si;
      s[i] = (int8_t)si;
      acc += 1;
    }
    ss += si;
    if (color == 1) bs += (long long)si * sum;
  }
  const long long a = block_sum_i64(acc, sh);
  const long long b = block_sum_i64(ss, sh);
  const long long c = block_sum_i64(bs, sh);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = a;
    part[3 * blockIdx.x + 1] = b;
    part[3 * blockIdx.x + 2] = c;
  }
}

// One block: the sweep's totals from the two halves' partials (n blocks each:
// spin and bond sums into acc[2 t], acc[2 t + 1], accepted flips onto
// *n_acc), then the sweep index advances.
__global__ __launch_bounds__(1024) void k_mh_reduce(const long long* __restrict__ part, int n, int* sweep,
                                                    long long* __restrict__ acc, unsigned long long* n_acc) {
  __shared__ long long sh[16];
  long long na = 0, ss = 0, bs = 0;
  for (int b = threadIdx.x; b < 2 * n; b += blockDim.x) {
    na += part[3 * b];
    ss += part[3 * b + 1];
    bs += part[3 * b + 2];
  }
  na = block_sum_i64(na, sh);
  ss = block_sum_i64(ss, sh);
  bs = block_sum_i64(bs, sh);
  if (threadIdx.x == 0) {
    const int t = *sweep;
    acc[2 * t] = ss;
    acc[2 * t + 1] = bs;
    *n_acc += (unsigned long long)na;
    *sweep = t + 1;
  }
}

__global__ void k_mh_clear(long long* acc, int64_t n, int* sweep, unsigned long long* n_acc) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) acc[i] = 0;
  if (i == 0) {
    *sweep = 0;
    *n_acc = 0ull;
  }
}


// ----------------------------------------------------------------- dense ---

struct DenseMhParams {
  int32_t N, Np;  // sites; row pitch of the padded K (multiple of the block size)
  int32_t h_kind; // 0: none, 1: uniform, 2: per site
  uint32_t seed_lo, seed_hi, chain0;
  double J, beta, h0;
};

constexpr int DMH_THREADS = 512;

__device__ __forceinline__ double dmh_uniform(const DenseMhParams& q, uint32_t chain, uint32_t i, uint32_t t,
                                              uint32_t tag) {
  const uint4 w = philox4x32_10(make_uint4(i, t, chain, tag), q.seed_lo, q.seed_hi);
  return unit53(w.x, w.y);
}

// Sum of one double per thread over the block, in a fixed order (waves by
// shuffle-free LDS tree), so the result does not depend on timing.
__device__ __forceinline__ double dmh_block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = DMH_THREADS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// One workgroup per chain, n_sweeps sweeps, with the spins proposed in blocks
// of 64 consecutive sites and the fields updated late (delayed updates).
// Thread t owns the sites j = t + DMH_THREADS r, r < R: lane j % 64 of wave
// (j % DMH_THREADS) / 64, register r, so the 64 sites of block n are the lanes
// of wave n % 8 in register n / 8.  Per block:
//   A  that wave runs the block's proposals in order: lane k decides from its
//      own field, the decision is broadcast within the wave (no barrier), and a
//      flip of s_k adds 2 s_k K_kl to the fields of the block's other lanes
//      from the block's 64 x 64 diagonal part of K, staged in LDS;
//   B  one barrier, then every thread adds the block's flips to the fields of
//      its other sites from the flipped rows of K only (a compacted list, rows
//      read four or eight at a time), while the next diagonal block is staged;
//      a barrier.
// Every field takes the flips in increasing site order, the order of a
// sweep, so it holds the same FP64 value as when each flip is applied at
// once.  The test u < exp(-beta dE) is taken as dE < -ln(u) / beta with the
// threshold computed for every site before the sweep (off the proposals'
// dependent chain); the two differ only where u and exp(-beta dE) agree to
// rounding.
// rec[(c * n_sweeps + t) * 3 + {0, 1, 2}] = sum s, s^T K s, sum h s after sweep t.
constexpr int DMH_BLK = 64;

template <int R>
__global__ __launch_bounds__(DMH_THREADS, 1) void k_dense_mh(DenseMhParams q, const double* __restrict__ K,
                                                            const double* __restrict__ hsite,
                                                            const int8_t* __restrict__ spins0,
                                                            int8_t* __restrict__ spins, int n_sweeps,
                                                            double* __restrict__ rec,
                                                            unsigned long long* __restrict__ n_acc) {
  constexpr int NW = DMH_THREADS / 64;
  constexpr int DMH_Q = R >= 8 ? 4 : 8;  // flipped rows read at once (R values each, in registers)
  static_assert(DMH_THREADS % 64 == 0 && DMH_BLK == 64, "one block per wave");
  __shared__ double sKd[2][DMH_BLK * DMH_BLK];
  __shared__ int sList[2][DMH_BLK];  // flipped block-local sites, increasing
  __shared__ int sNew[2][DMH_BLK];   // their new spins
  __shared__ int sCount[2];
  __shared__ int8_t sS[R * DMH_THREADS];
  __shared__ double sh[DMH_THREADS];
  const int c = blockIdx.x;
  const uint32_t chain = q.chain0 + (uint32_t)c;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int N = q.N;
  const int64_t Np = q.Np;
  const int NB = (N + DMH_BLK - 1) / DMH_BLK;

  // start spins: given, or +1 iff the uniform of (i, 0, chain, TAG_MH_INIT) < 1/2
  int s[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = t + DMH_THREADS * r;
    int v = 0;
    if (j < N) {
      if (spins0)
        v = spins0[(int64_t)c * N + j] > 0 ? 1 : -1;
      else
        v = dmh_uniform(q, chain, (uint32_t)j, 0u, TAG_MH_INIT) < 0.5 ? 1 : -1;
    }
    s[r] = v;
    sS[j] = (int8_t)v;
  }
  double hv[R], f[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = t + DMH_THREADS * r;
    hv[r] = (j < N) ? (q.h_kind == 2 ? hsite[j] : q.h0) : 0.0;
    f[r] = 0.0;
  }
  __syncthreads();
  // f_j = sum_{k != j} K_kj s_k over the rows k (K is symmetric); unrolled so
  // that several rows' loads are in flight
#pragma unroll 8
  for (int k = 0; k < N; ++k) {
    const double sk = (double)sS[k];
    const double* row = K + (int64_t)k * Np;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j = t + DMH_THREADS * r;
      if (j != k) f[r] = __builtin_fma(row[j], sk, f[r]);
    }
  }
  unsigned long long acc = 0ull;

  // the diagonal 64 x 64 part of K of block n, 8 values per thread
  auto diag_load = [&](int n, double (&v)[DMH_BLK * DMH_BLK / DMH_THREADS]) {
#pragma unroll
    for (int m = 0; m < DMH_BLK * DMH_BLK / DMH_THREADS; ++m) {
      const int e = t + DMH_THREADS * m, a = e >> 6, b = e & 63;
      v[m] = K[(int64_t)(DMH_BLK * n + a) * Np + DMH_BLK * n + b];
    }
  };
  auto diag_store = [&](int buf, const double (&v)[DMH_BLK * DMH_BLK / DMH_THREADS]) {
#pragma unroll
    for (int m = 0; m < DMH_BLK * DMH_BLK / DMH_THREADS; ++m) sKd[buf][t + DMH_THREADS * m] = v[m];
  };

  for (int ts = 0; ts < n_sweeps; ++ts) {
    // acceptance thresholds of the owned sites: accept iff dE < -ln(u)/beta
    double thr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j = t + DMH_THREADS * r;
      const double u = (j < N) ? dmh_uniform(q, chain, (uint32_t)j, (uint32_t)ts, TAG_MH) : 0.5;
      thr[r] = -ln_unit(u) / q.beta;  // +inf for beta = 0: every proposal is taken
    }
    {
      double v[DMH_BLK * DMH_BLK / DMH_THREADS];
      diag_load(0, v);
      diag_store(0, v);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      for (int w = 0; w < NW; ++w) {
        const int n = NW * r + w;  // block n: wave w, register r
        if (n >= NB) break;        // uniform over the workgroup
        const int buf = n & 1;
        // ---- A: the block's proposals, in order, on wave w
        if (wave == w) {
          const int kmax = min(DMH_BLK, N - DMH_BLK * n);
          double fl = f[r];
          int sl = s[r];
          for (int k = 0; k < kmax; ++k) {
            const double dE = 2.0 * (double)sl * (q.J * fl + hv[r]);
            const int take = __builtin_amdgcn_readlane((dE <= 0.0 || dE < thr[r]) ? 1 : 0, k);
            if (take) {
              const int sk = -__builtin_amdgcn_readlane(sl, k);  // the new spin of site k
              if (lane == k)
                sl = sk;
              else
                fl = __builtin_fma(sKd[buf][k * DMH_BLK + lane], 2.0 * (double)sk, fl);
            }
          }
          const bool flipped = (lane < kmax) && (sl != s[r]);
          const unsigned long long mask = __ballot(flipped);
          if (flipped) {
            const int idx = __popcll(mask & ((1ull << lane) - 1ull));
            sList[buf][idx] = lane;
            sNew[buf][idx] = sl;
          }
          if (lane == 0) sCount[buf] = __popcll(mask);
          acc += flipped ? 1ull : 0ull;
          f[r] = fl;
          s[r] = sl;
        }
        __syncthreads();
        // ---- B: the block's flips into every other field; the next diagonal block staged
        double v[DMH_BLK * DMH_BLK / DMH_THREADS];
        if (n + 1 < NB) diag_load(n + 1, v);
        const int cnt = sCount[buf];
        for (int q0 = 0; q0 < cnt; q0 += DMH_Q) {
          double kr[DMH_Q][R];
#pragma unroll
          for (int qq = 0; qq < DMH_Q; ++qq) {
            const int k = (q0 + qq < cnt) ? sList[buf][q0 + qq] : sList[buf][q0];
            const double* row = K + (int64_t)(DMH_BLK * n + k) * Np + t;
#pragma unroll
            for (int rr = 0; rr < R; ++rr) kr[qq][rr] = row[DMH_THREADS * rr];
          }
#pragma unroll
          for (int qq = 0; qq < DMH_Q; ++qq) {
            if (q0 + qq < cnt) {
              const double dv = 2.0 * (double)sNew[buf][q0 + qq];
#pragma unroll
              for (int rr = 0; rr < R; ++rr)
                if (rr != r || wave != w) f[rr] = __builtin_fma(kr[qq][rr], dv, f[rr]);
            }
          }
        }
        if (n + 1 < NB) diag_store(buf ^ 1, v);
        __syncthreads();
      }
    }
    // measurement of the sweep: sum s, s^T K s = sum_j s_j (f_j + K_jj s_j), sum h s
    double ss = 0.0, qf = 0.0, hs = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j = t + DMH_THREADS * r;
      const double sv = (double)s[r];
      const double kd = (j < N) ? K[(int64_t)j * Np + j] : 0.0;
      ss += sv;
      qf += sv * f[r] + kd * (sv * sv);
      hs += hv[r] * sv;
    }
    ss = dmh_block_sum(ss, sh);
    qf = dmh_block_sum(qf, sh);
    hs = dmh_block_sum(hs, sh);
    if (t == 0) {
      double* o = rec + ((int64_t)c * n_sweeps + ts) * 3;
      o[0] = ss;
      o[1] = qf;
      o[2] = hs;
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = t + DMH_THREADS * r;
    if (j < N) spins[(int64_t)c * N + j] = (int8_t)s[r];
  }
  // accepted flips of the chain
  const double a = dmh_block_sum((double)acc, sh);
  if (t == 0) n_acc[c] = (unsigned long long)a;
}

template <int R>
static void launch_dense_mh(int n_chains, hipStream_t st, const DenseMhParams& q, const double* K, const double* h,
                            const int8_t* s0, int8_t* s, int n_sweeps, double* rec, unsigned long long* n_acc) {
  k_dense_mh<R><<<n_chains, DMH_THREADS, 0, st>>>(q, K, h, s0, s, n_sweeps, rec, n_acc);
}

}  // namespace ihmc

using namespace ihmc;

extern "C" int ihmc_mh_run(ihmc_ctx* ctx, const ihmc_lattice* lat, int32_t n_sweeps, uint64_t seed, uint64_t chain_id,
                           const int8_t* spins0, double* m, double* beta_eps, int8_t* spins_final, double* stats) {
  CTX_OK(ctx);
  if (!lat) return set_error(IHMC_E_INVAL, "lat is NULL");
  if (lat->ndim != 2 && lat->ndim != 3) return set_error(IHMC_E_INVAL, "ndim must be 2 or 3");
  for (int d = 0; d < lat->ndim; ++d)
    if (lat->L[d] < 2 || lat->L[d] % 2 || lat->L[d] > (1 << 20))
      return set_error(IHMC_E_INVAL, "checkerboard sweeps need even extents in [2, 2^20]");
  if (lat->h_len != 0 && lat->h_len != 1)
    return set_error(IHMC_E_UNSUPPORTED, "Metropolis-Hastings takes h = 0 or a uniform field");
  if (lat->h_len == 1 && !lat->h) return set_error(IHMC_E_INVAL, "h is NULL");
  if (!(lat->beta >= 0.0) || !std::isfinite(lat->beta * lat->J))
    return set_error(IHMC_E_INVAL, "beta must be >= 0 and beta*J finite");
  if (n_sweeps < 0) return set_error(IHMC_E_INVAL, "n_sweeps must be >= 0");
  MhParams q;
  std::memset(&q, 0, sizeof q);
  q.ndim = lat->ndim;
  q.L0 = lat->L[0];
  q.L1 = lat->L[1];
  q.L2 = lat->ndim == 3 ? lat->L[2] : 1;
  q.N = (int64_t)q.L0 * q.L1 * q.L2;
  if (q.N >= (int64_t(1) << 32)) return set_error(IHMC_E_INVAL, "too many sites");
  q.seed_lo = (uint32_t)seed;
  q.seed_hi = (uint32_t)(seed >> 32);
  q.chain = (uint32_t)chain_id;
  q.J = lat->J;
  q.h = lat->h_len ? lat->h[0] : 0.0;
  for (int sp = 0; sp < 2; ++sp)
    for (int sum = -2 * q.ndim; sum <= 2 * q.ndim; ++sum) {
      const int si = sp ? 1 : -1;
      const double dE = 2.0 * si * (q.J * sum + q.h);
      q.p[sp][sum + 2 * q.ndim] = std::exp(-lat->beta * dE);
    }
  hipStream_t s = ctx->stream;
  const uint64_t nacc = 2 * (uint64_t)std::max(1, n_sweeps);
  // a fixed grid of at most 2048 workgroups per half-sweep (eight waves per
  // SIMD), so the one-block reduction reads at most 3 x 4096 partials
  const unsigned nb_all = (unsigned)((q.N + 255) / 256);
  const unsigned nh = std::min((unsigned)((q.N / 2 + 255) / 256), 2048u);
  const uint64_t parts = 8 * 3 * 2 * (uint64_t)nh;
  char* blk = (char*)ctx->arena.alloc(8 * nacc + 256 + parts + (uint64_t)q.N + (spins0 ? (uint64_t)q.N : 0) + 256);
  if (!blk) return set_error(IHMC_E_NOMEM, "arena exhausted");
  long long* acc = (long long*)blk;
  int* sweep = (int*)(blk + 8 * nacc);
  unsigned long long* n_acc = (unsigned long long*)(blk + 8 * nacc + 64);
  long long* part = (long long*)(blk + 8 * nacc + 256);
  int8_t* spins = (int8_t*)(blk + 8 * nacc + 256 + parts);
  int8_t* d_s0 = spins0 ? spins + q.N : nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipError_t e = hipSuccess;
  if (d_s0) e = hipMemcpyAsync(d_s0, spins0, (size_t)q.N, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    k_mh_clear<<<(unsigned)((nacc + 255) / 256), 256, 0, s>>>(acc, (int64_t)nacc, sweep, n_acc);
    k_mh_init<<<nb_all, 256, 0, s>>>(q, spins, d_s0);
    e = hipGetLastError();
  }
  if (e == hipSuccess && n_sweeps > 0) {
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      k_mh_half<<<nh, 256, 0, s>>>(q, spins, sweep, 0, part);
      k_mh_half<<<nh, 256, 0, s>>>(q, spins, sweep, 1, part + 3 * (uint64_t)nh);
      k_mh_reduce<<<1, 1024, 0, s>>>(part, (int)nh, sweep, acc, n_acc);
      hipError_t e2 = hipStreamEndCapture(s, &graph);
      e = e2 != hipSuccess ? e2 : hipGetLastError();
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int t = 0; e == hipSuccess && t < n_sweeps; ++t) e = hipGraphLaunch(gexec, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
  }
  std::vector<long long> h_acc(nacc);
  unsigned long long h_nacc = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(h_acc.data(), acc, 8 * nacc, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&h_nacc, n_acc, 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && spins_final) e = hipMemcpyAsync(spins_final, spins, (size_t)q.N, hipMemcpyDeviceToHost, s);
  hipError_t es = hipStreamSynchronize(s);
  float ms = 0.f;
  if (e == hipSuccess && es == hipSuccess && e0) e = hipEventElapsedTime(&ms, e0, e1);
  if (gexec) hipGraphExecDestroy(gexec);
  if (graph) hipGraphDestroy(graph);
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  ctx->arena.release(blk);
  if (e != hipSuccess) return hip_fail(ctx, e, "Metropolis-Hastings");
  if (es != hipSuccess) return hip_fail(ctx, es, "Metropolis-Hastings sync");
  for (int t = 0; t < n_sweeps; ++t) {
    const double ssum = (double)h_acc[2 * t], bsum = (double)h_acc[2 * t + 1];
    if (m) m[t] = ssum / (double)q.N;
    if (beta_eps) beta_eps[t] = lat->beta * (-q.J * bsum - q.h * ssum) / (double)q.N;
  }
  if (stats) {
    stats[0] = n_sweeps ? (double)h_nacc / ((double)q.N * n_sweeps) : 0.0;
    stats[1] = 1e-3 * (double)ms;
  }
  return IHMC_OK;
}

extern "C" int ihmc_dense_mh_run(ihmc_ctx* ctx, const ihmc_dense* model, int32_t n_chains, int32_t n_sweeps,
                                 uint64_t seed, uint64_t chain_id, const int8_t* spins0, double* m, double* beta_eps,
                                 int8_t* spins_final, double* acceptance, double* seconds) {
  CTX_OK(ctx);
  if (!model) return set_error(IHMC_E_INVAL, "model is NULL");
  const int64_t N = model->N;
  if (N < 1 || N > 4096) return set_error(IHMC_E_INVAL, "dense Metropolis-Hastings: N must be in [1, 4096]");
  if (!model->K) return set_error(IHMC_E_INVAL, "dense: K is NULL");
  if (n_chains < 1 || n_chains > 65535) return set_error(IHMC_E_INVAL, "n_chains must be in [1, 65535]");
  if (n_sweeps < 0) return set_error(IHMC_E_INVAL, "n_sweeps must be >= 0");
  if (!(model->beta >= 0.0) || !std::isfinite(model->beta) || !std::isfinite(model->J))
    return set_error(IHMC_E_INVAL, "beta must be finite and >= 0, J finite");
  if (!(model->h_len == 0 || model->h_len == 1 || model->h_len == N))
    return set_error(IHMC_E_INVAL, "dense: h_len must be 0, 1 or N");
  if (model->h_len > 0 && !model->h) return set_error(IHMC_E_INVAL, "dense: h is NULL");
  for (int64_t i = 0; i < model->h_len; ++i)
    if (!std::isfinite(model->h[i])) return set_error(IHMC_E_INVAL, "dense: h[%lld] is not finite", (long long)i);
  for (int64_t i = 0; i < N * N; ++i)
    if (!std::isfinite(model->K[i])) return set_error(IHMC_E_INVAL, "dense: K has a non-finite entry");
  // the fields are updated from rows of K in place of its columns
  for (int64_t i = 0; i < N; ++i)
    for (int64_t k = i + 1; k < N; ++k)
      if (model->K[i * N + k] != model->K[k * N + i])
        return set_error(IHMC_E_INVAL, "dense Metropolis-Hastings: K must be exactly symmetric (entry %lld, %lld)",
                         (long long)i, (long long)k);
  // sites per thread
  const int R = N <= DMH_THREADS ? 1 : N <= 2 * DMH_THREADS ? 2 : N <= 4 * DMH_THREADS ? 4 : 8;
  DenseMhParams q;
  std::memset(&q, 0, sizeof q);
  q.N = (int32_t)N;
  q.Np = R * DMH_THREADS;
  q.h_kind = model->h_len == 0 ? 0 : (model->h_len == 1 ? 1 : 2);
  q.seed_lo = (uint32_t)seed;
  q.seed_hi = (uint32_t)(seed >> 32);
  q.chain0 = (uint32_t)chain_id;
  q.J = model->J;
  q.beta = model->beta;
  q.h0 = model->h_len == 1 ? model->h[0] : 0.0;
  // rows padded with zeros to whole 64-site blocks (the diagonal blocks staged)
  const uint64_t krows = (uint64_t)((N + DMH_BLK - 1) / DMH_BLK) * DMH_BLK;
  const uint64_t kbytes = 8ull * krows * (uint64_t)q.Np;
  const uint64_t hbytes = q.h_kind == 2 ? 8ull * (uint64_t)N : 0;
  const uint64_t sbytes = (uint64_t)n_chains * (uint64_t)N;
  const uint64_t rbytes = 24ull * (uint64_t)n_chains * (uint64_t)std::max(1, n_sweeps);
  const uint64_t abytes = 8ull * (uint64_t)n_chains;
  auto up = [](uint64_t b) { return (b + 255) & ~uint64_t(255); };
  const uint64_t total = up(kbytes) + up(hbytes) + 2 * up(sbytes) + up(rbytes) + up(abytes);
  char* blk = (char*)ctx->arena.alloc(total);
  if (!blk) return set_error(IHMC_E_NOMEM, "arena exhausted");
  double* dK = (double*)blk;
  double* dh = (double*)(blk + up(kbytes));
  int8_t* ds = (int8_t*)(blk + up(kbytes) + up(hbytes));
  int8_t* ds0 = spins0 ? ds + up(sbytes) : nullptr;
  double* rec = (double*)(blk + up(kbytes) + up(hbytes) + 2 * up(sbytes));
  unsigned long long* nacc = (unsigned long long*)(blk + up(kbytes) + up(hbytes) + 2 * up(sbytes) + up(rbytes));
  hipStream_t st = ctx->stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMemsetAsync(dK, 0, kbytes, st);
  // rows of K at pitch Np, zero padded
  if (e == hipSuccess)
    e = hipMemcpy2DAsync(dK, 8 * (size_t)q.Np, model->K, 8 * (size_t)N, 8 * (size_t)N, (size_t)N,
                         hipMemcpyHostToDevice, st);
  if (e == hipSuccess && hbytes) e = hipMemcpyAsync(dh, model->h, hbytes, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && ds0) e = hipMemcpyAsync(ds0, spins0, sbytes, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  if (e == hipSuccess) {
    switch (R) {
      case 1: launch_dense_mh<1>(n_chains, st, q, dK, dh, ds0, ds, n_sweeps, rec, nacc); break;
      case 2: launch_dense_mh<2>(n_chains, st, q, dK, dh, ds0, ds, n_sweeps, rec, nacc); break;
      case 4: launch_dense_mh<4>(n_chains, st, q, dK, dh, ds0, ds, n_sweeps, rec, nacc); break;
      default: launch_dense_mh<8>(n_chains, st, q, dK, dh, ds0, ds, n_sweeps, rec, nacc); break;
    }
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  std::vector<double> h_rec(3 * (size_t)n_chains * (size_t)std::max(0, n_sweeps));
  std::vector<unsigned long long> h_acc((size_t)n_chains);
  if (e == hipSuccess && !h_rec.empty())
    e = hipMemcpyAsync(h_rec.data(), rec, 8 * h_rec.size(), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(h_acc.data(), nacc, 8 * h_acc.size(), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && spins_final) e = hipMemcpyAsync(spins_final, ds, sbytes, hipMemcpyDeviceToHost, st);
  hipError_t es = hipStreamSynchronize(st);
  float ms = 0.f;
  if (e == hipSuccess && es == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  ctx->arena.release(blk);
  if (e != hipSuccess) return hip_fail(ctx, e, "dense Metropolis-Hastings");
  if (es != hipSuccess) return hip_fail(ctx, es, "dense Metropolis-Hastings sync");
  for (int32_t c = 0; c < n_chains; ++c) {
    for (int32_t t = 0; t < n_sweeps; ++t) {
      const double* o = &h_rec[3 * ((size_t)c * n_sweeps + t)];
      if (m) m[(size_t)c * n_sweeps + t] = o[0] / (double)N;
      if (beta_eps) beta_eps[(size_t)c * n_sweeps + t] = q.beta * (-0.5 * q.J * o[1] - o[2]) / (double)N;
    }
    if (acceptance) acceptance[c] = n_sweeps ? (double)h_acc[c] / ((double)N * n_sweeps) : 0.0;
  }
  if (seconds) *seconds = 1e-3 * (double)ms;
  return IHMC_OK;
}
