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
