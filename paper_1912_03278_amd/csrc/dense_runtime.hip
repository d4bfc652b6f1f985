// Runtime of the dense-coupling chains: set-up (K's limbs, Lanczos shift, CG
// constants), the per-trajectory launch sequence, and its C ABI.
//
// All chains of one object share the coupling matrix; their fields form the
// columns of one N x B matrix, so every K~ application of a force evaluation
// is one GEMM over all chains (Sec. 3's force F = K~ (sqrt(J') tanh(sqrt(J')
// K~ psi) - psi) + h'/sqrt(J') applied column by column).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "dense_kernels.hpp"
#include "runtime_internal.hpp"

using namespace ihmc;

namespace ihmc {

static inline int64_t round_up(int64_t a, int64_t m) { return (a + m - 1) / m * m; }

// Lowest eigenvalue of the symmetric tridiagonal T (diagonal a[0..m), off-
// diagonal b[0..m-1)) by Sturm-count bisection, and the last component of its
// normalised eigenvector by inverse iteration with the LDL^T factors of the
// positive definite T - sigma 1, sigma just below theta.  (Back-substitution
// from the top-down factors of T - theta 1 alone is unreliable exactly when the
// Ritz pair has converged, i.e. when that last component is tiny.)
static void tridiag_min(const std::vector<double>& a, const std::vector<double>& b, int m, double* theta,
                        double* last) {
  double lo = a[0], hi = a[0];
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  auto count_below = [&](double x) {  // eigenvalues < x
    int c = 0;
    double d = 1.0;
    for (int i = 0; i < m; ++i) {
      const double off = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
      d = (a[i] - x) - (i > 0 ? off / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0.0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200 && hi - lo > 0.0; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (count_below(mid) >= 1) hi = mid;
    else lo = mid;
  }
  const double th = lo;  // no eigenvalue below lo
  const double sigma = th - 1e-9 * (std::fabs(th) + 1.0);
  std::vector<double> d(m), l(m > 1 ? m - 1 : 1), x(m, 1.0);
  d[0] = a[0] - sigma;
  for (int i = 1; i < m; ++i) {
    l[i - 1] = b[i - 1] / d[i - 1];
    d[i] = (a[i] - sigma) - l[i - 1] * b[i - 1];
  }
  for (int it = 0; it < 3; ++it) {
    for (int i = 1; i < m; ++i) x[i] -= l[i - 1] * x[i - 1];  // L y = x
    for (int i = 0; i < m; ++i) x[i] /= d[i];                 // D z = y
    for (int i = m - 2; i >= 0; --i) x[i] -= l[i] * x[i + 1];  // L^T s = z
    double nrm = 0.0;
    for (int i = 0; i < m; ++i) nrm += x[i] * x[i];
    nrm = std::sqrt(nrm);
    for (int i = 0; i < m; ++i) x[i] /= nrm;
  }
  *theta = th;
  *last = std::fabs(x[m - 1]);
}

// FP64 Lanczos on the padded device matrix K64 (zero shift), with full
// reorthogonalisation.  Stops when the Ritz residual |r| = beta_m |s_m| of the
// lowest Ritz value falls below 1e-10 (|theta| + 1), at an invariant subspace,
// or after min(N, kLanczosMaxSteps) steps.
static int lanczos_min(ihmc_ctx* ctx, const double* K64, int64_t N, int64_t Np, double* theta, double* resid,
                       int* steps) {
  hipStream_t s = ctx->stream;
  const int mmax = (int)std::min<int64_t>(N, kLanczosMaxSteps);
  double* Q = (double*)ctx->arena.alloc(8 * (uint64_t)Np * (mmax + 1));
  double* w = (double*)ctx->arena.alloc(8 * (uint64_t)Np);
  double* ab = (double*)ctx->arena.alloc(8 * 2 * (uint64_t)(mmax + 1));
  auto release = [&]() {
    hipStreamSynchronize(s);
    if (Q) ctx->arena.release(Q);
    if (w) ctx->arena.release(w);
    if (ab) ctx->arena.release(ab);
  };
  if (!Q || !w || !ab) {
    release();
    return set_error(IHMC_E_NOMEM, "arena exhausted (Lanczos basis of %d vectors)", mmax + 1);
  }
  hipError_t e = lanczos_start(Q, N, Np, s);
  std::vector<double> a(mmax + 1), b(mmax + 1);
  int m = 0;
  double th = 0.0, res = 0.0;
  const int chunk = 16;
  while (e == hipSuccess && m < mmax) {
    const int m_end = std::min(mmax, m + chunk);
    for (int k = m; k < m_end && e == hipSuccess; ++k) {
      e = dense_gemv(K64, Np, 0.0, Q + (int64_t)k * Np, w, nullptr, s);
      if (e == hipSuccess) e = lanczos_orth(Q, k, w, ab, ab + (mmax + 1), Np, s);
    }
    if (e != hipSuccess) break;
    if ((e = hipMemcpyAsync(a.data(), ab, 8 * (size_t)m_end, hipMemcpyDeviceToHost, s)) != hipSuccess) break;
    if ((e = hipMemcpyAsync(b.data(), ab + (mmax + 1), 8 * (size_t)m_end, hipMemcpyDeviceToHost, s)) != hipSuccess)
      break;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
    m = m_end;
    double last = 0.0;
    tridiag_min(a, b, m, &th, &last);
    res = std::fabs(b[m - 1]) * last;
    bool breakdown = false;
    for (int k = 0; k < m; ++k)
      if (!(b[k] > 1e-14 * (std::fabs(a[k]) + 1.0))) {
        // invariant subspace after step k: the Ritz values of T_{k+1} are exact
        breakdown = true;
        tridiag_min(a, b, k + 1, &th, &last);
        res = 0.0;
        m = k + 1;
        break;
      }
    if (breakdown || res <= 1e-10 * (std::fabs(th) + 1.0)) break;
  }
  release();
  if (e != hipSuccess) return hip_fail(ctx, e, "Lanczos");
  if (!std::isfinite(th) || !std::isfinite(res)) return set_error(IHMC_E_INVAL, "K: Lanczos did not converge");
  *theta = th;
  *resid = res;
  *steps = m;
  return IHMC_OK;
}

// x = Kt^-1 rhs by CG on the device (FP64; relative residual 1e-13, or at
// least 1e-9 when the iteration limit is reached first).
static int cg_solve(ihmc_ctx* ctx, const double* K64, int64_t N, int64_t Np, double C, const double* rhs, double* x,
                    double* work, int* iters) {
  hipStream_t s = ctx->stream;
  double *r = work, *d = work + Np, *q = work + 2 * Np, *scal = work + 3 * Np;
  int* it = (int*)(scal + 4);
  HIPCHK(cg_init(rhs, Np, 1e-13, x, r, d, scal, it, s), "CG init");
  const int max_it = (int)std::min<int64_t>(20000, 20 * N + 100);
  int host_it[2] = {0, 0};
  for (int done = 0; done < max_it; done += 32) {
    for (int k = 0; k < 32; ++k) {
      HIPCHK(dense_gemv(K64, Np, C, d, q, it + 1, s), "CG product");
      HIPCHK(cg_step(q, Np, x, r, d, scal, it, s), "CG step");
    }
    HIPCHK(hipMemcpyAsync(host_it, it, sizeof host_it, hipMemcpyDeviceToHost, s), "CG status");
    HIPCHK(hipStreamSynchronize(s), "CG sync");
    if (host_it[1]) break;
  }
  *iters = host_it[0];
  if (host_it[1] == 2) return set_error(IHMC_E_INVAL, "dense: K + C*1 is not positive definite (CG curvature <= 0)");
  if (host_it[1] == 0) {
    double sc[3];
    HIPCHK(hipMemcpy(sc, scal, sizeof sc, hipMemcpyDeviceToHost), "CG residual");
    if (!(sc[0] <= 1e-18 * sc[2]))
      return set_error(IHMC_E_INVAL, "dense: CG on K + C*1 did not converge in %d steps", max_it);
  }
  return IHMC_OK;
}

struct DenseChains {
  ihmc_ctx* ctx = nullptr;
  int B = 0;
  int64_t N = 0, Np = 0, Bp = 0;
  int S = 1, nprod = 6, n_pass = 0;
  std::vector<ChainDev> cd;
  ChainDev* d_cd = nullptr;
  double* K64 = nullptr;
  __bf16* Kl = nullptr;
  __bf16* Xl = nullptr;
  __bf16* Wl = nullptr;
  float* W32 = nullptr;
  float* part = nullptr;
  double* U64 = nullptr;
  double* hp = nullptr;
  float* bfield = nullptr;
  double C = 0.0, theta = 0.0, resid = 0.0;
  int lanczos_steps = 0, cg_iters = 0;
  std::vector<void*> allocs;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int enqueued = 0;
  std::vector<int> base;  // per chain: trajectory index at enqueued = 0 (non-zero after a restore)

  void* dalloc(uint64_t bytes) {
    void* p = ctx->arena.alloc(bytes);
    if (p) allocs.push_back(p);
    return p;
  }
  ~DenseChains() {
    if (gexec) hipGraphExecDestroy(gexec);
    if (graph) hipGraphDestroy(graph);
    for (void* p : allocs) ctx->arena.release(p);
  }
  int build(const ihmc_dense& md, int32_t n, const ihmc_run* runs, int32_t products);
  hipError_t enqueue_force(int mode, int j, hipStream_t s);
  hipError_t enqueue_round(hipStream_t s);
  int advance(int32_t n_traj);
};

static int validate_dense(const ihmc_dense& m) {
  if (m.N < 1) return set_error(IHMC_E_INVAL, "dense: N must be >= 1");
  if (!m.K) return set_error(IHMC_E_INVAL, "dense: K is NULL");
  if (!(m.beta * m.J > 0.0) || !std::isfinite(m.beta * m.J))
    return set_error(IHMC_E_INVAL, "dense: J' = beta*J must be finite and > 0");
  if (!std::isfinite(m.C)) return set_error(IHMC_E_INVAL, "dense: C must be finite (C < 0 selects the shift)");
  if (!(m.h_len == 0 || m.h_len == 1 || m.h_len == m.N))
    return set_error(IHMC_E_INVAL, "dense: h_len must be 0, 1 or N");
  if (m.h_len > 0 && !m.h) return set_error(IHMC_E_INVAL, "dense: h is NULL");
  for (int64_t i = 0; i < m.h_len; ++i)
    if (!std::isfinite(m.h[i])) return set_error(IHMC_E_INVAL, "dense: h[%lld] is not finite", (long long)i);
  const int64_t N = m.N;
  double kmax = 0.0;
  for (int64_t i = 0; i < N * N; ++i) {
    if (!std::isfinite(m.K[i])) return set_error(IHMC_E_INVAL, "dense: K has a non-finite entry");
    kmax = std::max(kmax, std::fabs(m.K[i]));
  }
  for (int64_t i = 0; i < N; ++i)
    for (int64_t k = i + 1; k < N; ++k)
      if (std::fabs(m.K[i * N + k] - m.K[k * N + i]) > 1e-12 * kmax)
        return set_error(IHMC_E_INVAL, "dense: K is not symmetric (entry %lld, %lld)", (long long)i, (long long)k);
  return IHMC_OK;
}

int DenseChains::build(const ihmc_dense& md, int32_t n, const ihmc_run* runs, int32_t products) {
  int rc = validate_dense(md);
  if (rc) return rc;
  if (products == 0) products = 6;
  if (products != 3 && products != 6) return set_error(IHMC_E_INVAL, "products must be 3 or 6");
  nprod = products;
  B = n;
  N = md.N;
  Np = round_up(N, 256);
  Bp = round_up(B, 128);
  const ihmc_run& r0 = runs[0];
  bool field_nonzero = false;
  for (int64_t k = 0; k < md.h_len && !field_nonzero; ++k) field_nonzero = md.h[k] != 0.0;
  for (int i = 0; i < n; ++i) {
    const ihmc_run& r = runs[i];
    if (r.n_md < 1) return set_error(IHMC_E_INVAL, "chain %d: n_md must be >= 1", i);
    if (r.n_traj < 0) return set_error(IHMC_E_INVAL, "chain %d: n_traj must be >= 0", i);
    if (!(r.traj_len > 0.0) || !std::isfinite(r.traj_len))
      return set_error(IHMC_E_INVAL, "chain %d: traj_len must be finite and > 0", i);
    if (r.integrator != LEAPFROG && r.integrator != OMELYAN)
      return set_error(IHMC_E_INVAL, "chain %d: unknown integrator %d", i, r.integrator);
    if (r.flip_every < 0) return set_error(IHMC_E_INVAL, "chain %d: flip_every must be >= 0", i);
    if (r.n_therm < 0) return set_error(IHMC_E_INVAL, "chain %d: n_therm must be >= 0", i);
    if (r.precision != IHMC_F32)
      return set_error(IHMC_E_UNSUPPORTED, "chain %d: dense chains keep FP32 state (precision 4)", i);
    if (r.form != FORM_PSI && r.form != FORM_SHIFTED)
      return set_error(IHMC_E_UNSUPPORTED, "chain %d: dense chains run the psi or the shifted form", i);
    if (r.form == FORM_SHIFTED && r.flip_every > 0 && field_nonzero)
      return set_error(IHMC_E_INVAL, "chain %d: psi -> -psi is no symmetry of the shifted form at h != 0", i);
    if (r.n_md != r0.n_md || r.integrator != r0.integrator || r.traj_len != r0.traj_len)
      return set_error(IHMC_E_INVAL, "chain %d: n_md, integrator and traj_len must agree across dense chains", i);
  }
  n_pass = r0.integrator == OMELYAN ? 2 * r0.n_md + 1 : r0.n_md + 1;
  // Split-K factor from the site count alone (so a chain's sums, and hence its
  // trajectory, do not depend on how many chains share the launch): about 128
  // workgroups per 128 chains, at most 4 slices.
  S = 1;
  while ((Np / 128) * S < 128 && S < 4) S *= 2;

  hipStream_t s = ctx->stream;
  std::vector<void*> temps;
  auto tmp_alloc = [&](uint64_t bytes) {
    void* p = ctx->arena.alloc(bytes);
    if (p) temps.push_back(p);
    return p;
  };
  auto cleanup = [&]() {
    hipStreamSynchronize(s);
    for (void* p : temps) ctx->arena.release(p);
    temps.clear();
  };
  auto nomem = [&](const char* what) {
    cleanup();
    return set_error(IHMC_E_NOMEM, "arena exhausted (%s; %llu of %llu bytes in use)", what,
                     (unsigned long long)ctx->arena.used, (unsigned long long)ctx->arena.size);
  };

  // ---- K: FP64 padded copy and BF16 limbs
  K64 = (double*)dalloc(8 * (uint64_t)(Np * Np));
  Kl = (__bf16*)dalloc(2 * 3 * (uint64_t)(Np * Np));
  Xl = (__bf16*)dalloc(2 * 3 * (uint64_t)(Bp * Np));
  Wl = (__bf16*)dalloc(2 * 3 * (uint64_t)(Bp * Np));
  W32 = (float*)dalloc(4 * (uint64_t)(Bp * Np));
  part = (float*)dalloc(4 * (uint64_t)S * (uint64_t)(Bp * Np));
  U64 = (double*)dalloc(8 * (uint64_t)B * (uint64_t)Np);
  if (!K64 || !Kl || !Xl || !Wl || !W32 || !part || !U64) return nomem("dense operands");
  HIPCHK(hipMemsetAsync(Xl, 0, 2 * 3 * (size_t)(Bp * Np), s), "clear limbs");
  HIPCHK(hipMemsetAsync(Wl, 0, 2 * 3 * (size_t)(Bp * Np), s), "clear limbs");
  {
    double* Kh = (double*)tmp_alloc(8 * (uint64_t)(N * N));
    if (!Kh) return nomem("K staging");
    HIPCHK(hipMemcpyAsync(Kh, md.K, 8 * (size_t)(N * N), hipMemcpyHostToDevice, s), "K upload");
    HIPCHK(dense_split_K(Kh, N, Np, Kl, K64, s), "K limbs");
  }

  // ---- shift: Lanczos for the lowest eigenvalue of K
  rc = lanczos_min(ctx, K64, N, Np, &theta, &resid, &lanczos_steps);
  if (rc) {
    cleanup();
    return rc;
  }
  if (md.C < 0.0) {
    C = -(theta - resid) + 0.1;
  } else {
    C = md.C;
    if (!(theta + C > 0.0)) {
      cleanup();
      return set_error(IHMC_E_INVAL, "dense: K + C*1 is not positive definite (lowest Ritz value %.6g, C = %.6g)",
                       theta, C);
    }
  }

  // ---- per-chain descriptors
  const double Jp = md.beta * md.J, sqJ = std::sqrt(Jp);
  const int h_kind = md.h_len == 0 ? 0 : (md.h_len == 1 ? 1 : 2);
  if (h_kind == 2) {
    hp = (double*)dalloc(8 * (uint64_t)Np);
    bfield = (float*)dalloc(4 * (uint64_t)Np);
    double* ht = (double*)tmp_alloc(8 * (uint64_t)N);
    if (!hp || !bfield || !ht) return nomem("field");
    HIPCHK(hipMemcpyAsync(ht, md.h, 8 * (size_t)N, hipMemcpyHostToDevice, s), "h upload");
    HIPCHK(dense_field(ht, N, Np, md.beta, sqJ, hp, bfield, s), "field");
  }
  cd.resize(B);
  base.assign(B, 0);
  for (int i = 0; i < B; ++i) {
    const ihmc_run& r = runs[i];
    ChainDev& c = cd[i];
    std::memset(&c, 0, sizeof c);
    c.ndim = 0;
    c.L0 = (int32_t)N;
    c.L1 = 1;
    c.L2 = 1;
    c.N = N;
    c.pitch = (int32_t)Np;
    c.NP = Np;
    c.n_pass = n_pass;
    c.integrator = r.integrator;
    c.flip_every = r.flip_every;
    c.h_kind = h_kind;
    c.chain_id = (uint32_t)r.chain_id;
    c.n_tiles = (uint32_t)(Np / 256);
    c.seed_lo = (uint32_t)r.seed;
    c.seed_hi = (uint32_t)(r.seed >> 32);
    c.C = C;
    c.Jp = Jp;
    c.sqJ = sqJ;
    c.hp0 = h_kind == 1 ? md.beta * md.h[0] : 0.0;
    c.b0 = h_kind == 1 ? c.hp0 / sqJ : 0.0;
    c.form = r.form;
    if (r.form == FORM_SHIFTED) {  // h' inside the log cosh, no linear term
      c.hw = c.hp0;
      c.b0 = 0.0;
    }
    c.eps = r.traj_len / r.n_md;
    c.cap = r.n_traj;
    c.n_therm = r.n_therm;
    c.precision = IHMC_F32;
    c.psi = dalloc(4 * 3 * (uint64_t)Np);
    c.p = dalloc(4 * (uint64_t)Np);
    c.rec = (TrajRecord*)dalloc(sizeof(TrajRecord) * (uint64_t)std::max(1, r.n_traj));
    c.st = (ChainState*)dalloc(sizeof(ChainState));
    void* pblk = dalloc(partials_bytes(c.n_tiles));
    c.b = bfield;
    c.hp = hp;
    if (!c.psi || !c.p || !c.rec || !c.st || !pblk) return nomem("chain state");
    HIPCHK(setup_partials(c, pblk, s), "partials");
    HIPCHK(hipMemsetAsync(c.psi, 0, 4 * 3 * (size_t)Np, s), "clear psi");
    HIPCHK(hipMemsetAsync(c.p, 0, 4 * (size_t)Np, s), "clear p");
    if (r.replay_accept && r.n_traj > 0) {
      uint8_t* d = (uint8_t*)dalloc((uint64_t)r.n_traj);
      if (!d) return nomem("replay");
      HIPCHK(hipMemcpyAsync(d, r.replay_accept, (size_t)r.n_traj, hipMemcpyHostToDevice, s), "replay upload");
      c.replay = d;
    }
    HIPCHK(launch_zero_state(c.st, s), "state");
  }

  // ---- estimator constants: g = Kt^-1 1, and Kt^-1 h' for a per-site field
  {
    double* work = (double*)tmp_alloc(8 * (uint64_t)(4 * Np + 8));
    double* ones = (double*)tmp_alloc(8 * (uint64_t)Np);
    double* g = (double*)tmp_alloc(8 * (uint64_t)Np);
    double* xh = (double*)tmp_alloc(8 * (uint64_t)Np);
    double* dots = (double*)tmp_alloc(8 * 4);
    if (!work || !ones || !g || !xh || !dots) return nomem("CG work space");
    HIPCHK(dense_fill(ones, N, Np, 1.0, s), "ones");
    int it1 = 0, it2 = 0;
    rc = cg_solve(ctx, K64, N, Np, C, ones, g, work, &it1);
    if (rc) {
      cleanup();
      return rc;
    }
    HIPCHK(dense_dot(ones, g, Np, dots, s), "dot");
    if (h_kind == 2) {
      rc = cg_solve(ctx, K64, N, Np, C, hp, xh, work, &it2);
      if (rc) {
        cleanup();
        return rc;
      }
      HIPCHK(dense_dot(hp, g, Np, dots + 1, s), "dot");
      HIPCHK(dense_dot(hp, xh, Np, dots + 2, s), "dot");
    }
    double hd[4] = {0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(hd, dots, sizeof hd, hipMemcpyDeviceToHost, s), "constants");
    HIPCHK(hipStreamSynchronize(s), "constants sync");
    cg_iters = std::max(it1, it2);
    for (int i = 0; i < B; ++i) {
      ChainDev& c = cd[i];
      c.c_v = hd[0];
      if (h_kind == 1) {
        c.c_m = c.hp0 * hd[0];
        c.c_e = c.hp0 * c.hp0 * hd[0];
      } else if (h_kind == 2) {
        c.c_m = hd[1];
        c.c_e = hd[2];
      }
      if (c.form == FORM_SHIFTED) c.c_m = c.c_e = 0.0;  // the estimators need no Kt^-1 h' terms
    }
  }
  d_cd = (ChainDev*)dalloc(sizeof(ChainDev) * (uint64_t)B);
  if (!d_cd) return nomem("chain table");
  HIPCHK(hipMemcpyAsync(d_cd, cd.data(), sizeof(ChainDev) * (size_t)B, hipMemcpyHostToDevice, s), "chain upload");

  // ---- initial fields and their action
  for (int i = 0; i < B; ++i) {
    const double* src = nullptr;
    if (runs[i].psi0) {
      double* t = (double*)tmp_alloc(8 * (uint64_t)N);
      if (!t) return nomem("psi0 staging");
      HIPCHK(hipMemcpyAsync(t, runs[i].psi0, 8 * (size_t)N, hipMemcpyHostToDevice, s), "psi0 upload");
      src = t;
    }
    HIPCHK(launch_init_psi(d_cd, i, src, N, IHMC_F32, s), "initial field");
  }
  HIPCHK(dense_gemm_f64(K64, d_cd, 0, 1, U64, Np, B, s), "measure product");
  HIPCHK(dense_h(PASS_MEASURE, d_cd, B, Np, U64, 0, s), "measure");
  hipError_t e = hipStreamSynchronize(s);
  cleanup();
  if (e != hipSuccess) return hip_fail(ctx, e, "dense set-up");
  return IHMC_OK;
}

// One force evaluation of pass j over all chains: U = K Psi (limbs in Xl),
// w, F = K W, then the pass epilogue (kick, drift, new limbs, kinetic sums).
hipError_t DenseChains::enqueue_force(int mode, int j, hipStream_t s) {
  hipError_t e;
  if ((e = dense_gemm_bf16(nprod, Kl, Xl, part, Np, Bp, S, s)) != hipSuccess) return e;
  if ((e = dense_epi_w(d_cd, B, Np, Bp, S, part, j, W32, Wl, s)) != hipSuccess) return e;
  if ((e = dense_gemm_bf16(nprod, Kl, Wl, part, Np, Bp, S, s)) != hipSuccess) return e;
  return dense_epi_f(mode, d_cd, B, Np, Bp, S, part, W32, j, Xl, s);
}

// One trajectory of every chain: limbs of the accepted fields, n_pass force
// evaluations (FIRST draws the momenta, MIDDLE kicks and drifts, LAST kicks),
// the FP64 product for H_new, and the closing Metropolis step per chain.
hipError_t DenseChains::enqueue_round(hipStream_t s) {
  hipError_t e;
  if ((e = dense_prep(d_cd, B, Np, Bp, Xl, s)) != hipSuccess) return e;
  for (int j = 0; j < n_pass; ++j) {
    const int mode = j == 0 ? PASS_FIRST : (j == n_pass - 1 ? PASS_LAST : PASS_MIDDLE);
    if ((e = enqueue_force(mode, j, s)) != hipSuccess) return e;
  }
  if ((e = dense_gemm_f64(K64, d_cd, n_pass - 1, 0, U64, Np, B, s)) != hipSuccess) return e;
  return dense_h(PASS_LAST, d_cd, B, Np, U64, n_pass - 1, s);
}

int DenseChains::advance(int32_t n_traj) {
  if (n_traj < 0) return set_error(IHMC_E_INVAL, "n_traj must be >= 0");
  for (int i = 0; i < B; ++i)
    if (base[i] + enqueued + n_traj > cd[i].cap)
      return set_error(IHMC_E_INVAL, "chain %d: %d trajectories exceed the capacity %d", i,
                       base[i] + enqueued + n_traj, cd[i].cap);
  hipStream_t s = ctx->stream;
  if (n_traj == 0) return IHMC_OK;
  if (n_traj == 1 && !gexec) {
    HIPCHK(enqueue_round(s), "round launch");
  } else {
    if (!gexec) {
      HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
      hipError_t e = enqueue_round(s);
      hipGraph_t gr = nullptr;
      hipError_t e2 = hipStreamEndCapture(s, &gr);
      if (e != hipSuccess) return hip_fail(ctx, e, "capture round");
      if (e2 != hipSuccess) return hip_fail(ctx, e2, "end capture");
      graph = gr;
      HIPCHK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0), "graph instantiate");
    }
    for (int t = 0; t < n_traj; ++t) HIPCHK(hipGraphLaunch(gexec, s), "graph launch");
  }
  enqueued += n_traj;
  return IHMC_OK;
}

}  // namespace ihmc

struct ihmc_dense_chains {
  DenseChains impl;
};

static int make_dense(ihmc_ctx* ctx, const ihmc_dense* model, int32_t n, const ihmc_run* runs, int32_t products,
                      ihmc_dense_chains** out) {
  if (!model || !runs || n < 1) return set_error(IHMC_E_INVAL, "need a model and n >= 1 run descriptors");
  ihmc_dense_chains* c = new (std::nothrow) ihmc_dense_chains();
  if (!c) return set_error(IHMC_E_NOMEM, "host allocation failed");
  c->impl.ctx = ctx;
  int rc = c->impl.build(*model, n, runs, products);
  if (rc) {
    hipStreamSynchronize(ctx->stream);
    delete c;
    return rc;
  }
  *out = c;
  return IHMC_OK;
}

extern "C" int ihmc_dense_create(ihmc_ctx* ctx, const ihmc_dense* model, int32_t n, const ihmc_run* runs,
                                 int32_t products, ihmc_dense_chains** out) {
  CTX_OK(ctx);
  if (!out) return set_error(IHMC_E_INVAL, "out is NULL");
  *out = nullptr;
  return make_dense(ctx, model, n, runs, products, out);
}

extern "C" int ihmc_dense_advance(ihmc_dense_chains* ch, int32_t n_traj) {
  if (!ch) return set_error(IHMC_E_INVAL, "chains is NULL");
  CTX_OK(ch->impl.ctx);
  return ch->impl.advance(n_traj);
}

extern "C" int ihmc_dense_result(ihmc_dense_chains* ch, int32_t i, ihmc_result* out) {
  if (!ch) return set_error(IHMC_E_INVAL, "chains is NULL");
  CTX_OK(ch->impl.ctx);
  DenseChains& d = ch->impl;
  if (i < 0 || i >= d.B) return set_error(IHMC_E_INVAL, "chain index %d out of range", i);
  return result_from_device(d.ctx, d.cd[i], d.d_cd, i, out);
}

extern "C" int ihmc_dense_checkpoint(ihmc_dense_chains* ch, int32_t i, void* buf, uint64_t* bytes) {
  if (!ch) return set_error(IHMC_E_INVAL, "chains is NULL");
  CTX_OK(ch->impl.ctx);
  DenseChains& d = ch->impl;
  if (i < 0 || i >= d.B) return set_error(IHMC_E_INVAL, "chain index %d out of range", i);
  return chain_checkpoint(d.ctx, d.cd[i], 0x100u + (uint64_t)d.nprod, buf, bytes);
}

extern "C" int ihmc_dense_restore(ihmc_dense_chains* ch, int32_t i, const void* buf, uint64_t bytes) {
  if (!ch) return set_error(IHMC_E_INVAL, "chains is NULL");
  CTX_OK(ch->impl.ctx);
  DenseChains& d = ch->impl;
  if (i < 0 || i >= d.B) return set_error(IHMC_E_INVAL, "chain index %d out of range", i);
  int traj = 0;
  int rc = chain_restore(d.ctx, d.cd[i], 0x100u + (uint64_t)d.nprod, buf, bytes, &traj);
  if (rc) return rc;
  d.base[i] = traj - d.enqueued;
  return IHMC_OK;
}

extern "C" int ihmc_dense_info(ihmc_dense_chains* ch, double* out) {
  if (!ch || !out) return set_error(IHMC_E_INVAL, "NULL argument");
  const DenseChains& d = ch->impl;
  out[0] = d.C;
  out[1] = d.theta;
  out[2] = d.resid;
  out[3] = d.lanczos_steps;
  out[4] = d.cg_iters;
  return IHMC_OK;
}

extern "C" int ihmc_dense_time(ihmc_dense_chains* ch, int32_t what, int32_t reps, double* avg_us, int64_t* mnk_s) {
  if (!ch || !avg_us) return set_error(IHMC_E_INVAL, "NULL argument");
  ihmc_ctx* ctx = ch->impl.ctx;
  CTX_OK(ctx);
  DenseChains& d = ch->impl;
  if (what < 0 || what > 2) return set_error(IHMC_E_INVAL, "what must be 0, 1 or 2");
  if (reps < 1) return set_error(IHMC_E_INVAL, "reps must be >= 1");
  hipStream_t s = ctx->stream;
  auto launch = [&]() -> hipError_t {
    if (what == 0) return dense_gemm_bf16(d.nprod, d.Kl, d.Xl, d.part, d.Np, d.Bp, d.S, s);
    if (what == 1) return dense_gemm_f64(d.K64, d.d_cd, 0, 1, d.U64, d.Np, d.B, s);
    hipError_t e = dense_prep(d.d_cd, d.B, d.Np, d.Bp, d.Xl, s);
    return e == hipSuccess ? d.enqueue_force(PASS_FORCE, 0, s) : e;
  };
  HIPCHK(hipStreamSynchronize(s), "sync");
  HIPCHK(launch(), "warm-up");
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0), "event");
  HIPCHK(hipEventCreate(&e1), "event");
  hipError_t e = hipEventRecord(e0, s);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(ctx, e, "dense timing");
  *avg_us = 1000.0 * ms / reps;
  if (mnk_s) {
    mnk_s[0] = d.Np;
    mnk_s[1] = d.Bp;
    mnk_s[2] = d.Np;
    mnk_s[3] = d.S;
  }
  return IHMC_OK;
}

extern "C" int ihmc_dense_destroy(ihmc_dense_chains* ch) {
  if (!ch) return IHMC_OK;
  hipSetDevice(ch->impl.ctx->device);
  hipStreamSynchronize(ch->impl.ctx->stream);
  delete ch;
  return IHMC_OK;
}

extern "C" int ihmc_run_dense(ihmc_ctx* ctx, const ihmc_dense* model, int32_t n, const ihmc_run* runs,
                              int32_t products, ihmc_result* outs) {
  CTX_OK(ctx);
  if (!outs) return set_error(IHMC_E_INVAL, "outs is NULL");
  ihmc_dense_chains* c = nullptr;
  int rc = make_dense(ctx, model, n, runs, products, &c);
  if (rc) return rc;
  for (int i = 0; i < n && rc == IHMC_OK; ++i)
    if (runs[i].n_traj != runs[0].n_traj) rc = set_error(IHMC_E_INVAL, "ihmc_run_dense: runs differ in n_traj");
  if (rc == IHMC_OK) rc = c->impl.advance(runs[0].n_traj);
  for (int i = 0; i < n && rc == IHMC_OK; ++i) rc = result_from_device(ctx, c->impl.cd[i], c->impl.d_cd, i, &outs[i]);
  ihmc_dense_destroy(c);
  return rc;
}

extern "C" int ihmc_dense_force(ihmc_ctx* ctx, const ihmc_dense* model, int32_t n, const double* psi,
                                int32_t products, double* F) {
  CTX_OK(ctx);
  if (!model || !psi || !F || n < 1) return set_error(IHMC_E_INVAL, "NULL argument or n < 1");
  const int64_t N = model->N;
  std::vector<ihmc_run> runs((size_t)n);
  for (int i = 0; i < n; ++i) {
    ihmc_run& r = runs[i];
    std::memset(&r, 0, sizeof r);
    r.n_md = 1;
    r.n_traj = 0;
    r.traj_len = 1.0;
    r.precision = IHMC_F32;
    r.psi0 = psi + (int64_t)i * N;
  }
  ihmc_dense_chains* c = nullptr;
  int rc = make_dense(ctx, model, n, runs.data(), products, &c);
  if (rc) return rc;
  DenseChains& d = c->impl;
  hipStream_t s = ctx->stream;
  double* t = (double*)ctx->arena.alloc(8 * (uint64_t)N);
  hipError_t e = t ? dense_prep(d.d_cd, d.B, d.Np, d.Bp, d.Xl, s) : hipErrorOutOfMemory;
  if (e == hipSuccess) e = d.enqueue_force(PASS_FORCE, 0, s);
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    e = launch_export_field(d.d_cd, i, t, d.cd[i].p, N, IHMC_F32, s);
    if (e == hipSuccess) e = hipMemcpyAsync(F + (int64_t)i * N, t, 8 * (size_t)N, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  hipStreamSynchronize(s);
  if (t) ctx->arena.release(t);
  ihmc_dense_destroy(c);
  if (!t) return set_error(IHMC_E_NOMEM, "arena exhausted (export)");
  if (e != hipSuccess) return hip_fail(ctx, e, "dense force");
  return IHMC_OK;
}

extern "C" int ihmc_min_eig(ihmc_ctx* ctx, const double* K, int64_t N, double* theta, double* resid,
                            int32_t* steps) {
  CTX_OK(ctx);
  if (!K || N < 1 || !theta || !resid) return set_error(IHMC_E_INVAL, "NULL argument or N < 1");
  ihmc_dense m;
  std::memset(&m, 0, sizeof m);
  m.N = N;
  m.K = K;
  m.J = 1.0;
  m.beta = 1.0;
  int rc = validate_dense(m);
  if (rc) return rc;
  const int64_t Np = round_up(N, 256);
  hipStream_t s = ctx->stream;
  double* K64 = (double*)ctx->arena.alloc(8 * (uint64_t)(Np * Np));
  double* Kh = (double*)ctx->arena.alloc(8 * (uint64_t)(N * N));
  __bf16* Kl = (__bf16*)ctx->arena.alloc(2 * 3 * (uint64_t)(Np * Np));
  auto release = [&]() {
    hipStreamSynchronize(s);
    if (K64) ctx->arena.release(K64);
    if (Kh) ctx->arena.release(Kh);
    if (Kl) ctx->arena.release(Kl);
  };
  if (!K64 || !Kh || !Kl) {
    release();
    return set_error(IHMC_E_NOMEM, "arena exhausted (K)");
  }
  hipError_t e = hipMemcpyAsync(Kh, K, 8 * (size_t)(N * N), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = dense_split_K(Kh, N, Np, Kl, K64, s);
  if (e != hipSuccess) {
    release();
    return hip_fail(ctx, e, "K upload");
  }
  int st = 0;
  rc = lanczos_min(ctx, K64, N, Np, theta, resid, &st);
  release();
  if (steps) *steps = st;
  return rc;
}
