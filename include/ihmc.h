/*
 * ihmc.h -- C ABI of the MI355X Hybrid Monte Carlo library for the
 * Hubbard-Stratonovich-transformed Ising model (Ostmeyer, Berkowitz, Luu,
 * Petschlies, Pittler, "The Ising Model with Hybrid Monte Carlo",
 * arXiv:1912.03278).
 *
 * The model (Sec. 2, eq. hamilton_matrix_notation) is H(s) = -1/2 J s^T K s - h.s
 * with K the periodic nearest-neighbour connectivity of a 2D or 3D hypercubic
 * lattice, or an explicit symmetric coupling matrix in place of J K.  With
 * J' = beta J, h' = beta h and the shift Kt = K + C*1 (C > n, so that J' Kt is
 * positive definite, Sec. 2 after eq. eigen_spectrum_K) the library samples the
 * auxiliary field psi with the action of eq. phi_psi_substitution,
 *     S(psi) = 1/2 psi.Kt psi - psi.h'/sqrt(J') - sum_i log cosh(sqrt(J') (Kt psi)_i),
 * by HMC (Sec. 3): N(0,1) momenta, a reversible symplectic integrator over one
 * trajectory, and a Metropolis test with min(1, exp(-dH)).  After every
 * trajectory it records the estimators of Sec. 4 (eqs. formula_for_m and
 * formula_for_e, in their general-field form).
 *
 * Conventions for every entry point:
 *   - Return IHMC_OK (0) or a negative status; never throw across the ABI.
 *     ihmc_last_error() returns a thread-local message for the last failure.
 *   - Host pointers are read during the call (or copied before it returns);
 *     the caller keeps ownership and may free them afterwards.
 *   - Output arrays are caller-owned host memory of the stated length; any
 *     output pointer may be NULL to skip it.
 *   - Device memory is owned by the context: it is carved from one arena
 *     obtained at ihmc_ctx_create (from the caller's allocator callback, or
 *     hipMalloc).  Exceeding the arena gives IHMC_E_NOMEM.
 *   - Work is enqueued on the context's HIP stream.  A context is not
 *     thread-safe unless an entry point says otherwise.
 *   - Lattice sites are numbered x + L0 (y + L1 z) (x fastest).
 */
#ifndef IHMC_H
#define IHMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IHMC_OK 0
#define IHMC_E_INVAL (-1)       /* invalid argument (message says which) */
#define IHMC_E_NOMEM (-2)       /* device arena exhausted */
#define IHMC_E_AGAIN (-3)       /* serving queue full / result not ready */
#define IHMC_E_DEVICE (-4)      /* HIP runtime error; the context stays unusable */
#define IHMC_E_CANCELLED (-5)   /* request was cancelled */
#define IHMC_E_UNSUPPORTED (-6) /* valid but not implemented (e.g. 1D lattices on the GPU) */

#define IHMC_F32 4 /* state (psi, p) in FP32; H, dH, Metropolis in FP64 */
#define IHMC_F64 8 /* state in FP64 */

#define IHMC_LEAPFROG 0 /* kick-drift-kick leap-frog (Sec. 3) */
#define IHMC_OMELYAN 1  /* second-order minimum-norm integrator, named in Sec. 3 */

/* The field a chain samples (Sec. 2): */
#define IHMC_FORM_PSI 0 /* psi of eq. phi_psi_substitution: no inverse of Kt (the hot path) */
#define IHMC_FORM_PHI 1 /* phi of eq. cosh_in_exponent: a CG solve of Kt per force evaluation;
                           the A/B baseline of the substitution (FP64 leap-frog lattice chains of
                           at most 1453 sites, 1272 with a per-site field; no flips) */
#define IHMC_FORM_SHIFTED 2 /* psi of the substitution phi = sqrt(J') Kt psi in eq. did_HS_trafo:
                           S = 1/2 psi.Kt psi - sum log cosh(sqrt(J') (Kt psi)_i + h'), no linear
                           term; the same fused passes (flips only at h = 0).  A lattice chain
                           with a per-site field runs as a paper-form chain in coordinates
                           translated by Kt^-1 h'/sqrt(J') (one CG solve at set-up; HMC with
                           unit mass commutes with translations); its results are reported in
                           its own coordinates (psi, and H offset by h'.Kt^-1 h'/(2J')).  psi differs from the paper's by the
                           constant Kt^-1 h'/sqrt(J'); the records hold the paper's estimators at
                           that translate: m = sum psi/(N sqrt(J')), beta*eps = C J'/2
                           - psi.h'/(2N sqrt(J')) - sum y tanh(y)/(2N), y = sqrt(J') Kt psi + h' */

#define IHMC_TAG_INIT 1u /* Philox stream tags (counter word 3) */
#define IHMC_TAG_MOM 2u
#define IHMC_TAG_ACC 3u
#define IHMC_TAG_FLIP 4u

typedef struct ihmc_ctx ihmc_ctx;
typedef struct ihmc_chains ihmc_chains;
typedef struct ihmc_dense_chains ihmc_dense_chains;
typedef struct ihmc_server ihmc_server;

/* Device allocator hook (e.g. PyTorch's caching allocator).  alloc returns a
 * device pointer or NULL; free releases it. */
typedef void* (*ihmc_alloc_fn)(uint64_t bytes, void* user);
typedef void (*ihmc_free_fn)(void* ptr, void* user);

/* Periodic hypercubic lattice with nearest-neighbour K (Sec. 2).
 *   ndim       2 or 3 on the GPU (1 is IHMC_E_UNSUPPORTED).
 *   L[ndim]    extents, each >= 3 (periodic neighbours must be distinct).
 *   J, beta    J' = beta*J must be > 0 (eq. def_J_prime).
 *   C          shift of K, must exceed n = 2*ndim (Sec. 2).
 *   h, h_len   host field: h_len 0 (h = 0), 1 (uniform h[0], eq. constant_h),
 *              or N (one value per site). */
typedef struct {
  int32_t ndim;
  int32_t L[3];
  double J, beta, C;
  const double* h;
  int64_t h_len;
} ihmc_lattice;

/* Explicit coupling matrix in place of the lattice's J K (Sec. 2 allows any
 * symmetric coupling; App. A's infinite-range model is one instance).
 *   N          sites, >= 1.
 *   K          host, N x N, row-major, symmetric, finite (checked).  The
 *              model's couplings are J * K.
 *   J, beta    J' = beta*J must be > 0.
 *   C          shift of K.  C >= 0: used as given, rejected when the lowest
 *              Ritz value theta of K gives theta + C <= 0 (K + C*1 then is
 *              certainly not positive definite).  C < 0: chosen as
 *              -(theta - |r|) + 0.1 from FP64 Lanczos (theta the lowest Ritz
 *              value, |r| its residual norm, so theta - |r| bounds the lowest
 *              eigenvalue from below once theta has converged to it).
 *   h, h_len   as for the lattice: 0, 1 (uniform) or N values. */
typedef struct {
  int64_t N;
  const double* K;
  double J, beta, C;
  const double* h;
  int64_t h_len;
} ihmc_dense;

/* Parameters of one chain (Sec. 3).
 *   n_md        integrator steps per trajectory (>= 1).
 *   n_traj      trajectories to record (capacity of the series, >= 0).
 *   traj_len    MD time per trajectory (> 0; the paper uses one time unit).
 *   integrator  IHMC_LEAPFROG or IHMC_OMELYAN.
 *   flip_every  > 0: propose the global sign flip psi -> -psi with its own
 *               Metropolis test after every flip_every-th trajectory (Sec. 3).
 *   precision   IHMC_F32 or IHMC_F64 (state precision).
 *   seed        64-bit Philox4x32-10 key.
 *   chain_id    counter word 2 (low 32 bits used): independent streams.
 *   psi0        host, N values, or NULL: psi0 ~ N(0,1) from the TAG_INIT stream.
 *   replay_accept host, n_traj bytes, or NULL: force the accept decisions
 *               (test hook for comparing trajectories past a point where FP32
 *               and FP64 decisions could differ).
 *   n_therm     thermalisation trajectories (>= 0; the paper leaves the length
 *               open): the summary (acceptance, mean exp(-dH), non-finite
 *               count) covers trajectories n_therm, n_therm + 1, ... only;
 *               every trajectory is still recorded in the series.  0 (a
 *               zero-initialised struct) counts them all.
 *   form        IHMC_FORM_PSI (0) or IHMC_FORM_PHI.  In the phi form, psi0 is
 *               the starting phi (NULL: phi0 = sqrt(J') Kt psi0 - h' with psi0
 *               the TAG_INIT normals, the substitution that links the forms),
 *               psi_final the final phi, and the records hold the spin
 *               expectations given phi (m = mean tanh(h' + phi), m^2 and beta*eps
 *               likewise, no bias correction needed).  IHMC_FORM_SHIFTED: psi0
 *               is the starting psi of that form (NULL: the TAG_INIT normals);
 *               flips at h != 0 give IHMC_E_INVAL; the server runs psi and
 *               shifted chains (any field), not phi ones. */
typedef struct {
  int32_t n_md;
  int32_t n_traj;
  double traj_len;
  int32_t integrator;
  int32_t flip_every;
  int32_t precision;
  int32_t n_therm;
  uint64_t seed;
  uint64_t chain_id;
  const double* psi0;
  const uint8_t* replay_accept;
  int32_t form;
  int32_t reserved;
} ihmc_run;

/* Per-chain results.  Series are indexed by trajectory; after trajectory t
 * they hold dH = H_new - H_old, the accept/flip decisions and the estimators
 * of the accepted field: m, |m|, m^2 minus its Gaussian-noise bias
 * 1^T Kt^-1 1 / (N^2 J'), and beta*eps (Sec. 4). */
typedef struct {
  double *dH, *H_old, *H_new, *m, *abs_m, *m2c, *beta_eps; /* host, n_traj each, or NULL */
  uint8_t *accepted, *flipped;                            /* host, n_traj each, or NULL */
  double* psi_final;                                      /* host, N, or NULL */
  double acceptance;        /* accepted / trajectories done */
  double mean_exp_minus_dH; /* over trajectories with finite dH */
  int64_t n_nonfinite;      /* trajectories with a non-finite or out-of-range H term */
  int64_t n_traj_done;
  int64_t cg_iterations;    /* phi form: CG iterations of the set-up and all trajectories (0 for psi) */
} ihmc_result;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device` with a device arena of arena_bytes
 * (0: 1 GiB).  alloc/free may be NULL (then hipMalloc/hipFree); `user` is
 * passed to them.  The context creates its own HIP stream (default priority). */
int ihmc_ctx_create(int32_t device, uint64_t arena_bytes, ihmc_alloc_fn alloc, ihmc_free_fn free_fn,
                    void* user, ihmc_ctx** out);
void ihmc_ctx_destroy(ihmc_ctx* ctx);
/* The context's hipStream_t. */
void* ihmc_ctx_stream(ihmc_ctx* ctx);
/* Wait for all work enqueued on the context. */
int ihmc_ctx_sync(ihmc_ctx* ctx);
/* Bytes of the arena in use / in total. */
int ihmc_ctx_memory(ihmc_ctx* ctx, uint64_t* used, uint64_t* total);
/* Small chains run whole trajectories in one workgroup with the field, the
 * momenta and w held in LDS (one launch per round, or per advance when every
 * chain of a set is resident), instead of one launch per pass.  The per-site
 * arithmetic and the grouping of the exact sums are those of the tiled
 * passes, so results are bit-identical either way.  Chains created after this
 * call with at most max_sites sites, and small enough for the LDS, run
 * resident: max_sites < 0 (the default) admits every chain that fits, 0 none.
 * *fp32_fit / *fp64_fit (may be NULL) receive the largest chains that fit
 * without a per-site field (a per-site field takes a fifth array). */
int ihmc_ctx_set_resident(ihmc_ctx* ctx, int64_t max_sites, int64_t* fp32_fit, int64_t* fp64_fit);
/* 2D chains on the tiled passes run their middle leap-frog steps two per
 * launch (on != 0, the default): the first step is evaluated on the tile plus
 * a 2-wide ring, the second on the tile, with the field read and written once
 * per pair.  The per-site arithmetic is that of one step per launch, so
 * results are bit-identical either way.  Applies to chain sets created after
 * the call, to the serving rounds that follow it, and to tuning. */
int ihmc_ctx_set_step_fusion(ihmc_ctx* ctx, int32_t on);
const char* ihmc_last_error(void);

/* ---- resident chains (the hot path) --------------------------------------- */

/* Create n independent chains, each with its own lattice and run parameters
 * (2D and 3D, FP32 and FP64 may be mixed).  Performs the set-up of every chain
 * on the device: field constants, initial field, S(psi0).  Synchronous. */
int ihmc_chains_create(ihmc_ctx* ctx, int32_t n, const ihmc_lattice* lats, const ihmc_run* runs,
                       ihmc_chains** out);
/* Enqueue n_traj further trajectories of every chain (asynchronous; repeated
 * calls continue the chains).  Fails with IHMC_E_INVAL past the capacity
 * n_traj given at creation.  Launch sequences are captured once into a HIP
 * graph and replayed. */
int ihmc_chains_advance(ihmc_chains* chains, int32_t n_traj);
/* Wait, then copy the series and summary of chain i (0 <= i < n). */
int ihmc_chains_result(ihmc_chains* chains, int32_t i, ihmc_result* out);
int ihmc_chains_destroy(ihmc_chains* chains);

/* Checkpoint and resume of chain i (0 <= i < n).  The Philox streams are
 * counter based (key = seed, counters = site pair, trajectory, chain_id,
 * purpose), so a chain's state after t trajectories is its accepted field,
 * S of that field in exact fixed point, the estimator sums, the sign, the
 * counters and the series so far; a chain restored from it continues exactly
 * (bit for bit) as the original would have.
 *
 * ihmc_chains_checkpoint waits for the chains' queued work, then writes the
 * state into the caller's host buffer `buf` of *bytes bytes.  With buf NULL it
 * only stores the size needed in *bytes.  A buffer smaller than that fails
 * with IHMC_E_INVAL (and *bytes = the size needed).  The layout is private to
 * this library version: a header with the chain's identity and state, the
 * stored field (state precision, row pitch included), then the records.
 *
 * ihmc_chains_restore waits for queued work, then replaces chain i's state
 * with the checkpoint in buf (bytes long).  Chain i must have been created
 * with the same lattice and run parameters (dimensions, precision, couplings,
 * field, C, n_md, traj_len, integrator, flip_every, seed, chain_id; n_traj may
 * be larger, and must cover the trajectories already done).  A buffer that is
 * not such a checkpoint, is truncated, or belongs to a chain with other
 * parameters fails with IHMC_E_INVAL and leaves the chain unchanged.  The
 * chain then continues at the checkpoint's trajectory index; further
 * ihmc_chains_advance calls count against its capacity from there. */
int ihmc_chains_checkpoint(ihmc_chains* chains, int32_t i, void* buf, uint64_t* bytes);
int ihmc_chains_restore(ihmc_chains* chains, int32_t i, const void* buf, uint64_t bytes);

/* One chain: create, advance run->n_traj, fetch, destroy.  Synchronous. */
int ihmc_run_lattice(ihmc_ctx* ctx, const ihmc_lattice* lat, const ihmc_run* run, ihmc_result* out);
/* n chains (arrays of n descriptors and n results).  Synchronous. */
int ihmc_run_batch(ihmc_ctx* ctx, int32_t n, const ihmc_lattice* lats, const ihmc_run* runs,
                   ihmc_result* outs);

/* ---- dense couplings (many chains of one model) ---------------------------- */

/* Create n chains of one dense model (runs[i] gives each chain's seed,
 * chain_id, psi0, replay and capacity; n_md, traj_len, integrator and
 * flip_every must agree across the chains, and precision must be IHMC_F32).
 * The fields of all chains form one N x n matrix, so both K~ applications of
 * a force evaluation are matrix products on the MFMA units.  `products`
 * selects their precision: 6 (K and the FP32 operand each held as three BF16
 * limbs, all limb products of order <= 2, ~FP32 accuracy; the default when 0)
 * or 3 (two limbs each, products of order <= 1, ~2^-16 relative).  The
 * Hamiltonian uses an FP64 product of the stored field with the FP64 K.
 * Set-up (synchronous): K's limbs, Lanczos for C (see ihmc_dense), CG solves
 * for the estimator constants 1^T Kt^-1 1, 1^T Kt^-1 h', h'^T Kt^-1 h', the
 * initial fields and S(psi0). */
int ihmc_dense_create(ihmc_ctx* ctx, const ihmc_dense* model, int32_t n, const ihmc_run* runs, int32_t products,
                      ihmc_dense_chains** out);
/* Enqueue n_traj trajectories of every chain (asynchronous, graph-replayed). */
int ihmc_dense_advance(ihmc_dense_chains* chains, int32_t n_traj);
/* Wait, then copy chain i's series and summary, as ihmc_chains_result. */
int ihmc_dense_result(ihmc_dense_chains* chains, int32_t i, ihmc_result* out);
/* Checkpoint and resume of dense chain i, as ihmc_chains_checkpoint and
 * ihmc_chains_restore (the model, the products and the run parameters of the
 * restoring chain must match; C must be the same number). */
int ihmc_dense_checkpoint(ihmc_dense_chains* chains, int32_t i, void* buf, uint64_t* bytes);
int ihmc_dense_restore(ihmc_dense_chains* chains, int32_t i, const void* buf, uint64_t bytes);
/* The shift in use and the Lanczos estimate: out[0] = C, out[1] = theta,
 * out[2] = |r|, out[3] = Lanczos steps, out[4] = CG iterations (largest of
 * the solves). */
int ihmc_dense_info(ihmc_dense_chains* chains, double* out);
/* Time one of the dense launches `reps` times after a warm-up, with HIP
 * events on the context stream: what = 0 the BF16-limb GEMM of one K~
 * application over all chains, 1 the FP64 GEMM of the Hamiltonian, 2 a whole
 * force evaluation (two GEMMs and their epilogues).  Returns microseconds per
 * launch and the GEMM dimensions (m = padded sites, n = padded chains,
 * k = padded sites) and split-K factor of the BF16 GEMM.  Overwrites the
 * momenta: call only when the results are no longer needed. */
int ihmc_dense_time(ihmc_dense_chains* chains, int32_t what, int32_t reps, double* avg_us, int64_t* mnk_s);
int ihmc_dense_destroy(ihmc_dense_chains* chains);
/* n chains of one dense model: create, advance, fetch n results, destroy. */
int ihmc_run_dense(ihmc_ctx* ctx, const ihmc_dense* model, int32_t n, const ihmc_run* runs, int32_t products,
                   ihmc_result* outs);
/* Forces of n host fields (psi: n x N, row-major) through the dense GEMM path
 * into host F (n x N). */
int ihmc_dense_force(ihmc_ctx* ctx, const ihmc_dense* model, int32_t n, const double* psi, int32_t products,
                     double* F);
/* Lowest eigenvalue of a symmetric N x N host matrix K by FP64 Lanczos with
 * full reorthogonalisation on the device: theta (lowest Ritz value, an upper
 * bound), resid (|r| of its Ritz pair; theta - resid is a lower bound once
 * theta has converged to the lowest eigenvalue) and the steps taken. */
int ihmc_min_eig(ihmc_ctx* ctx, const double* K, int64_t N, double* theta, double* resid, int32_t* steps);

/* ---- serving (continuous batching of lattice requests) --------------------- */

#define IHMC_REQ_QUEUED 0
#define IHMC_REQ_RUNNING 1
#define IHMC_REQ_DONE 2
#define IHMC_REQ_CANCELLED 3
#define IHMC_REQ_FAILED 4

/* Start a server on the context: a scheduler thread with its own HIP streams.
 * Before every round it admits queued requests in arrival order while their
 * device footprint fits budget_bytes (0: half the arena) and one of max_active
 * chain slots (0: 1024) is free; a round advances every resident chain by one
 * trajectory (the fused lattice passes of all resident chains share the
 * launches); a chain that reached its n_traj is retired: results are copied to
 * host memory and its device memory and slot go to the next request.  Results
 * are bit-identical to the same request run alone (ihmc_run_lattice). */
int ihmc_server_create(ihmc_ctx* ctx, uint64_t budget_bytes, int32_t max_active, ihmc_server** out);
/* Stop: queued requests are cancelled, running ones are retired as cancelled,
 * the scheduler is joined and every unfetched request is released. */
int ihmc_server_destroy(ihmc_server* server);
/* Queue one request (lattice and run as for ihmc_run_lattice; h, psi0 and
 * replay_accept are copied before the call returns).  Thread-safe.  Errors:
 * IHMC_E_INVAL (invalid parameters), IHMC_E_NOMEM (footprint above the
 * budget), IHMC_E_AGAIN (queue full), IHMC_E_DEVICE (server stopped by a
 * device error). */
int ihmc_submit(ihmc_server* server, const ihmc_lattice* lat, const ihmc_run* run, uint64_t* ticket);
/* State of a request (IHMC_REQ_*).  Thread-safe. */
int ihmc_poll(ihmc_server* server, uint64_t ticket, int32_t* state);
/* Block until the request has finished (done, cancelled or failed) or
 * timeout_s seconds have passed; returns its state.  Thread-safe. */
int ihmc_wait(ihmc_server* server, uint64_t ticket, double timeout_s, int32_t* state);
/* Copy a finished request's results into `out` (as ihmc_chains_result; the
 * series hold n_traj values) and release it; the ticket is invalid afterwards.
 * times (3 doubles, or NULL): submission, admission and completion, in seconds
 * since the server started.  IHMC_E_AGAIN while the request is still queued or
 * running, IHMC_E_CANCELLED for a cancelled one (the trajectories done before
 * the cancellation are still copied).  Thread-safe. */
int ihmc_fetch(ihmc_server* server, uint64_t ticket, ihmc_result* out, double* times);
/* Cancel a request: a queued one at once, a running one at the next round
 * boundary.  Thread-safe. */
int ihmc_cancel(ihmc_server* server, uint64_t ticket);
/* Checkpoint of a request, by ticket, into the caller's host buffer `buf` of
 * *bytes bytes (buf NULL: *bytes = the size needed, the largest the request
 * can take; a smaller buffer fails with IHMC_E_INVAL).  On success *bytes = the
 * bytes written.  The checkpoint holds the request (lattice, field, run
 * parameters with the form, given initial field, replayed decisions) and, once it has run,
 * its chain's state after a whole number of trajectories: the accepted field,
 * S of it in exact fixed point, the estimator sums, the sign, the counters and
 * the records.  The momenta, accept and flip uniforms of later trajectories
 * are Philox draws at counters that name the trajectory (Sec. 3 needs nothing
 * else), so a request restored from it continues bit for bit as the original.
 * A queued request gives the request alone; a running one is checkpointed by
 * the scheduler at the next round boundary (the call blocks until then; it
 * keeps running); a finished or cancelled one (not yet fetched) from its
 * retired results.  Thread-safe; must not overlap ihmc_server_destroy.  The
 * layout is private to this library version. */
int ihmc_checkpoint(ihmc_server* server, uint64_t ticket, void* buf, uint64_t* bytes);
/* Queue a request restored from a checkpoint of ihmc_checkpoint (of this or
 * another server, in this or another process) under a new ticket: it is
 * admitted like any request, set up, then given the checkpoint's state, and
 * runs its remaining trajectories; its fetched series hold all of them.
 * IHMC_E_INVAL for a buffer that is not such a checkpoint or is truncated, and
 * for a chain state that does not match its parameters.  Thread-safe. */
int ihmc_restore(ihmc_server* server, const void* buf, uint64_t bytes, uint64_t* ticket);
/* out[4]: state (IHMC_REQ_*), lattice sites, n_traj, trajectories done or
 * enqueued (the server enqueues a round while the previous one runs).
 * Thread-safe. */
int ihmc_request_info(ihmc_server* server, uint64_t ticket, int64_t* out);
/* out[10]: rounds, seconds spent in rounds, site-MD-steps done, largest
 * number of resident chains, completed requests, queued now, resident now,
 * seconds since start, device bytes held, budget. */
int ihmc_server_stats(ihmc_server* server, double* out);

/* ---- the comparison method: local Metropolis-Hastings ---------------------- */

/* n_sweeps sweeps of single-spin Metropolis-Hastings on the spins of a
 * periodic lattice (the method the paper compares HMC with, Sec. 4), on the
 * GPU.  A sweep proposes every spin once in checkerboard order (sites of even
 * parity x + y + z, then odd: independent updates, which needs every extent
 * even); flipping s_i changes the energy by dE = 2 s_i (J sum_nb s_j + h) and
 * is accepted iff dE <= 0 or u < exp(-beta dE), u the 53-bit uniform of the
 * Philox counter (site, sweep, chain_id, tag 5).  Start: spins0 (host, N int8
 * values of sign +-1) or, if NULL, s_i = +1 iff the uniform of (site, 0,
 * chain_id, tag 6) is below 1/2.  h_len must be 0 or 1 (IHMC_E_UNSUPPORTED
 * for a per-site field); C is not used.  Outputs (host, may be NULL): m and
 * beta_eps per sweep (n_sweeps each; beta*eps = beta H(s) / N), spins_final (N
 * int8), stats[0] = acceptance, stats[1] = GPU seconds of the sweeps (HIP
 * events around them).  Synchronous. */
int ihmc_mh_run(ihmc_ctx* ctx, const ihmc_lattice* lat, int32_t n_sweeps, uint64_t seed, uint64_t chain_id,
                const int8_t* spins0, double* m, double* beta_eps, int8_t* spins_final, double* stats);

/* Single-spin Metropolis-Hastings with an explicit coupling matrix (the
 * all-to-all models of Sec. 2 and App. A; Sec. 5 expects the gap between HMC
 * and local updates to shrink as every site gains neighbours), n_chains
 * independent chains on the GPU, one workgroup each.  Every spin couples to
 * every other, so a sweep proposes the spins one after another in site order
 * i = 0 .. N-1: flipping s_i changes H(s) = -1/2 J s^T K s - h.s by
 * dE = 2 s_i (J sum_{j != i} K_ij s_j + h_i), accepted iff dE <= 0 or
 * u < exp(-beta dE), u the 53-bit uniform of the Philox counter (site, sweep,
 * chain_id + c, tag 5), evaluated as dE < -ln(u) / beta.  The local fields
 * are carried from flip to flip in FP64 (not re-summed), so they differ from
 * a fresh sum by rounding only; a decision can differ from one taken with
 * exact arithmetic only where u and exp(-beta dE) agree to rounding.
 *   model       K (host, N x N row-major, exactly symmetric, finite), J, beta
 *               (finite, >= 0), h/h_len (0, 1 or N values); C is not used.
 *               1 <= N <= 4096.
 *   spins0      host, n_chains x N int8 (sign taken), or NULL: s_i = +1 iff the
 *               uniform of (site, 0, chain, tag 6) is below 1/2.
 *   m, beta_eps host, n_chains x n_sweeps each (chain-major), or NULL: after
 *               every sweep m = sum s / N and beta*eps = beta H(s) / N (the full
 *               quadratic form, diagonal included).
 *   spins_final host, n_chains x N int8, or NULL.
 *   acceptance  host, n_chains (accepted flips / (N n_sweeps)), or NULL.
 *   seconds     host, one value: GPU time of the sweeps' launch, or NULL.
 * IHMC_E_INVAL for an invalid model or sizes, IHMC_E_NOMEM when the arena
 * cannot hold K (N x N FP64, rows padded to a multiple of 512).  Synchronous. */
int ihmc_dense_mh_run(ihmc_ctx* ctx, const ihmc_dense* model, int32_t n_chains, int32_t n_sweeps, uint64_t seed,
                      uint64_t chain_id, const int8_t* spins0, double* m, double* beta_eps, int8_t* spins_final,
                      double* acceptance, double* seconds);

/* ---- diagnostics (same kernels as the hot path) --------------------------- */

/* F = -dS/dpsi at the host field psi (N values) into host F (N values), with
 * the state rounded to `precision` (Sec. 3 equations of motion). */
int ihmc_force(ihmc_ctx* ctx, const ihmc_lattice* lat, int32_t precision, const double* psi, double* F);
/* Allocation-free variant of ihmc_force, for callers that cannot allocate
 * device memory (code under HIP stream capture, tight serving loops, harnesses
 * that forbid hipMalloc): F = -dS/dpsi of the device field `psi` into the
 * device array `F`, both N values of the state `precision` (4: float, 8:
 * double) in site order, caller-owned, enqueued on `stream` (a hipStream_t;
 * NULL: the context stream) and not waited for.  The lattice may carry no
 * field or a uniform one (h_len 0 or 1; a per-site field is
 * IHMC_E_UNSUPPORTED).  It allocates nothing: the chain descriptor, tile table
 * and padded field staging live in a fixed 32 MiB device array per GPU (a
 * lattice whose staging exceeds it, about 3.9M FP32 or 1.9M FP64 sites, is
 * IHMC_E_INVAL).  Every call on one GPU uses that GPU's array, which keeps the
 * last call's contents: calls that overlap on one GPU (other streams, other
 * host threads, other contexts of the device) race and must be serialised by
 * the caller.  Same force pass and bits as ihmc_force. */
int ihmc_force_noalloc(ihmc_ctx* ctx, const ihmc_lattice* lat, int32_t precision, const void* psi, void* F,
                       void* stream);
/* Action and estimators of a host field psi: out[0] = S(psi) (FP64, eq.
 * phi_psi_substitution without constants), out[1] = m, out[2] = |m|,
 * out[3] = m^2 corrected, out[4] = beta*eps (Sec. 4). */
int ihmc_action(ihmc_ctx* ctx, const ihmc_lattice* lat, int32_t precision, const double* psi, double* out);
/* The HMC Hamiltonian H(psi, p) = 1/2 p.p + S(psi) of Sec. 3 (S as in
 * ihmc_action) at host psi and p (N values each, rounded to the state
 * `precision` as a chain holds them), into *H.  Computed by the hot path's own
 * kernels: the kinetic sum of a first pass that reads the given momenta and
 * the set-up measurement of S, added in exact fixed point (as every
 * trajectory's H_old).  IHMC_E_INVAL (and *H = NaN) when a site term is
 * non-finite or reaches 2^28 in magnitude. */
int ihmc_hamiltonian(ihmc_ctx* ctx, const ihmc_lattice* lat, int32_t precision, const double* psi, const double* p,
                     double* H);
/* One trajectory of molecular dynamics from host (psi, p), in place, with
 * run->n_md, traj_len, integrator, precision (no Metropolis test). */
int ihmc_integrate(ihmc_ctx* ctx, const ihmc_lattice* lat, const ihmc_run* run, double* psi, double* p);
/* The normals of the GPU generator for sites 0..n-1 of (seed, chain_id, traj,
 * tag) into host out, exactly as a pass of state precision `precision` (4 or
 * 8) draws them: Box-Muller in FP64 on the Philox pair's two 53-bit uniforms
 * (sites 2i and 2i+1 from pair i), rounded to FP32 for precision 4 (Sec. 3, eq.
 * momentum distribution). */
int ihmc_philox_normals(ihmc_ctx* ctx, uint64_t seed, uint64_t chain_id, uint32_t traj, uint32_t tag,
                        int32_t precision, int64_t n, double* out);
/* Raw Philox4x32-10 words: for k < n, out[4k..4k+3] = philox(ctr[4k..4k+3],
 * key[2k..2k+1]), computed on the GPU. */
int ihmc_philox_words(ihmc_ctx* ctx, int64_t n, const uint32_t* ctr, const uint32_t* key, uint32_t* out);

/* Host-only (no device needed).  The launch plan that n chains (lats, runs)
 * would form in one chain set of a context with step fusion `fuse_steps` and
 * LDS-resident limit `resident_sites` (as ihmc_ctx_set_resident; tile classes
 * from the built-in rule), and a dry run of one round of it: *taken = the
 * fork/join events the round records, *reserved = the events a chain set
 * creates for it.  A round that would need more than the chain set holds fails
 * with IHMC_E_DEVICE rather than record past them. */
int ihmc_plan_events(int32_t n, const ihmc_lattice* lats, const ihmc_run* runs, int32_t fuse_steps,
                     int64_t resident_sites, int64_t* taken, int64_t* reserved);
/* Host-only.  The exact fixed-point form (unit 2^-64, 128-bit two's
 * complement, rounded to nearest with ties away from zero) that single action
 * changes of any size take, such as the sign flip's (Sec. 3): for k < n,
 * out[2k] / out[2k+1] = low / high word of round(x[k] 2^64), ok[k] = 1; ok[k] =
 * 0 (and zero words) when |x[k]| >= 2^62 or x[k] is not finite, in which case
 * the flip is rejected and counted as non-finite. */
int ihmc_fixed_point(int64_t n, const double* x, uint64_t* out, int32_t* ok);

/* ---- measurement ----------------------------------------------------------- */

/* Number of launch groups of a chain set (chains of equal precision,
 * dimension and tile class share launches; groups are ordered by (precision,
 * ndim, tile class)). */
int ihmc_chains_groups(ihmc_chains* chains, int32_t* n_groups);
/* Launch group `group` (0 <= group < n_groups): out[0..5] = state precision,
 * ndim, tile class (see ihmc_tile_shape), chains, lattice sites, tiles. */
int ihmc_chains_group_info(ihmc_chains* chains, int32_t group, int64_t* out);
/* The chains (indices into the set) of launch group `group`, in launch order
 * (descending pass count), into chain_idx (out[3] of ihmc_chains_group_info
 * entries). */
int ihmc_chains_group_chains(ihmc_chains* chains, int32_t group, int32_t* chain_idx);
/* Time the fused pass kind `mode` (0 = first, 1 = middle, 2 = last, 5 = two
 * middle steps in one launch, 2D groups whose chains have at least two middle
 * steps) of launch group `group`: one warm-up launch, then `reps` launches bracketed by HIP
 * events on the context stream.  Returns the mean duration per launch in
 * microseconds and the lattice sites one launch covers.  The repeated passes
 * overwrite the chains' momenta and field buffers (and a last pass closes a
 * trajectory of every chain in the group): call it only when the chains'
 * results have been fetched or are no longer needed. */
int ihmc_chains_time_pass(ihmc_chains* chains, int32_t group, int32_t mode, int32_t reps, double* avg_us,
                          int64_t* sites, int32_t* ndim, int32_t* precision);

/* Copy `bytes` (>= 4096) between two arena buffers with a plain 16-byte-vector
 * streaming kernel, `reps` times after one warm-up, timed with HIP events on
 * the context stream; returns the mean microseconds per copy (read + write
 * traffic = 2 * bytes).  The achievable-bandwidth reference of the roofline. */
int ihmc_copy_bandwidth(ihmc_ctx* ctx, uint64_t bytes, int32_t reps, double* avg_us);

/* ---- tile autotuner ---------------------------------------------------------- */

/* A lattice pass covers its chain in tiles of one of a few shapes, the tile
 * classes: in 2D 0 = 64 x 16, 1 = 16 x 16, 2 = 32 x 32 sites; in 3D boxes of
 * 0 = 32 x 8 x 4, 1 = 16 x 16 x 4, 2 = 32 x 8 x 8, 3 = 16 x 16 x 8.  The class
 * changes speed only: every class gives bitwise the same trajectories, since
 * all sums are formed per x-aligned quad of sites and per aligned four-plane
 * column and then added in exact fixed point.  A chain takes its class when it is
 * created (ihmc_chains_create, ihmc_run_*, ihmc_submit) from its context's
 * table, keyed by (precision, ndim, L, per-site field or not), and without a
 * table entry from a built-in rule (narrower tiles where a row ends just past a
 * multiple of the wide tile; in 3D eight-plane boxes where L[2] is a multiple
 * of 8 and L[0] of 4).  When the environment variable IHMC_TUNE_CACHE
 * names a file, ihmc_ctx_create loads the table from it if it exists (failing
 * with IHMC_E_INVAL if it is malformed) and ihmc_tune saves the table there. */
#define IHMC_TUNE_RULE 0     /* no entry: the built-in rule */
#define IHMC_TUNE_MEASURED 1 /* chosen by ihmc_tune */
#define IHMC_TUNE_PINNED 2   /* set by ihmc_tune_pin; ihmc_tune leaves it */
#define IHMC_TUNE_FORCE 1    /* ihmc_tune flag: measure keys that have a measured entry again */

/* Tile extent of class cls in dimension ndim: out[0..2] = sites in x, y and
 * planes in z (1 in 2D); IHMC_E_INVAL for an unknown class.  *n_classes (if
 * not NULL) = number of classes of ndim (out may be NULL to ask only that). */
int ihmc_tile_shape(int32_t ndim, int32_t cls, int32_t* out, int32_t* n_classes);
/* Autotune: for each distinct key among lats[0..n) (state precision
 * precision[i]), time the middle steps of every tile class (two per launch in 2D
 * when step fusion is on, see ihmc_ctx_set_step_fusion) and keep the fastest
 * in the table (the built-in rule's class stays unless another is over 3 % faster).  A measurement
 * runs on the context stream over replicas of the lattice with synthetic
 * fields, about `sites` sites in all (at most 65536 replicas): the working set
 * the choice is for, since whether the state streams from HBM or stays in the
 * last-level cache decides which tile is fastest.  sites = 0 takes the total
 * sites of lats[0..n), repeats included (pass the lattices of the chains that
 * will run together); the value is clamped to [2^20, 2^26].  Per class, `reps`
 * launches (0: 10, or 4 above 2^23 sites) after a warm-up, in three rounds
 * interleaved across the classes, keeping the least mean.  The arena must hold
 * the replicas (6 state fields, 7 with a per-site field, each replica) for the
 * duration of one key.  Keys with a measured entry are skipped unless flags has
 * IHMC_TUNE_FORCE; pinned keys are always skipped.  Synchronous; *n_measured
 * (may be NULL) = keys measured.  Existing chains keep their classes. */
int ihmc_tune(ihmc_ctx* ctx, int32_t n, const ihmc_lattice* lats, const int32_t* precision, int64_t sites,
              int32_t reps, int32_t flags, int32_t* n_measured);
/* The class that chains of (lat, precision) would take on this context, its
 * source (IHMC_TUNE_*) and, if ns_site is not NULL, ns_site[0..3] = measured
 * middle-pass nanoseconds per site of each class (NaN where not measured or
 * the class does not exist). */
int ihmc_tune_lookup(ihmc_ctx* ctx, const ihmc_lattice* lat, int32_t precision, int32_t* cls, int32_t* source,
                     double* ns_site);
/* Pin class cls for (lat, precision); cls < 0 removes the entry (the rule
 * applies again).  IHMC_E_INVAL for a class that does not exist. */
int ihmc_tune_pin(ihmc_ctx* ctx, const ihmc_lattice* lat, int32_t precision, int32_t cls);
/* Write the table to `path` as JSON / merge the JSON table at `path` into the
 * context's (entries replace equal keys; IHMC_E_INVAL for a missing, malformed
 * or out-of-range file, leaving the table unchanged). */
int ihmc_tune_save(ihmc_ctx* ctx, const char* path);
int ihmc_tune_load(ihmc_ctx* ctx, const char* path);
/* Read and check the JSON table at `path` without a context or GPU;
 * *n_entries (may be NULL) = distinct keys in it. */
int ihmc_tune_check(const char* path, int32_t* n_entries);

#ifdef __cplusplus
}
#endif

#endif /* IHMC_H */
