/*
 * ihmc_oracle.c -- plain FP64 CPU reference for Hybrid Monte Carlo on the
 * Hubbard-Stratonovich-transformed Ising model (Ostmeyer, Berkowitz, Luu,
 * Petschlies, Pittler: "The Ising Model with Hybrid Monte Carlo",
 * arXiv:1912.03278).
 *
 * TEST INFRASTRUCTURE.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * constant generator with the HIP path, and the HIP path never calls it.
 *
 * Everything is written for clarity, not speed: plain site loops, explicit
 * neighbour arithmetic, no tiling, no fusion, FP64 throughout, compensated
 * (Neumaier) summation for every global sum.  Compile without fast-math and
 * without FP contraction.
 *
 * What it computes (paper section / equation in brackets):
 *   model      H(s) = -1/2 J s^T K s - h.s, periodic nearest-neighbour K on a
 *              d-dimensional torus, or an explicit symmetric coupling matrix
 *              in place of K                    [Sec. 2, eq. hamilton_matrix_notation]
 *   shift      Kt = K + C*1, J' = beta*J, h' = beta*h
 *                                                [Sec. 2, eqs. def_J_prime .. eigen_spectrum_K]
 *   action     S(psi) = 1/2 psi.Kt psi - psi.h'/sqrt(J')
 *                       - sum_i log cosh(sqrt(J') (Kt psi)_i)
 *              (the psi-dependent part of eq. phi_psi_substitution)
 *   HMC        H = 1/2 p^2 + S(psi), momenta N(0,1)   [Sec. 3, eq. momentum distribution]
 *   EOM        dpsi/dt = p,
 *              dp/dt = -Kt psi + h'/sqrt(J') + sqrt(J') Kt tanh(sqrt(J') Kt psi)   [Sec. 3]
 *   integrator leap-frog (kick-drift-kick) over one MD time unit, optionally
 *              the Omelyan second-order minimum-norm scheme  [Sec. 3]
 *   accept     min(1, exp(-dH)); a rejected proposal repeats the old state
 *                                                [Sec. 3]
 *   flip       optional global sign flip psi -> -psi with its own Metropolis
 *              test every `flip_every` trajectories   [Sec. 3, last paragraph]
 *   estimators m = (sum psi / sqrt(J') - 1^T Kt^-1 h' / J') / N,
 *              beta*eps = C J'/2 + h'^T Kt^-1 h' / (2 N J')
 *                         - psi.h' / (2 N sqrt(J'))
 *                         - sqrt(J')/(2N) (Kt psi).tanh(sqrt(J') Kt psi)
 *              (eqs. formula_for_m and formula_for_e written for a general
 *              field; they reduce to the printed forms for constant h)
 *   shifted    the substitution phi = sqrt(J') Kt psi in eq. did_HS_trafo
 *              (field inside the log cosh, no linear term), with the paper's
 *              estimators carried over by psi -> psi + Kt^-1 h'/sqrt(J')
 *                                                [Sec. 2, eqs. did_HS_trafo, phi_psi_substitution]
 *   phi form   the inverse formulation of eq. cosh_in_exponent  [Sec. 2]
 *   MH         single-spin Metropolis-Hastings on the spins, checkerboard
 *              sweeps on a lattice and sequential sweeps with an explicit
 *              coupling matrix (the comparison method)  [Secs. 4, 5]
 *
 * Randomness: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by the
 * 64-bit seed, counter = (pair index, trajectory, chain id, tag); two 53-bit
 * uniforms in (0,1) per call; Box-Muller in FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_FORM_PSI 0
#define ORC_FORM_SHIFTED 2

#define ORC_TAG_INIT 1u
#define ORC_TAG_MOM 2u
#define ORC_TAG_ACC 3u
#define ORC_TAG_FLIP 4u
#define ORC_TAG_MH 5u
#define ORC_TAG_MH_INIT 6u

#define ORC_LEAPFROG 0
#define ORC_OMELYAN 1

/* ------------------------------------------------------------------------ */
/* Public structures (mirrored by the ctypes wrapper in oracle/__init__.py). */

typedef struct {
    int32_t ndim;       /* 1, 2 or 3 */
    int32_t L[3];       /* extents, each >= 3 (periodic) */
    double J, beta, C;  /* J' = beta*J > 0, C > 2*ndim */
    const double* h;    /* field: NULL/h_len 0 -> 0, h_len 1 -> uniform, N -> per site */
    int64_t h_len;
} orc_lattice;

typedef struct {
    int64_t N;          /* number of sites */
    const double* K;    /* N*N symmetric couplings, row-major, replaces K of the lattice */
    double J, beta, C;  /* Kt = K + C*1 must be positive definite */
    const double* h;
    int64_t h_len;
} orc_dense;

typedef struct {
    int32_t n_md;          /* MD steps per trajectory */
    double traj_len;       /* MD time per trajectory */
    int32_t n_traj;        /* trajectories */
    int32_t flip_every;    /* 0: no sign-flip proposals */
    int32_t integrator;    /* ORC_LEAPFROG | ORC_OMELYAN */
    int32_t form;          /* ORC_FORM_PSI (0) | ORC_FORM_SHIFTED (2) */
    uint64_t seed;         /* Philox key */
    uint64_t chain_id;     /* Philox counter word 2 (low 32 bits used) */
    const double* psi0;    /* NULL: psi0 ~ N(0,1) from the TAG_INIT stream */
    const uint8_t* replay_accept; /* NULL, or forced accept decisions (test hook) */
} orc_run;

typedef struct {
    double *dH, *m, *abs_m, *m2c, *beta_eps, *H_old, *H_new; /* each n_traj, may be NULL */
    uint8_t* accepted;     /* n_traj, may be NULL */
    uint8_t* flipped;      /* n_traj, may be NULL */
    double* psi_final;     /* N, may be NULL */
    double acceptance;
    double mean_exp_minus_dH;
    int64_t n_nonfinite;
} orc_result;

/* ------------------------------------------------------------------------ */
/* Compensated summation (Neumaier's variant of Kahan summation).            */

typedef struct { double s, c; } nsum;

static void ns_add(nsum* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double ns_val(const nsum* a) { return a->s + a->c; }

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition: 10 rounds; each round      */
/* multiplies words 0 and 2 by two fixed odd constants, keeps the 64-bit     */
/* products split into hi/lo halves, and mixes the hi halves with words 1,3  */
/* and the round key; the key is advanced by two Weyl constants per round.   */

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw4(uint64_t seed, uint32_t i, uint32_t traj, uint64_t chain, uint32_t tag, uint32_t out[4]) {
    uint32_t ctr[4] = { i, traj, (uint32_t)chain, tag };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    orc_philox4x32_10(ctr, key, out);
}

/* 53 random bits -> (k + 1/2) / 2^53, strictly inside (0, 1). */
static double u53(uint32_t a, uint32_t b) {
    uint64_t k = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
    return ((double)k + 0.5) * (1.0 / 9007199254740992.0);
}

double orc_uniform(uint64_t seed, uint64_t chain, uint32_t traj, uint32_t tag) {
    uint32_t w[4];
    draw4(seed, 0u, traj, chain, tag, w);
    return u53(w[0], w[1]);
}

/* Standard normals for sites 0..n-1: pair i feeds sites 2i (cos) and 2i+1 (sin). */
void orc_normals(uint64_t seed, uint64_t chain, uint32_t traj, uint32_t tag, int64_t n, double* out) {
    const double two_pi = 6.283185307179586;
    for (int64_t i = 0; 2 * i < n; ++i) {
        uint32_t w[4];
        draw4(seed, (uint32_t)i, traj, chain, tag, w);
        double u1 = u53(w[0], w[1]);
        double u2 = u53(w[2], w[3]);
        double r = sqrt(-2.0 * log(u1));
        double th = two_pi * u2;
        out[2 * i] = r * cos(th);
        if (2 * i + 1 < n) out[2 * i + 1] = r * sin(th);
    }
}

/* ------------------------------------------------------------------------ */
/* Model: the shifted coupling matrix Kt and the field terms.                */

typedef struct {
    int dense;
    int64_t N;
    int ndim;
    int L[3];
    const double* K;      /* dense couplings (not owned) */
    double C, Jp, sqJ;    /* shift, J' = beta J, sqrt(J') */
    double* hp;           /* h' = beta*h per site, or NULL when h = 0 */
    double* b;            /* h'/sqrt(J') per site, or NULL */
    double c_m;           /* 1^T Kt^-1 h' */
    double c_e;           /* h'^T Kt^-1 h' */
    double c_v;           /* 1^T Kt^-1 1 */
    int shifted;          /* the h'-inside-log-cosh form (see action) */
    double* scratch[4];   /* work vectors of length N */
} model;

/* u = Kt psi for the periodic nearest-neighbour lattice: C*psi_x plus the
 * two neighbours along every axis (multiplicity counted for small L).      */
static void lattice_apply(const model* M, const double* psi, double* u) {
    const int L0 = M->L[0], L1 = M->ndim > 1 ? M->L[1] : 1, L2 = M->ndim > 2 ? M->L[2] : 1;
    for (int z = 0; z < L2; ++z)
        for (int y = 0; y < L1; ++y)
            for (int x = 0; x < L0; ++x) {
                int64_t s = x + (int64_t)L0 * (y + (int64_t)L1 * z);
                double acc = M->C * psi[s];
                int xp = (x + 1) % L0, xm = (x + L0 - 1) % L0;
                acc += psi[xp + (int64_t)L0 * (y + (int64_t)L1 * z)];
                acc += psi[xm + (int64_t)L0 * (y + (int64_t)L1 * z)];
                if (M->ndim > 1) {
                    int yp = (y + 1) % L1, ym = (y + L1 - 1) % L1;
                    acc += psi[x + (int64_t)L0 * (yp + (int64_t)L1 * z)];
                    acc += psi[x + (int64_t)L0 * (ym + (int64_t)L1 * z)];
                }
                if (M->ndim > 2) {
                    int zp = (z + 1) % L2, zm = (z + L2 - 1) % L2;
                    acc += psi[x + (int64_t)L0 * (y + (int64_t)L1 * zp)];
                    acc += psi[x + (int64_t)L0 * (y + (int64_t)L1 * zm)];
                }
                u[s] = acc;
            }
}

static void dense_apply(const model* M, const double* psi, double* u) {
    const int64_t N = M->N;
    for (int64_t i = 0; i < N; ++i) {
        const double* row = M->K + i * N;
        double acc = 0.0;
        for (int64_t j = 0; j < N; ++j) acc += row[j] * psi[j];
        u[i] = acc + M->C * psi[i];
    }
}

static void apply_Kt(const model* M, const double* psi, double* u) {
    if (M->dense) dense_apply(M, psi, u);
    else lattice_apply(M, psi, u);
}

static double dot(const double* a, const double* b, int64_t n) {
    nsum s = {0, 0};
    for (int64_t i = 0; i < n; ++i) ns_add(&s, a[i] * b[i]);
    return ns_val(&s);
}

/* Conjugate gradient for Kt x = rhs (Kt symmetric positive definite). */
static int cg_solve(const model* M, const double* rhs, double* x) {
    const int64_t N = M->N;
    double* r = (double*)malloc(sizeof(double) * N);
    double* d = (double*)malloc(sizeof(double) * N);
    double* q = (double*)malloc(sizeof(double) * N);
    for (int64_t i = 0; i < N; ++i) { x[i] = 0.0; r[i] = rhs[i]; d[i] = rhs[i]; }
    double rr = dot(r, r, N);
    const double stop = 1e-30 * (rr > 0 ? rr : 1.0);
    int it = 0;
    for (; it < 20 * N + 100 && rr > stop; ++it) {
        apply_Kt(M, d, q);
        double alpha = rr / dot(d, q, N);
        for (int64_t i = 0; i < N; ++i) { x[i] += alpha * d[i]; r[i] -= alpha * q[i]; }
        double rr_new = dot(r, r, N);
        double beta = rr_new / rr;
        rr = rr_new;
        for (int64_t i = 0; i < N; ++i) d[i] = r[i] + beta * d[i];
    }
    free(r); free(d); free(q);
    return it;
}

static int model_init(model* M, int dense, int64_t N, int ndim, const int* L, const double* K,
                      double J, double beta, double C, const double* h, int64_t h_len) {
    memset(M, 0, sizeof(*M));
    M->dense = dense;
    M->N = N;
    M->ndim = ndim;
    for (int i = 0; i < 3; ++i) M->L[i] = (L && i < ndim) ? L[i] : 1;
    M->K = K;
    M->C = C;
    M->Jp = beta * J;
    if (!(M->Jp > 0.0)) return -1;
    M->sqJ = sqrt(M->Jp);
    for (int i = 0; i < 4; ++i) M->scratch[i] = (double*)calloc((size_t)N, sizeof(double));
    if (h_len != 0 && h_len != 1 && h_len != N) return -1;
    if (h_len > 0) {
        M->hp = (double*)malloc(sizeof(double) * N);
        M->b = (double*)malloc(sizeof(double) * N);
        for (int64_t i = 0; i < N; ++i) {
            M->hp[i] = beta * (h_len == 1 ? h[0] : h[i]);
            M->b[i] = M->hp[i] / M->sqJ;
        }
    }
    /* Observable constants (Sec. 2 after eq. phi_psi_substitution; Sec. 4). */
    if (!dense) {
        const double n0 = 2.0 * ndim;
        /* Kt 1 = (n0 + C) 1 on a regular periodic lattice (eq. hKh_for_constant_h). */
        M->c_v = (double)N / (n0 + C);
        if (M->hp) {
            nsum s = {0, 0};
            for (int64_t i = 0; i < N; ++i) ns_add(&s, M->hp[i]);
            M->c_m = ns_val(&s) / (n0 + C);
            if (h_len == 1) {
                M->c_e = (double)N * M->hp[0] * M->hp[0] / (n0 + C);
            } else {
                double* x = M->scratch[0];
                cg_solve(M, M->hp, x);
                M->c_e = dot(M->hp, x, N);
            }
        }
    } else {
        double* ones = M->scratch[1];
        double* g = M->scratch[0];
        for (int64_t i = 0; i < N; ++i) ones[i] = 1.0;
        cg_solve(M, ones, g); /* g = Kt^-1 1 */
        M->c_v = dot(ones, g, N);
        if (M->hp) {
            M->c_m = dot(g, M->hp, N);
            double* x = M->scratch[2];
            cg_solve(M, M->hp, x);
            M->c_e = dot(M->hp, x, N);
        }
    }
    return 0;
}

static void model_free(model* M) {
    free(M->hp); free(M->b);
    for (int i = 0; i < 4; ++i) free(M->scratch[i]);
}

static double logcosh(double y) {
    double a = fabs(y);
    return a + log1p(exp(-2.0 * a)) - 0.6931471805599453;
}

/* S(psi) and the observable partial sums.  `u` receives Kt psi.
 *
 * The shifted form substitutes phi = sqrt(J') Kt psi in eq. did_HS_trafo
 * instead of phi = sqrt(J') Kt psi - h' (eq. phi_psi_substitution); both are
 * exact.  The field then sits inside the log cosh and the linear term drops:
 *     S(psi) = 1/2 psi.Kt psi - sum_i log cosh(sqrt(J') (Kt psi)_i + h'_i).
 * For such a model sum_ut holds sum_i y_i tanh(y_i), y = sqrt(J') Kt psi + h'. */
typedef struct { double S, sum_psi, sum_psih, sum_ut; } action_parts;

static action_parts action(const model* M, const double* psi, double* u) {
    const int64_t N = M->N;
    apply_Kt(M, psi, u);
    nsum S = {0, 0}, sp = {0, 0}, sph = {0, 0}, sut = {0, 0};
    for (int64_t i = 0; i < N; ++i) {
        const double hpi = M->hp ? M->hp[i] : 0.0;
        ns_add(&S, 0.5 * psi[i] * u[i]);
        ns_add(&sp, psi[i]);
        if (M->hp) ns_add(&sph, psi[i] * hpi);
        if (M->shifted) {
            double y = M->sqJ * u[i] + hpi;
            ns_add(&S, -logcosh(y));
            ns_add(&sut, y * tanh(y));
        } else {
            double y = M->sqJ * u[i];
            if (M->b) ns_add(&S, -psi[i] * M->b[i]);
            ns_add(&S, -logcosh(y));
            ns_add(&sut, u[i] * tanh(y));
        }
    }
    action_parts a = { ns_val(&S), ns_val(&sp), ns_val(&sph), ns_val(&sut) };
    return a;
}

/* F = -dS/dpsi = Kt (sqrt(J') tanh(sqrt(J') Kt psi) - psi) + h'/sqrt(J');
 * shifted form: F = Kt (sqrt(J') tanh(sqrt(J') Kt psi + h') - psi). */
static void force(const model* M, const double* psi, double* F) {
    const int64_t N = M->N;
    double* u = M->scratch[2];
    double* w = M->scratch[3];
    apply_Kt(M, psi, u);
    for (int64_t i = 0; i < N; ++i) {
        double y = M->sqJ * u[i];
        if (M->shifted && M->hp) y += M->hp[i];
        w[i] = M->sqJ * tanh(y) - psi[i];
    }
    apply_Kt(M, w, F);
    if (M->b && !M->shifted)
        for (int64_t i = 0; i < N; ++i) F[i] += M->b[i];
}

static double kinetic(const double* p, int64_t N) {
    nsum s = {0, 0};
    for (int64_t i = 0; i < N; ++i) ns_add(&s, 0.5 * p[i] * p[i]);
    return ns_val(&s);
}

/* Observables from the partial sums (Sec. 4, general-field form). */
typedef struct { double m, abs_m, m2c, beta_eps; } observables;

static observables estimators(const model* M, const action_parts* a) {
    const double N = (double)M->N;
    observables o;
    if (M->shifted) {
        /* The paper's estimators at psi + Kt^-1 h'/sqrt(J'), the point of the
         * substituted field that carries the same phi: the Kt^-1 terms cancel,
         * m = sum psi / (N sqrt(J')) and
         * beta*eps = C J'/2 - psi.h'/(2 N sqrt(J')) - sum_i y_i tanh(y_i) / (2N). */
        o.m = a->sum_psi / M->sqJ / N;
        o.beta_eps = 0.5 * M->C * M->Jp - a->sum_psih / (2.0 * N * M->sqJ) - a->sum_ut / (2.0 * N);
    } else {
        o.m = (a->sum_psi / M->sqJ - M->c_m / M->Jp) / N;
        o.beta_eps = 0.5 * M->C * M->Jp + M->c_e / (2.0 * N * M->Jp)
                   - a->sum_psih / (2.0 * N * M->sqJ)
                   - M->sqJ / (2.0 * N) * a->sum_ut;
    }
    o.abs_m = fabs(o.m);
    o.m2c = o.m * o.m - M->c_v / (N * N * M->Jp);
    return o;
}

/* One trajectory of molecular dynamics, in place. */
static void md(const model* M, int n_md, double tau, int integrator, double* psi, double* p) {
    const int64_t N = M->N;
    const double eps = tau / n_md;
    double* F = M->scratch[1];
    if (integrator == ORC_OMELYAN) {
        /* Second-order minimum-norm scheme (Omelyan, Mryglod, Folk 2003),
         * momentum-first form: per step kick lambda*eps, drift eps/2,
         * kick (1-2 lambda)*eps, drift eps/2, kick lambda*eps. */
        const double lam = 0.1931833275037836;
        for (int k = 0; k < n_md; ++k) {
            force(M, psi, F);
            for (int64_t i = 0; i < N; ++i) p[i] += lam * eps * F[i];
            for (int64_t i = 0; i < N; ++i) psi[i] += 0.5 * eps * p[i];
            force(M, psi, F);
            for (int64_t i = 0; i < N; ++i) p[i] += (1.0 - 2.0 * lam) * eps * F[i];
            for (int64_t i = 0; i < N; ++i) psi[i] += 0.5 * eps * p[i];
            force(M, psi, F);
            for (int64_t i = 0; i < N; ++i) p[i] += lam * eps * F[i];
        }
        return;
    }
    /* Leap-frog, kick-drift-kick: half kick, n_md drifts with full kicks in
     * between, half kick at the end. */
    force(M, psi, F);
    for (int64_t i = 0; i < N; ++i) p[i] += 0.5 * eps * F[i];
    for (int k = 1; k <= n_md; ++k) {
        for (int64_t i = 0; i < N; ++i) psi[i] += eps * p[i];
        force(M, psi, F);
        const double kick = (k < n_md) ? eps : 0.5 * eps;
        for (int64_t i = 0; i < N; ++i) p[i] += kick * F[i];
    }
}

static int hmc(const model* M0, const orc_run* R, orc_result* out) {
    const int64_t N = M0->N;
    if (R->n_md < 1 || R->n_traj < 0 || !(R->traj_len > 0)) return -1;
    if (R->form != ORC_FORM_PSI && R->form != ORC_FORM_SHIFTED) return -1;
    model Mf = *M0;
    Mf.shifted = R->form == ORC_FORM_SHIFTED;
    const model* M = &Mf;
    /* psi -> -psi leaves the shifted action unchanged only at h = 0. */
    if (M->shifted && M->hp && R->flip_every > 0) return -1;
    double* psi = (double*)malloc(sizeof(double) * N);
    double* trial = (double*)malloc(sizeof(double) * N);
    double* p = (double*)malloc(sizeof(double) * N);
    double* u = (double*)malloc(sizeof(double) * N);
    if (R->psi0) memcpy(psi, R->psi0, sizeof(double) * N);
    else orc_normals(R->seed, R->chain_id, 0u, ORC_TAG_INIT, N, psi);

    action_parts cur = action(M, psi, u);
    observables ocur = estimators(M, &cur);
    int64_t n_acc = 0, n_nonfinite = 0;
    nsum emdh = {0, 0};
    for (int32_t t = 0; t < R->n_traj; ++t) {
        orc_normals(R->seed, R->chain_id, (uint32_t)t, ORC_TAG_MOM, N, p);
        const double H_old = kinetic(p, N) + cur.S;
        memcpy(trial, psi, sizeof(double) * N);
        md(M, R->n_md, R->traj_len, R->integrator, trial, p);
        action_parts nw = action(M, trial, u);
        const double H_new = kinetic(p, N) + nw.S;
        const double dH = H_new - H_old;
        const int finite = isfinite(dH);
        int acc;
        if (!finite) ++n_nonfinite;
        if (R->replay_accept) {
            acc = R->replay_accept[t] != 0;
        } else {
            const double r = orc_uniform(R->seed, R->chain_id, (uint32_t)t, ORC_TAG_ACC);
            acc = finite && (dH <= 0.0 || r < exp(-dH));
        }
        if (finite) ns_add(&emdh, exp(-dH));
        if (acc) {
            double* tmp = psi; psi = trial; trial = tmp;
            cur = nw;
            ocur = estimators(M, &cur);
            ++n_acc;
        }
        int flipped = 0;
        if (R->flip_every > 0 && (t + 1) % R->flip_every == 0) {
            /* S(-psi) - S(psi) = 2 psi.h'/sqrt(J'): only the linear term changes sign. */
            double dS = 0.0;
            if (M->b) dS = 2.0 * dot(psi, M->b, N);
            const double r = orc_uniform(R->seed, R->chain_id, (uint32_t)t, ORC_TAG_FLIP);
            if (dS <= 0.0 || r < exp(-dS)) {
                for (int64_t i = 0; i < N; ++i) psi[i] = -psi[i];
                cur.S += dS;
                cur.sum_psi = -cur.sum_psi;
                cur.sum_psih = -cur.sum_psih;
                ocur = estimators(M, &cur);
                flipped = 1;
            }
        }
        if (out) {
            if (out->dH) out->dH[t] = dH;
            if (out->H_old) out->H_old[t] = H_old;
            if (out->H_new) out->H_new[t] = H_new;
            if (out->accepted) out->accepted[t] = (uint8_t)acc;
            if (out->flipped) out->flipped[t] = (uint8_t)flipped;
            if (out->m) out->m[t] = ocur.m;
            if (out->abs_m) out->abs_m[t] = ocur.abs_m;
            if (out->m2c) out->m2c[t] = ocur.m2c;
            if (out->beta_eps) out->beta_eps[t] = ocur.beta_eps;
        }
    }
    if (out) {
        if (out->psi_final) memcpy(out->psi_final, psi, sizeof(double) * N);
        out->acceptance = R->n_traj ? (double)n_acc / R->n_traj : 0.0;
        int64_t nf = R->n_traj - n_nonfinite;
        out->mean_exp_minus_dH = nf ? ns_val(&emdh) / (double)nf : 0.0;
        out->n_nonfinite = n_nonfinite;
    }
    free(psi); free(trial); free(p); free(u);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The inverse (phi) formulation, before the substitution: eq.               */
/* cosh_in_exponent gives the phi-dependent action                           */
/*     S(phi) = 1/(2J') phi.Kt^-1 phi - sum_i log cosh(h'_i + phi_i),        */
/* whose force -dS/dphi = -Kt^-1 phi / J' + tanh(h' + phi) needs the solve   */
/* Kt x = phi (CG, to a relative residual of 1e-15) at every evaluation.     */
/* Observables are the exact expectations given phi: the spins are then      */
/* independent with E[s_i | phi] = t_i = tanh(h'_i + phi_i) (eq.             */
/* did_HS_trafo with phi held fixed), so m = sum t / N,                      */
/* m^2 = ((sum t)^2 - sum t^2 + N) / N^2 and                                 */
/* beta eps = (-1/2 J' (t.K t - sum_i K_ii t_i^2 + sum_i K_ii) - h'.t) / N. */

typedef struct { double S, sum_t, sum_t2, sum_ht, tKt; } phi_parts;

static phi_parts phi_action(const model* M, const double* phi, double* x) {
    const int64_t N = M->N;
    double* t = M->scratch[3];
    double* Kt = M->scratch[2];
    cg_solve(M, phi, x);
    nsum S = {0, 0}, st = {0, 0}, st2 = {0, 0}, sht = {0, 0}, q = {0, 0};
    for (int64_t i = 0; i < N; ++i) {
        const double a = phi[i] + (M->hp ? M->hp[i] : 0.0);
        ns_add(&S, 0.5 * phi[i] * x[i] / M->Jp);
        ns_add(&S, -logcosh(a));
        t[i] = tanh(a);
        ns_add(&st, t[i]);
        ns_add(&st2, t[i] * t[i]);
        if (M->hp) ns_add(&sht, M->hp[i] * t[i]);
    }
    /* t.K t with K = Kt - C 1 (the diagonal of K itself handled below) */
    apply_Kt(M, t, Kt);
    for (int64_t i = 0; i < N; ++i) {
        double kii = M->dense ? M->K[i * N + i] : 0.0;
        ns_add(&q, t[i] * (Kt[i] - M->C * t[i]) - kii * t[i] * t[i] + kii);
    }
    phi_parts r = { ns_val(&S), ns_val(&st), ns_val(&st2), ns_val(&sht), ns_val(&q) };
    return r;
}

static observables phi_estimators(const model* M, const phi_parts* a) {
    const double N = (double)M->N;
    observables o;
    o.m = a->sum_t / N;
    o.abs_m = fabs(o.m);
    o.m2c = (a->sum_t * a->sum_t - a->sum_t2 + N) / (N * N);
    o.beta_eps = (-0.5 * M->Jp * a->tKt - a->sum_ht) / N;
    return o;
}

static void phi_force(const model* M, const double* phi, double* F) {
    const int64_t N = M->N;
    double* x = M->scratch[2];
    cg_solve(M, phi, x);
    for (int64_t i = 0; i < N; ++i)
        F[i] = -x[i] / M->Jp + tanh(phi[i] + (M->hp ? M->hp[i] : 0.0));
}

/* Leap-frog (kick-drift-kick) in phi, as md() does in psi. */
static void phi_md(const model* M, int n_md, double tau, double* phi, double* p) {
    const int64_t N = M->N;
    const double eps = tau / n_md;
    double* F = M->scratch[1];
    phi_force(M, phi, F);
    for (int64_t i = 0; i < N; ++i) p[i] += 0.5 * eps * F[i];
    for (int k = 1; k <= n_md; ++k) {
        for (int64_t i = 0; i < N; ++i) phi[i] += eps * p[i];
        phi_force(M, phi, F);
        const double kick = (k < n_md) ? eps : 0.5 * eps;
        for (int64_t i = 0; i < N; ++i) p[i] += kick * F[i];
    }
}

/* The starting field: phi0 given, or phi0 = sqrt(J') Kt psi0 - h' with psi0
 * ~ N(0,1) from the TAG_INIT stream (the substitution that links the forms). */
static void phi_start(const model* M, const orc_run* R, const double* phi0, double* phi) {
    const int64_t N = M->N;
    if (phi0) {
        memcpy(phi, phi0, sizeof(double) * N);
        return;
    }
    double* psi = M->scratch[3];
    orc_normals(R->seed, R->chain_id, 0u, ORC_TAG_INIT, N, psi);
    apply_Kt(M, psi, phi);
    for (int64_t i = 0; i < N; ++i) phi[i] = M->sqJ * phi[i] - (M->hp ? M->hp[i] : 0.0);
}

static int hmc_phi(const model* M, const orc_run* R, orc_result* out) {
    const int64_t N = M->N;
    if (R->n_md < 1 || R->n_traj < 0 || !(R->traj_len > 0) || R->flip_every != 0 || R->integrator != ORC_LEAPFROG)
        return -1;
    double* phi = (double*)malloc(sizeof(double) * N);
    double* trial = (double*)malloc(sizeof(double) * N);
    double* p = (double*)malloc(sizeof(double) * N);
    double* x = (double*)malloc(sizeof(double) * N);
    phi_start(M, R, R->psi0, phi);
    phi_parts cur = phi_action(M, phi, x);
    observables ocur = phi_estimators(M, &cur);
    int64_t n_acc = 0, n_nonfinite = 0;
    nsum emdh = {0, 0};
    for (int32_t t = 0; t < R->n_traj; ++t) {
        orc_normals(R->seed, R->chain_id, (uint32_t)t, ORC_TAG_MOM, N, p);
        const double H_old = kinetic(p, N) + cur.S;
        memcpy(trial, phi, sizeof(double) * N);
        phi_md(M, R->n_md, R->traj_len, trial, p);
        phi_parts nw = phi_action(M, trial, x);
        const double H_new = kinetic(p, N) + nw.S;
        const double dH = H_new - H_old;
        const int finite = isfinite(dH);
        int acc;
        if (!finite) ++n_nonfinite;
        if (R->replay_accept) {
            acc = R->replay_accept[t] != 0;
        } else {
            const double r = orc_uniform(R->seed, R->chain_id, (uint32_t)t, ORC_TAG_ACC);
            acc = finite && (dH <= 0.0 || r < exp(-dH));
        }
        if (finite) ns_add(&emdh, exp(-dH));
        if (acc) {
            double* tmp = phi; phi = trial; trial = tmp;
            cur = nw;
            ocur = phi_estimators(M, &cur);
            ++n_acc;
        }
        if (out) {
            if (out->dH) out->dH[t] = dH;
            if (out->H_old) out->H_old[t] = H_old;
            if (out->H_new) out->H_new[t] = H_new;
            if (out->accepted) out->accepted[t] = (uint8_t)acc;
            if (out->flipped) out->flipped[t] = 0;
            if (out->m) out->m[t] = ocur.m;
            if (out->abs_m) out->abs_m[t] = ocur.abs_m;
            if (out->m2c) out->m2c[t] = ocur.m2c;
            if (out->beta_eps) out->beta_eps[t] = ocur.beta_eps;
        }
    }
    if (out) {
        if (out->psi_final) memcpy(out->psi_final, phi, sizeof(double) * N);
        out->acceptance = R->n_traj ? (double)n_acc / R->n_traj : 0.0;
        int64_t nf = R->n_traj - n_nonfinite;
        out->mean_exp_minus_dH = nf ? ns_val(&emdh) / (double)nf : 0.0;
        out->n_nonfinite = n_nonfinite;
    }
    free(phi); free(trial); free(p); free(x);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Exported entry points.                                                    */

static int64_t lattice_sites(const orc_lattice* lat) {
    int64_t n = 1;
    for (int i = 0; i < lat->ndim; ++i) n *= lat->L[i];
    return n;
}

static int lattice_model(model* M, const orc_lattice* lat) {
    memset(M, 0, sizeof(*M));
    if (lat->ndim < 1 || lat->ndim > 3) return -1;
    for (int i = 0; i < lat->ndim; ++i)
        if (lat->L[i] < 3) return -1;
    if (!(lat->C > 2.0 * lat->ndim)) return -1;
    return model_init(M, 0, lattice_sites(lat), lat->ndim, lat->L, NULL, lat->J, lat->beta,
                      lat->C, lat->h, lat->h_len);
}

static int dense_model(model* M, const orc_dense* d) {
    memset(M, 0, sizeof(*M));
    if (d->N < 1 || !d->K || !(d->C > -1e300)) return -1;
    return model_init(M, 1, d->N, 0, NULL, d->K, d->J, d->beta, d->C, d->h, d->h_len);
}

int orc_lattice_apply(const orc_lattice* lat, const double* psi, double* u) {
    model M;
    if (lattice_model(&M, lat)) { model_free(&M); return -1; }
    apply_Kt(&M, psi, u);
    model_free(&M);
    return 0;
}

int orc_dense_apply(const orc_dense* d, const double* psi, double* u) {
    model M;
    if (dense_model(&M, d)) { model_free(&M); return -1; }
    apply_Kt(&M, psi, u);
    model_free(&M);
    return 0;
}

static int with_model(const orc_lattice* lat, const orc_dense* d, model* M) {
    return lat ? lattice_model(M, lat) : dense_model(M, d);
}

/* F(psi), S(psi) with observables, H(psi, p), MD in place, full HMC runs.
 * Exactly one of `lat` / `dense` is non-NULL. */
int orc_force(const orc_lattice* lat, const orc_dense* d, const double* psi, double* F) {
    model M;
    if (with_model(lat, d, &M)) { model_free(&M); return -1; }
    force(&M, psi, F);
    model_free(&M);
    return 0;
}

/* out[0] = S, out[1] = m, out[2] = |m|, out[3] = m^2 corrected, out[4] = beta*eps,
 * out[5] = sum psi, out[6] = sum psi h', out[7] = sum u tanh(sqrt(J') u). */
int orc_action(const orc_lattice* lat, const orc_dense* d, const double* psi, double* out) {
    model M;
    if (with_model(lat, d, &M)) { model_free(&M); return -1; }
    double* u = (double*)malloc(sizeof(double) * M.N);
    action_parts a = action(&M, psi, u);
    observables o = estimators(&M, &a);
    out[0] = a.S; out[1] = o.m; out[2] = o.abs_m; out[3] = o.m2c; out[4] = o.beta_eps;
    out[5] = a.sum_psi; out[6] = a.sum_psih; out[7] = a.sum_ut;
    free(u);
    model_free(&M);
    return 0;
}

int orc_hamiltonian(const orc_lattice* lat, const orc_dense* d, const double* psi,
                    const double* p, double* H) {
    model M;
    if (with_model(lat, d, &M)) { model_free(&M); return -1; }
    double* u = (double*)malloc(sizeof(double) * M.N);
    action_parts a = action(&M, psi, u);
    *H = kinetic(p, M.N) + a.S;
    free(u);
    model_free(&M);
    return 0;
}

int orc_md(const orc_lattice* lat, const orc_dense* d, int32_t n_md, double traj_len,
           int32_t integrator, double* psi, double* p) {
    model M;
    if (with_model(lat, d, &M) || n_md < 1) { model_free(&M); return -1; }
    md(&M, n_md, traj_len, integrator, psi, p);
    model_free(&M);
    return 0;
}

/* out[0] = 1^T Kt^-1 h', out[1] = h'^T Kt^-1 h', out[2] = 1^T Kt^-1 1. */
int orc_constants(const orc_lattice* lat, const orc_dense* d, double* out) {
    model M;
    if (with_model(lat, d, &M)) { model_free(&M); return -1; }
    out[0] = M.c_m; out[1] = M.c_e; out[2] = M.c_v;
    model_free(&M);
    return 0;
}

/* The same three with the shifted form (h' inside the log cosh). */
int orc_shifted_force(const orc_lattice* lat, const orc_dense* d, const double* psi, double* F) {
    model M;
    if (with_model(lat, d, &M)) { model_free(&M); return -1; }
    M.shifted = 1;
    force(&M, psi, F);
    model_free(&M);
    return 0;
}
int orc_shifted_action(const orc_lattice* lat, const orc_dense* d, const double* psi, double* out) {
    model M;
    if (with_model(lat, d, &M)) { model_free(&M); return -1; }
    M.shifted = 1;
    double* u = (double*)malloc(sizeof(double) * M.N);
    action_parts a = action(&M, psi, u);
    observables o = estimators(&M, &a);
    out[0] = a.S; out[1] = o.m; out[2] = o.abs_m; out[3] = o.m2c; out[4] = o.beta_eps;
    out[5] = a.sum_psi; out[6] = a.sum_psih; out[7] = a.sum_ut;
    free(u);
    model_free(&M);
    return 0;
}
int orc_shifted_md(const orc_lattice* lat, const orc_dense* d, int32_t n_md, double traj_len,
                   int32_t integrator, double* psi, double* p) {
    model M;
    if (with_model(lat, d, &M) || n_md < 1) { model_free(&M); return -1; }
    M.shifted = 1;
    md(&M, n_md, traj_len, integrator, psi, p);
    model_free(&M);
    return 0;
}
int orc_run_lattice(const orc_lattice* lat, const orc_run* run, orc_result* res) {
    model M;
    if (lattice_model(&M, lat)) { model_free(&M); return -1; }
    int rc = hmc(&M, run, res);
    model_free(&M);
    return rc;
}

int orc_run_dense(const orc_dense* d, const orc_run* run, orc_result* res) {
    model M;
    if (dense_model(&M, d)) { model_free(&M); return -1; }
    int rc = hmc(&M, run, res);
    model_free(&M);
    return rc;
}

/* The inverse (phi) formulation: force, action with the observables, the
 * starting field and whole chains (leap-frog only, no sign flip). */
int orc_phi_force(const orc_lattice* lat, const orc_dense* d, const double* phi, double* F) {
    model M;
    if (with_model(lat, d, &M)) { model_free(&M); return -1; }
    phi_force(&M, phi, F);
    model_free(&M);
    return 0;
}

/* out[0] = S(phi), out[1] = m, out[2] = |m|, out[3] = m^2, out[4] = beta*eps. */
int orc_phi_action(const orc_lattice* lat, const orc_dense* d, const double* phi, double* out) {
    model M;
    if (with_model(lat, d, &M)) { model_free(&M); return -1; }
    double* x = (double*)malloc(sizeof(double) * M.N);
    phi_parts a = phi_action(&M, phi, x);
    observables o = phi_estimators(&M, &a);
    out[0] = a.S; out[1] = o.m; out[2] = o.abs_m; out[3] = o.m2c; out[4] = o.beta_eps;
    free(x);
    model_free(&M);
    return 0;
}

int orc_phi_start(const orc_lattice* lat, const orc_dense* d, const orc_run* run, double* phi) {
    model M;
    if (with_model(lat, d, &M)) { model_free(&M); return -1; }
    phi_start(&M, run, run->psi0, phi);
    model_free(&M);
    return 0;
}

int orc_phi_md(const orc_lattice* lat, const orc_dense* d, int32_t n_md, double traj_len, double* phi, double* p) {
    model M;
    if (with_model(lat, d, &M) || n_md < 1) { model_free(&M); return -1; }
    phi_md(&M, n_md, traj_len, phi, p);
    model_free(&M);
    return 0;
}

int orc_run_phi(const orc_lattice* lat, const orc_dense* d, const orc_run* run, orc_result* res) {
    model M;
    if (with_model(lat, d, &M)) { model_free(&M); return -1; }
    int rc = hmc_phi(&M, run, res);
    model_free(&M);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Local Metropolis-Hastings on the spins, the comparison method of Sec. 4. */
/* A sweep proposes every spin once: first the sites of even parity          */
/* x + y + z, then the odd ones (on a lattice of even extents no two sites   */
/* of one parity are neighbours, so each half is a set of independent       */
/* single-site updates).  Flipping s_i changes the energy by                */
/* dE = 2 s_i (J sum_nb s_j + h); the flip is accepted iff dE <= 0 or       */
/* u < exp(-beta dE), u the 53-bit uniform of counter (i, sweep, chain,      */
/* TAG_MH).  Start: s_i = +1 iff the uniform of (i, 0, chain, TAG_MH_INIT)   */
/* is below 1/2.  After every sweep: m = sum s / N and                      */
/* beta eps = beta (-J sum_i sum_mu s_i s_{i+mu} - h sum s) / N.            */

static int mh_sum_nb(const int8_t* s, const int* L, int ndim, int x, int y, int z) {
    const int L0 = L[0], L1 = L[1], L2 = ndim > 2 ? L[2] : 1;
    int acc = 0;
    acc += s[(x + 1) % L0 + (int64_t)L0 * (y + (int64_t)L1 * z)];
    acc += s[(x + L0 - 1) % L0 + (int64_t)L0 * (y + (int64_t)L1 * z)];
    acc += s[x + (int64_t)L0 * ((y + 1) % L1 + (int64_t)L1 * z)];
    acc += s[x + (int64_t)L0 * ((y + L1 - 1) % L1 + (int64_t)L1 * z)];
    if (ndim > 2) {
        acc += s[x + (int64_t)L0 * (y + (int64_t)L1 * ((z + 1) % L2))];
        acc += s[x + (int64_t)L0 * (y + (int64_t)L1 * ((z + L2 - 1) % L2))];
    }
    return acc;
}

int orc_mh_run(const orc_lattice* lat, int32_t n_sweeps, uint64_t seed, uint64_t chain, const int8_t* spins0,
               double* m, double* beta_eps, int8_t* spins_final, double* acceptance) {
    if (lat->ndim < 2 || lat->ndim > 3 || n_sweeps < 0) return -1;
    if (lat->h_len != 0 && lat->h_len != 1) return -1;
    for (int i = 0; i < lat->ndim; ++i)
        if (lat->L[i] < 2 || lat->L[i] % 2) return -1;
    const int ndim = lat->ndim;
    const int L[3] = {lat->L[0], lat->L[1], ndim > 2 ? lat->L[2] : 1};
    const int64_t N = (int64_t)L[0] * L[1] * L[2];
    const double J = lat->J, beta = lat->beta, h = lat->h_len ? lat->h[0] : 0.0;
    int8_t* s = (int8_t*)malloc((size_t)N);
    for (int64_t i = 0; i < N; ++i) {
        if (spins0) {
            s[i] = spins0[i] > 0 ? 1 : -1;
        } else {
            uint32_t w[4];
            draw4(seed, (uint32_t)i, 0u, chain, ORC_TAG_MH_INIT, w);
            s[i] = u53(w[0], w[1]) < 0.5 ? 1 : -1;
        }
    }
    int64_t accepted = 0;
    for (int32_t t = 0; t < n_sweeps; ++t) {
        for (int color = 0; color < 2; ++color)
            for (int z = 0; z < L[2]; ++z)
                for (int y = 0; y < L[1]; ++y)
                    for (int x = 0; x < L[0]; ++x) {
                        if (((x + y + z) & 1) != color) continue;
                        const int64_t i = x + (int64_t)L[0] * (y + (int64_t)L[1] * z);
                        const int sum = mh_sum_nb(s, L, ndim, x, y, z);
                        const double dE = 2.0 * s[i] * (J * sum + h);
                        uint32_t w[4];
                        draw4(seed, (uint32_t)i, (uint32_t)t, chain, ORC_TAG_MH, w);
                        if (dE <= 0.0 || u53(w[0], w[1]) < exp(-beta * dE)) {
                            s[i] = (int8_t)(-s[i]);
                            ++accepted;
                        }
                    }
        int64_t ssum = 0, bsum = 0;
        for (int z = 0; z < L[2]; ++z)
            for (int y = 0; y < L[1]; ++y)
                for (int x = 0; x < L[0]; ++x) {
                    const int64_t i = x + (int64_t)L[0] * (y + (int64_t)L[1] * z);
                    ssum += s[i];
                    bsum += s[i] * s[(x + 1) % L[0] + (int64_t)L[0] * (y + (int64_t)L[1] * z)];
                    bsum += s[i] * s[x + (int64_t)L[0] * ((y + 1) % L[1] + (int64_t)L[1] * z)];
                    if (ndim > 2) bsum += s[i] * s[x + (int64_t)L[0] * (y + (int64_t)L[1] * ((z + 1) % L[2]))];
                }
        if (m) m[t] = (double)ssum / (double)N;
        if (beta_eps) beta_eps[t] = beta * (-J * (double)bsum - h * (double)ssum) / (double)N;
    }
    if (spins_final) memcpy(spins_final, s, (size_t)N);
    if (acceptance) *acceptance = n_sweeps ? (double)accepted / ((double)N * n_sweeps) : 0.0;
    free(s);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Single-spin Metropolis-Hastings with an explicit coupling matrix (the     */
/* comparison method of Sec. 4 on the all-to-all models of Sec. 2 / App. A). */
/* Every spin couples to every other, so no two sites can be updated         */
/* independently: a sweep proposes the spins one after another in site       */
/* order i = 0 .. N-1.  Flipping s_i changes H(s) = -1/2 J s^T K s - h.s by  */
/* dE = 2 s_i (J sum_{j != i} K_ij s_j + h_i) (the diagonal term K_ii s_i^2   */
/* does not change); the flip is accepted iff dE <= 0 or u < exp(-beta dE),  */
/* u the 53-bit uniform of counter (i, sweep, chain, TAG_MH).  The local      */
/* field is summed afresh for every proposal.  Start as in the lattice       */
/* version.  After every sweep: m = sum s / N and                            */
/* beta eps = beta H(s) / N with the full quadratic form (diagonal included). */

int orc_dense_mh_run(const orc_dense* d, int32_t n_sweeps, uint64_t seed, uint64_t chain, const int8_t* spins0,
                     double* m, double* beta_eps, int8_t* spins_final, double* acceptance) {
    if (!d || d->N < 1 || !d->K || n_sweeps < 0) return -1;
    if (d->h_len != 0 && d->h_len != 1 && d->h_len != d->N) return -1;
    if (d->h_len && !d->h) return -1;
    const int64_t N = d->N;
    const double J = d->J, beta = d->beta;
    int8_t* s = (int8_t*)malloc((size_t)N);
    for (int64_t i = 0; i < N; ++i) {
        if (spins0) {
            s[i] = spins0[i] > 0 ? 1 : -1;
        } else {
            uint32_t w[4];
            draw4(seed, (uint32_t)i, 0u, chain, ORC_TAG_MH_INIT, w);
            s[i] = u53(w[0], w[1]) < 0.5 ? 1 : -1;
        }
    }
    int64_t accepted = 0;
    for (int32_t t = 0; t < n_sweeps; ++t) {
        for (int64_t i = 0; i < N; ++i) {
            nsum fs = {0.0, 0.0};
            for (int64_t j = 0; j < N; ++j)
                if (j != i) ns_add(&fs, d->K[i * N + j] * s[j]);
            const double f = ns_val(&fs);
            const double hi = d->h_len == 0 ? 0.0 : (d->h_len == 1 ? d->h[0] : d->h[i]);
            const double dE = 2.0 * s[i] * (J * f + hi);
            uint32_t w[4];
            draw4(seed, (uint32_t)i, (uint32_t)t, chain, ORC_TAG_MH, w);
            if (dE <= 0.0 || u53(w[0], w[1]) < exp(-beta * dE)) {
                s[i] = (int8_t)(-s[i]);
                ++accepted;
            }
        }
        nsum quad = {0.0, 0.0}, field = {0.0, 0.0};
        int64_t ssum = 0;
        for (int64_t i = 0; i < N; ++i) {
            ssum += s[i];
            for (int64_t j = 0; j < N; ++j) ns_add(&quad, d->K[i * N + j] * s[i] * s[j]);
            const double hi = d->h_len == 0 ? 0.0 : (d->h_len == 1 ? d->h[0] : d->h[i]);
            ns_add(&field, hi * s[i]);
        }
        if (m) m[t] = (double)ssum / (double)N;
        if (beta_eps) beta_eps[t] = beta * (-0.5 * J * ns_val(&quad) - ns_val(&field)) / (double)N;
    }
    if (spins_final) memcpy(spins_final, s, (size_t)N);
    if (acceptance) *acceptance = (n_sweeps && N) ? (double)accepted / ((double)N * n_sweeps) : 0.0;
    free(s);
    return 0;
}
