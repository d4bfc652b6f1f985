"""GPU parity of the shifted form (IHMC_FORM_SHIFTED: h' inside the log cosh,
no linear term) against the FP64 oracle, on the same fused passes as the paper's
form: LDS-resident whole trajectories, tiled passes with two leap-frog steps per
launch, and tiled passes with one.

Tolerances as for the paper's form: one trajectory from identical inputs
(psi0, Philox momenta) 1e-12 normwise in FP64 and 1e-5 in FP32 (dense chains,
FP32 state, any field: 1e-5); FP64 chains take the oracle's accept decisions;
served shifted requests equal the same chains alone bit for bit.  Properties checked on the GPU alone: at
h = 0 the two forms give the same chain (bitwise, flips included, beta*eps to
rounding), and with a uniform field a shifted chain started at
psi0 - Kt^-1 h'/sqrt(J') takes the paper-form chain's decisions with the same
observables.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def nrm(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module", params=["resident", "tiled_pairs", "tiled_single"])
def ctx(request):
    from paper_1912_03278_amd import ihmc
    kw = dict(arena_bytes=1 << 30)
    if request.param == "resident":
        kw["resident"] = -1
    else:
        kw["resident"] = 0
        kw["fuse_steps"] = request.param == "tiled_pairs"
    c = ihmc.Context(**kw)
    yield c
    c.close()


CASES = [
    ("2d_ragged_h0", (70, 19), 0.44, 4.1, None),
    ("2d_uniform", (64, 32), 0.35, 4.3, 0.07),
    ("2d_small_wrap", (8, 8), 0.40, 4.1, 0.1),
    ("2d_tiles_ragged", (130, 35), 0.44, 4.1, -0.02),
    ("3d_ragged", (67, 9, 6), 0.22, 6.1, 0.05),
    ("3d_small_wrap", (5, 3, 7), 0.3, 6.5, 0.1),
    ("2d_smallest", (3, 3), 0.4, 4.1, 0.1),
    ("3d_smallest", (3, 3, 3), 0.2, 6.1, "site"),
    ("2d_site_h", (33, 17), 0.5, 4.1, "site"),
    ("3d_site_h", (20, 6, 9), 0.25, 6.1, "site"),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("prec,integ", [(8, 0), (4, 0), (8, 1), (4, 1)])
def test_one_trajectory(ctx, orc, case, prec, integ):
    from paper_1912_03278_amd import ihmc
    name, L, beta, C, h = case
    N = int(np.prod(L))
    if isinstance(h, str):
        h = np.random.default_rng(11).normal(0, 0.2, N)
    psi = np.random.default_rng(2).standard_normal(N)
    n_md = 7 if integ == 0 else 4
    run = ihmc.Run(n_md=n_md, n_traj=1, precision=prec, integrator=integ, seed=5, chain_id=2,
                   psi0=psi, replay_accept=[1], form=ihmc.FORM_SHIFTED)
    g = ctx.run_lattice(ihmc.Lattice(L, beta=beta, C=C, h=h), run)
    psi_ref0 = psi.astype(np.float32).astype(np.float64) if prec == 4 else psi
    r = orc.run(orc.Lattice(L, beta=beta, C=C, h=h), 1, n_md, seed=5, chain_id=2, psi0=psi_ref0,
                replay_accept=[1], integrator=integ, form="shifted")
    tol = 1e-12 if prec == 8 else 1e-5
    assert nrm(g["psi_final"], r.psi_final) < tol
    for k in ("H_old", "H_new"):
        assert abs(g[k][0] - getattr(r, k)[0]) <= tol * abs(getattr(r, k)[0]), k
    for k in ("m", "m2c", "beta_eps"):
        assert abs(g[k][0] - getattr(r, k)[0]) <= tol * max(1.0, abs(getattr(r, k)[0])), k


@pytest.mark.parametrize("prec", [8, 4])
@pytest.mark.parametrize("L,site", [((40, 24), False), ((9, 8, 7), False), ((30, 22), True)])
def test_integrate_arbitrary_momenta(ctx, orc, prec, L, site):
    """ihmc_integrate with a shifted-form run follows the oracle's shifted MD."""
    from paper_1912_03278_amd import ihmc
    rng = np.random.default_rng(4)
    N = int(np.prod(L))
    beta, C = (0.45, 4.1) if len(L) == 2 else (0.22, 6.1)
    psi, p = rng.standard_normal(N), rng.standard_normal(N)
    if prec == 4:
        psi = psi.astype(np.float32).astype(np.float64)
        p = p.astype(np.float32).astype(np.float64)
    h = rng.normal(0, 0.1, N) if site else 0.06
    run = ihmc.Run(n_md=9, n_traj=1, precision=prec, form=ihmc.FORM_SHIFTED)
    gpsi, gp = ctx.integrate(ihmc.Lattice(L, beta=beta, C=C, h=h), run, psi, p)
    rpsi, rp = orc.md(orc.Lattice(L, beta=beta, C=C, h=h), psi, p, 9, form="shifted")
    tol = 1e-12 if prec == 8 else 1e-5
    assert nrm(gpsi, rpsi) < tol and nrm(gp, rp) < tol
    # and differs from the paper form's dynamics from the same point
    ppsi, _ = ctx.integrate(ihmc.Lattice(L, beta=beta, C=C, h=h), ihmc.Run(n_md=9, n_traj=1, precision=prec), psi, p)
    assert nrm(ppsi, rpsi) > 1e-3


@pytest.mark.parametrize("L,h", [((16, 12), 0.05), ((6, 5, 7), 0.08), ((14, 10), "site")])
def test_fp64_chain_takes_the_oracles_decisions(ctx, orc, L, h):
    from paper_1912_03278_amd import ihmc
    beta, C = (0.42, 4.1) if len(L) == 2 else (0.22, 6.1)
    if isinstance(h, str):
        h = np.random.default_rng(12).normal(0, 0.1, int(np.prod(L)))
    g = ctx.run_lattice(ihmc.Lattice(L, beta=beta, C=C, h=h),
                        ihmc.Run(n_md=8, n_traj=300, precision=8, seed=7, chain_id=4, form=ihmc.FORM_SHIFTED))
    r = orc.run(orc.Lattice(L, beta=beta, C=C, h=h), 300, 8, seed=7, chain_id=4, form="shifted")
    # The kernels form y = sqrt(J') u + h' with one rounding (FMA), the oracle
    # with two; such one-ulp differences grow along the chaotic MD flow (from
    # 1e-14 in the first trajectories to about 1e-7 after 300 on the 3D case)
    # while every decision stays the oracle's.
    assert np.array_equal(g["accepted"], r.accepted) and 0.5 < r.acceptance < 1.0
    assert np.max(np.abs(g["dH"][:50] - r.dH[:50])) < 1e-9
    assert np.max(np.abs(g["dH"] - r.dH)) < 1e-6
    for k in ("m", "m2c", "beta_eps"):
        assert np.max(np.abs(g[k][:50] - getattr(r, k)[:50])) < 1e-9, k
        assert np.max(np.abs(g[k] - getattr(r, k))) < 1e-6, k
    assert nrm(g["psi_final"], r.psi_final) < 1e-6


@pytest.mark.parametrize("prec", [8, 4])
def test_zero_field_equals_paper_form(ctx, prec):
    from paper_1912_03278_amd import ihmc
    lat = ihmc.Lattice((40, 24), beta=0.44, C=4.1)
    out = []
    for form in (ihmc.FORM_PSI, ihmc.FORM_SHIFTED):
        out.append(ctx.run_lattice(lat, ihmc.Run(n_md=7, n_traj=30, precision=prec, seed=3, chain_id=1,
                                                 flip_every=4, form=form)))
    a, b = out
    for k in ("dH", "accepted", "flipped", "psi_final", "m", "m2c"):
        assert np.array_equal(a[k], b[k]), k
    assert np.max(np.abs(a["beta_eps"] - b["beta_eps"])) < 1e-13
    assert b["flipped"].sum() > 0


@pytest.mark.parametrize("L", [(48, 40), (12, 10, 9)])
def test_translate_of_the_paper_form(ctx, L):
    """psi_paper = psi_shifted + h'/(sqrt(J') (n0 + C)) for a uniform field
    (Kt 1 = (n0 + C) 1 on the periodic lattice, eq. hKh_for_constant_h)."""
    from paper_1912_03278_amd import ihmc
    beta, C, h = (0.44, 4.1, 0.03) if len(L) == 2 else (0.22, 6.1, 0.04)
    N = int(np.prod(L))
    lat = ihmc.Lattice(L, beta=beta, C=C, h=h)
    delta = beta * h / (math.sqrt(beta) * (2 * len(L) + C))
    psi0 = np.random.default_rng(8).standard_normal(N)
    a = ctx.run_lattice(lat, ihmc.Run(n_md=8, n_traj=40, precision=8, seed=6, chain_id=2, psi0=psi0))
    b = ctx.run_lattice(lat, ihmc.Run(n_md=8, n_traj=40, precision=8, seed=6, chain_id=2, psi0=psi0 - delta,
                                      form=ihmc.FORM_SHIFTED))
    assert np.array_equal(a["accepted"], b["accepted"]) and a["acceptance"] > 0.5
    assert np.max(np.abs(a["dH"] - b["dH"])) < 1e-8
    for k in ("m", "m2c", "beta_eps"):
        assert np.max(np.abs(a[k] - b[k])) < 1e-10, k
    assert np.max(np.abs(a["psi_final"] - (b["psi_final"] + delta))) < 1e-10


def test_mixed_forms_in_one_set_equal_alone(ctx):
    """Paper-form and shifted chains of one shape share launch groups; each
    chain's series equal those of the chain run alone, bitwise."""
    from paper_1912_03278_amd import ihmc
    lats = [ihmc.Lattice((48, 40), beta=0.44, C=4.1, h=0.02 * (i + 1)) for i in range(4)]
    lats.append(ihmc.Lattice((12, 10, 9), beta=0.22, C=6.1, h=0.03))
    lats.append(ihmc.Lattice((48, 40), beta=0.44, C=4.1, h=np.random.default_rng(3).normal(0, 0.05, 1920)))
    runs = [ihmc.Run(n_md=6 + i, n_traj=5, seed=4, chain_id=i, precision=4 if i % 2 else 8,
                     form=ihmc.FORM_SHIFTED if i in (1, 2, 4, 5) else ihmc.FORM_PSI) for i in range(6)]
    ch = ihmc.Chains(ctx, lats, runs)
    ch.advance(5)
    mixed = [ch.result(i) for i in range(6)]
    ch.close()
    for i in range(6):
        alone = ctx.run_lattice(lats[i], runs[i])
        for k in ("dH", "accepted", "psi_final", "m", "m2c", "beta_eps"):
            assert np.array_equal(mixed[i][k], alone[k]), (i, k)


def _rand_K(N, seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(0.0, 1.0 / np.sqrt(N), (N, N))
    K = np.triu(A, 1)
    return K + K.T


@pytest.mark.parametrize("integ,n_md", [(0, 8), (1, 4)])
@pytest.mark.parametrize("N,h", [(300, 0.05), (500, "site"), (301, None)])
def test_dense_one_trajectory(ctx, orc, integ, n_md, N, h):
    """Dense chains (BF16-limb GEMMs, FP32 state): any field, 1e-5 as for the paper's form."""
    from paper_1912_03278_amd import ihmc
    rng = np.random.default_rng(N + 7 * integ)
    K = _rand_K(N, 3)
    C = -np.linalg.eigvalsh(K)[0] + 0.1
    hv = rng.normal(0, 0.1, N) if h == "site" else h
    B = 4
    psi0 = [rng.standard_normal(N) for _ in range(B)]
    runs = [ihmc.Run(n_md=n_md, n_traj=1, integrator=integ, seed=7, chain_id=10 + i, psi0=psi0[i],
                     replay_accept=[1], form=ihmc.FORM_SHIFTED if i != 2 else ihmc.FORM_PSI) for i in range(B)]
    g = ctx.run_dense(ihmc.Dense(K, beta=0.9, C=C, h=hv), runs)
    for i in range(B):
        r = orc.run(orc.Dense(K, beta=0.9, C=C, h=hv), 1, n_md, seed=7, chain_id=10 + i,
                    psi0=psi0[i].astype(np.float32).astype(np.float64), replay_accept=[1], integrator=integ,
                    form="shifted" if i != 2 else "psi")
        assert nrm(g[i]["psi_final"], r.psi_final) < 1e-5, (i, nrm(g[i]["psi_final"], r.psi_final))
        for k in ("H_old", "H_new"):
            assert abs(g[i][k][0] - getattr(r, k)[0]) <= 1e-5 * abs(getattr(r, k)[0]), (i, k)
        for k in ("m", "m2c", "beta_eps"):
            assert abs(g[i][k][0] - getattr(r, k)[0]) <= 1e-5 * max(1.0, abs(getattr(r, k)[0])), (i, k)


def test_dense_shifted_alone_equals_mixed_bitwise(ctx):
    from paper_1912_03278_amd import ihmc
    N = 300
    model = ihmc.Dense(_rand_K(N, 6), beta=0.8, C=2.2, h=0.04)
    runs = [ihmc.Run(n_md=5, n_traj=6, seed=9, chain_id=i, form=ihmc.FORM_SHIFTED if i % 3 else ihmc.FORM_PSI)
            for i in range(40)]
    both = ctx.run_dense(model, runs)
    for i in (1, 3, 38):
        alone = ctx.run_dense(model, [runs[i]])[0]
        for k in ("dH", "beta_eps", "psi_final"):
            assert np.array_equal(both[i][k], alone[k]), (i, k)


def test_served_shifted_requests_equal_alone(ctx):
    """Served shifted and paper-form requests (2D/3D, FP32/FP64, uniform and per-site
    fields, flips at h = 0, Omelyan) equal the same chains run alone, bit for bit."""
    import time
    from paper_1912_03278_amd import ihmc
    reqs = []
    rng = np.random.default_rng(9)
    for i in range(14):
        L = (24 + 4 * i, 20) if i % 3 else (8, 6, 5 + i)
        h = 0.02 * (i % 4) if i % 4 else None
        if i >= 12:  # per-site fields: translated coordinates
            L = (70 + 10 * i, 40)
            h = rng.normal(0, 0.05, L[0] * L[1])
        lat = ihmc.Lattice(L, beta=0.4 if len(L) == 2 else 0.22, C=4.1 if len(L) == 2 else 6.1, h=h)
        reqs.append((lat, ihmc.Run(n_md=4 + i % 5, n_traj=6, seed=3, chain_id=i, precision=8 if i % 2 else 4,
                                   integrator=i % 2 if i % 4 == 3 else 0, flip_every=2 if i % 4 == 0 and i < 12 else 0,
                                   form=ihmc.FORM_SHIFTED if i % 4 != 1 else ihmc.FORM_PSI)))
    sv = ihmc.Server(ctx, budget_bytes=8 << 20, max_active=6)
    tickets = []
    for k, (lat, run) in enumerate(reqs):
        tickets.append(sv.submit(lat, run))
        if k % 4 == 3:
            time.sleep(0.01)
    served = []
    for t in tickets:
        assert sv.wait(t, 120.0) == ihmc.REQ_DONE
        served.append(sv.fetch(t))
    sv.close()
    for (lat, run), g in zip(reqs, served):
        alone = ctx.run_lattice(lat, run)
        for k in ("dH", "H_old", "H_new", "m", "beta_eps", "psi_final", "accepted", "flipped"):
            assert np.array_equal(g[k], alone[k]), (lat.L, k)


@pytest.mark.parametrize("dense,site", [(False, False), (False, True), (True, False)])
def test_checkpoint_resume_and_form_mismatch(ctx, dense, site):
    """A shifted chain resumed from a checkpoint continues bit for bit; the
    checkpoint does not restore into a paper-form chain of the same model."""
    from paper_1912_03278_amd import ihmc
    if dense:
        model = ihmc.Dense(_rand_K(200, 2), beta=0.8, C=2.3, h=np.random.default_rng(1).normal(0, 0.1, 200))
    else:
        model = ihmc.Lattice((24, 20), beta=0.42, C=4.1,
                             h=np.random.default_rng(5).normal(0, 0.05, 480) if site else 0.04)

    def make(run):
        return ihmc.DenseChains(ctx, model, [run]) if dense else ihmc.Chains(ctx, [model], [run])

    run = ihmc.Run(n_md=6, n_traj=10, seed=12, chain_id=3, form=ihmc.FORM_SHIFTED)
    ref = make(run)
    ref.advance(10)
    want = ref.result(0)
    ref.close()
    a = make(run)
    a.advance(4)
    blob = a.checkpoint(0)
    a.close()
    b = make(run)
    b.restore(0, blob)
    b.advance(6)
    got = b.result(0)
    b.close()
    for k in ("dH", "accepted", "m", "m2c", "beta_eps", "psi_final"):
        assert np.array_equal(got[k], want[k]), k
    other = make(ihmc.Run(n_md=6, n_traj=10, seed=12, chain_id=3, form=ihmc.FORM_PSI))
    with pytest.raises(ihmc.IhmcError):
        other.restore(0, blob)
    other.close()


@pytest.mark.parametrize("h", ["uniform", "site"])
def test_fp32_statistics_4x4(ctx, h):
    """FP32 shifted-form chains are exact HMC: 4x4 at beta 0.4 against enumeration (4 sigma),
    a uniform field (in-cosh operand) and a per-site one (translated coordinates)."""
    from paper_1912_03278_amd import ihmc
    from oracle import exact as E
    from oracle import stats as S
    hv = 0.1 if h == "uniform" else np.random.default_rng(6).normal(0.05, 0.1, 16)
    ex = E.brute_force(E.torus_adjacency((4, 4)), 0.4, h=hv)
    g = ctx.run_lattice(ihmc.Lattice((4, 4), beta=0.4, C=4.1, h=hv),
                        ihmc.Run(n_md=10, n_traj=30000, precision=4, seed=3, form=ihmc.FORM_SHIFTED),
                        want_psi=False)
    for k, ref in (("beta_eps", ex["be"]), ("m", ex["m"]), ("m2c", ex["m2"])):
        st = S.gamma_method(g[k][500:])
        assert abs(st["mean"] - ref) < 4 * st["err"], (k, st, ref)
    st = S.gamma_method(np.exp(-g["dH"][500:]))
    assert abs(st["mean"] - 1) < 4 * st["err"]


def test_no_trajectories(ctx):
    """n_traj = 0: empty series, the summary of nothing, the starting field back."""
    from paper_1912_03278_amd import ihmc
    psi0 = np.random.default_rng(1).standard_normal(120)
    for h in (0.05, np.random.default_rng(2).normal(0, 0.1, 120)):
        g = ctx.run_lattice(ihmc.Lattice((12, 10), beta=0.4, C=4.1, h=h),
                            ihmc.Run(n_md=5, n_traj=0, precision=8, psi0=psi0, form=ihmc.FORM_SHIFTED))
        assert g["n_traj_done"] == 0 and g["acceptance"] == 0.0 and len(g["dH"]) == 0
        assert np.max(np.abs(g["psi_final"] - psi0)) < 1e-14


def test_refusals(ctx):
    from paper_1912_03278_amd import ihmc
    site = ihmc.Lattice((16, 16), beta=0.4, C=4.1, h=np.full(256, 0.01))
    with pytest.raises(ihmc.IhmcError):  # flips with a nonzero per-site field
        ctx.run_lattice(site, ihmc.Run(n_md=4, n_traj=2, flip_every=1, form=ihmc.FORM_SHIFTED))
    sv = ihmc.Server(ctx, budget_bytes=1 << 20, max_active=2)
    with pytest.raises(ihmc.IhmcError):  # flips at h != 0, served
        sv.submit(site, ihmc.Run(n_md=4, n_traj=2, flip_every=1, form=ihmc.FORM_SHIFTED))
    sv.close()
    uni = ihmc.Lattice((16, 16), beta=0.4, C=4.1, h=0.01)
    with pytest.raises(ihmc.IhmcError):
        ctx.run_lattice(uni, ihmc.Run(n_md=4, n_traj=2, flip_every=1, form=ihmc.FORM_SHIFTED))
    with pytest.raises(ihmc.IhmcError):
        ctx.run_lattice(uni, ihmc.Run(n_md=4, n_traj=1, form=3))
    K = (np.ones((8, 8)) - np.eye(8)) / 8
    with pytest.raises(ihmc.IhmcError):  # flips at h != 0 in the shifted form
        ctx.run_dense(ihmc.Dense(K, beta=0.5, C=1.2, h=0.1),
                      [ihmc.Run(n_md=4, n_traj=2, flip_every=1, form=ihmc.FORM_SHIFTED)])
    with pytest.raises(ihmc.IhmcError):
        ctx.run_dense(ihmc.Dense(K, beta=0.5, C=1.2), [ihmc.Run(n_md=4, n_traj=1, form=ihmc.FORM_PHI)])
    ctx.run_dense(ihmc.Dense(K, beta=0.5, C=1.2), [ihmc.Run(n_md=4, n_traj=2, flip_every=1, form=ihmc.FORM_SHIFTED)])
    sv = ihmc.Server(ctx, budget_bytes=1 << 20, max_active=2)
    with pytest.raises(ihmc.IhmcError):
        sv.submit(ihmc.Lattice((16, 16), beta=0.4, C=4.1), ihmc.Run(n_md=4, n_traj=1, precision=8, form=ihmc.FORM_PHI))
    sv.close()
