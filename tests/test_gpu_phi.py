"""The inverse (phi) formulation on the GPU (eq. cosh_in_exponent), the A/B
baseline of the paper's substitution, against the phi-form oracle.

The GPU solves Kt x = phi by CG to a relative residual of 1e-14 at every
force evaluation, the oracle to 1e-15; with kappa(Kt) = (C + 2d)/(C - 2d) the
solutions differ by up to ~kappa 1e-14 relative, so one FP64 trajectory from
identical inputs is compared at 1e-10 (final field normwise, H_old and H_new
relative), not the psi form's 1e-12.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def nrm(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def ctx():
    from paper_1912_03278_amd import ihmc
    c = ihmc.Context(arena_bytes=512 << 20)
    yield c
    c.close()


CASES = [
    ("2d_ragged", (30, 17), 0.44, 4.1, None),
    ("2d_uniform_h", (24, 20), 0.35, 4.3, 0.07),
    ("2d_site_h", (21, 19), 0.5, 4.1, "site"),
    ("3d", (9, 10, 11), 0.22, 6.1, None),
    ("3d_site_h", (7, 6, 5), 0.25, 6.2, "site"),
]


def _case(case, seed):
    name, L, beta, C, h = case
    rng = np.random.default_rng(seed)
    N = int(np.prod(L))
    if isinstance(h, str):
        h = rng.normal(0, 0.2, N)
    return L, beta, C, h


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("given_start", [False, True])
def test_phi_one_trajectory(ctx, orc, case, given_start):
    from paper_1912_03278_amd import ihmc
    L, beta, C, h = _case(case, 1)
    olat = orc.Lattice(L, beta=beta, C=C, h=h)
    phi0 = orc.phi_start(olat, seed=3, chain_id=4) * 0.9 if given_start else None
    r = orc.run(olat, 1, 6, seed=3, chain_id=4, psi0=phi0, replay_accept=[1], form="phi")
    g = ctx.run_lattice(ihmc.Lattice(L, beta=beta, C=C, h=h),
                        ihmc.Run(n_md=6, n_traj=1, precision=ihmc.F64, seed=3, chain_id=4, psi0=phi0,
                                 replay_accept=[1], form=ihmc.FORM_PHI))
    assert nrm(g["psi_final"], r.psi_final) < 1e-10
    assert abs(g["H_old"][0] - r.H_old[0]) <= 1e-10 * abs(r.H_old[0])
    assert abs(g["H_new"][0] - r.H_new[0]) <= 1e-10 * abs(r.H_new[0])
    for k in ("m", "m2c", "beta_eps"):
        assert abs(g[k][0] - getattr(r, k)[0]) <= 1e-10 * max(1.0, abs(getattr(r, k)[0])), k
    assert g["cg_iterations"] > 7 * 5


def test_phi_natural_decisions_follow_oracle(ctx, orc):
    """FP64 on both sides: the accept decisions of 40 natural trajectories agree."""
    from paper_1912_03278_amd import ihmc
    L, beta, C, h = (16, 16), 0.44, 4.1, 0.02
    r = orc.run(orc.Lattice(L, beta=beta, C=C, h=h), 40, 8, seed=5, form="phi")
    g = ctx.run_lattice(ihmc.Lattice(L, beta=beta, C=C, h=h),
                        ihmc.Run(n_md=8, n_traj=40, precision=ihmc.F64, seed=5, form=ihmc.FORM_PHI))
    assert np.array_equal(g["accepted"], r.accepted)
    assert np.max(np.abs(g["dH"] - r.dH)) < 1e-8
    assert nrm(g["psi_final"], r.psi_final) < 1e-8


def test_phi_statistics_4x4_against_enumeration(ctx):
    from paper_1912_03278_amd import ihmc
    from oracle import exact as E
    from oracle import stats as S
    ex = E.brute_force(E.torus_adjacency((4, 4)), 0.4, h=0.1)
    g = ctx.run_lattice(ihmc.Lattice((4, 4), beta=0.4, C=4.1, h=0.1),
                        ihmc.Run(n_md=10, n_traj=40000, precision=ihmc.F64, seed=6, form=ihmc.FORM_PHI),
                        want_psi=False)
    for k, ref in (("beta_eps", ex["be"]), ("m2c", ex["m2"]), ("m", ex["m"])):
        st = S.gamma_method(g[k][500:])
        assert abs(st["mean"] - ref) < 4 * st["err"], (k, st, ref)


def test_phi_and_psi_chains_in_one_set_equal_alone(ctx):
    from paper_1912_03278_amd import ihmc
    rng = np.random.default_rng(2)
    lats = [ihmc.Lattice((20, 20), beta=0.4, C=4.1, h=rng.normal(0, 0.05, 400)),
            ihmc.Lattice((10, 9, 8), beta=0.22, C=6.1), ihmc.Lattice((33, 33), beta=0.44, C=4.1),
            ihmc.Lattice((70, 40), beta=0.4, C=4.1)]
    runs = [ihmc.Run(n_md=5, n_traj=6, precision=ihmc.F64, seed=8, chain_id=0, form=ihmc.FORM_PHI),
            ihmc.Run(n_md=4, n_traj=6, precision=ihmc.F64, seed=8, chain_id=1, form=ihmc.FORM_PHI),
            ihmc.Run(n_md=5, n_traj=6, precision=ihmc.F32, seed=8, chain_id=2),
            ihmc.Run(n_md=7, n_traj=6, precision=ihmc.F32, seed=8, chain_id=3)]
    both = ctx.run_batch(lats, runs)
    for i in range(len(lats)):
        alone = ctx.run_lattice(lats[i], runs[i])
        for k in ("dH", "H_old", "m", "beta_eps", "psi_final", "accepted"):
            assert np.array_equal(both[i][k], alone[k]), (i, k)
        assert (both[i]["cg_iterations"] > 0) == (runs[i].form == ihmc.FORM_PHI)


def test_phi_checkpoint_resume(ctx):
    from paper_1912_03278_amd import ihmc
    lat = ihmc.Lattice((25, 22), beta=0.42, C=4.1, h=0.03)
    run = ihmc.Run(n_md=5, n_traj=10, precision=ihmc.F64, seed=9, chain_id=1, form=ihmc.FORM_PHI)
    whole = ctx.run_lattice(lat, run)
    a = ihmc.Chains(ctx, [lat], [run])
    a.advance(4)
    blob = a.checkpoint(0)
    a.close()
    b = ihmc.Chains(ctx, [lat], [run])
    b.restore(0, blob)
    b.advance(6)
    res = b.result(0)
    b.close()
    for k in ("dH", "m", "beta_eps", "psi_final", "accepted"):
        assert np.array_equal(res[k], whole[k]), k
    # a psi-form chain of the same parameters refuses the phi checkpoint
    c = ihmc.Chains(ctx, [lat], [ihmc.Run(n_md=5, n_traj=10, precision=ihmc.F64, seed=9, chain_id=1)])
    with pytest.raises(ihmc.IhmcError):
        c.restore(0, blob)
    c.close()


def test_phi_refusals(ctx):
    from paper_1912_03278_amd import ihmc
    lat = ihmc.Lattice((16, 16), beta=0.4, C=4.1)
    bad = [ihmc.Run(n_md=4, n_traj=2, precision=ihmc.F32, form=ihmc.FORM_PHI),
           ihmc.Run(n_md=4, n_traj=2, precision=ihmc.F64, form=ihmc.FORM_PHI, flip_every=2),
           ihmc.Run(n_md=4, n_traj=2, precision=ihmc.F64, form=ihmc.FORM_PHI, integrator=ihmc.OMELYAN)]
    for run in bad:
        with pytest.raises(ihmc.IhmcError) as e:
            ctx.run_lattice(lat, run)
        assert e.value.code == -6
    with pytest.raises(ihmc.IhmcError) as e:  # beyond one workgroup's LDS
        ctx.run_lattice(ihmc.Lattice((40, 40), beta=0.4, C=4.1),
                        ihmc.Run(n_md=4, n_traj=2, precision=ihmc.F64, form=ihmc.FORM_PHI))
    assert e.value.code == -6
    with pytest.raises(ihmc.IhmcError) as e:
        ctx.run_lattice(lat, ihmc.Run(n_md=4, n_traj=2, precision=ihmc.F64, form=7))
    assert e.value.code == -1
    sv = ihmc.Server(ctx, budget_bytes=16 << 20, max_active=4)
    with pytest.raises(ihmc.IhmcError) as e:
        sv.submit(lat, ihmc.Run(n_md=4, n_traj=2, precision=ihmc.F64, form=ihmc.FORM_PHI))
    assert e.value.code == -6
    sv.close()
