"""Checkpoint and resume of chains, and the thermalisation cut of the summary.

The random numbers of a trajectory are Philox draws at counters that name the
trajectory, so a chain resumed from a checkpoint after k trajectories must
continue bit for bit as the uninterrupted chain: the whole series (records of
the first k come from the checkpoint, the rest are recomputed), the summary
and the final field are compared with np.array_equal.  Error cases: a
truncated or foreign buffer, a chain with other parameters, a capacity that
does not cover the trajectories already done.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SERIES = ("dH", "H_old", "H_new", "m", "abs_m", "m2c", "beta_eps", "accepted", "flipped", "psi_final")


@pytest.fixture(scope="module")
def ctx():
    from paper_1912_03278_amd import ihmc
    c = ihmc.Context(arena_bytes=512 << 20)
    yield c
    c.close()


def same(a, b):
    for k in SERIES:
        assert np.array_equal(a[k], b[k]), k
    for k in ("acceptance", "mean_exp_minus_dH", "n_nonfinite", "n_traj_done"):
        assert a[k] == b[k], k


CASES = [
    # (lattice, h, beta, C, precision, integrator, flip_every)
    ((33, 17), "site", 0.44, 4.1, 4, 0, 0),
    ((20, 6, 9), 0.05, 0.22, 6.1, 8, 1, 3),
    ((12, 12), None, 0.40, 4.1, 8, 0, 2),
]


@pytest.mark.parametrize("case", CASES, ids=["2d_f32_site_h", "3d_f64_omelyan_flips", "2d_f64_flips"])
def test_resume_equals_uninterrupted(ctx, case):
    from paper_1912_03278_amd import ihmc
    L, h, beta, C, prec, integ, flip = case
    N = int(np.prod(L))
    hv = np.random.default_rng(3).normal(0, 0.1, N) if h == "site" else h
    k = 7
    lat = ihmc.Lattice(L, beta=beta, C=C, h=hv)
    run = ihmc.Run(n_md=6, n_traj=2 * k, precision=prec, integrator=integ, flip_every=flip, seed=11, chain_id=4)
    ref = ihmc.Chains(ctx, [lat], [run])
    ref.advance(2 * k)
    full = ref.result(0)
    ref.close()

    first = ihmc.Chains(ctx, [lat], [run])
    first.advance(k)
    blob = first.checkpoint(0)
    half = first.result(0)
    first.close()
    assert half["n_traj_done"] == k

    second = ihmc.Chains(ctx, [lat], [run])
    second.restore(0, blob)
    second.advance(k)
    same(second.result(0), full)
    # the capacity counts from the checkpoint's trajectory index
    with pytest.raises(ihmc.IhmcError):
        second.advance(1)
    second.close()


def test_restore_one_chain_of_a_batch(ctx):
    """A checkpoint restored into chain 1 of a mixed 2D/3D set; the other chains
    are unaffected and the restored one continues as if never stopped."""
    from paper_1912_03278_amd import ihmc
    lats = [ihmc.Lattice((16, 16), beta=0.4, C=4.1), ihmc.Lattice((8, 8, 8), beta=0.2, C=6.1),
            ihmc.Lattice((30, 10), beta=0.5, C=4.3, h=0.02)]
    runs = [ihmc.Run(n_md=5, n_traj=10, seed=2, chain_id=i) for i in range(3)]
    ref = ihmc.Chains(ctx, lats, runs)
    ref.advance(10)
    want = [ref.result(i) for i in range(3)]
    ref.close()

    a = ihmc.Chains(ctx, [lats[1]], [runs[1]])
    a.advance(4)
    blob = a.checkpoint(0)
    a.close()

    b = ihmc.Chains(ctx, lats, runs)
    b.restore(1, blob)  # chain 1 is now at trajectory 4, the others at 0
    b.advance(6)        # chain 1 reaches 10
    same(b.result(1), want[1])
    for i in (0, 2):
        r = b.result(i)
        assert r["n_traj_done"] == 6
        for key in ("dH", "m", "accepted"):
            assert np.array_equal(r[key][:6], want[i][key][:6]), (i, key)
    with pytest.raises(ihmc.IhmcError):
        b.advance(1)  # chain 1 is at its capacity
    b.close()


def test_dense_resume_equals_uninterrupted(ctx):
    from paper_1912_03278_amd import ihmc
    N = 200
    rng = np.random.default_rng(5)
    K = rng.normal(0, 1 / np.sqrt(N), (N, N))
    K = np.triu(K, 1)
    K = K + K.T
    model = ihmc.Dense(K, beta=1.0, C=-1.0)
    runs = [ihmc.Run(n_md=5, n_traj=8, seed=9, chain_id=i) for i in range(3)]
    ref = ihmc.DenseChains(ctx, model, runs)
    ref.advance(8)
    want = ref.result(2)
    ref.close()
    a = ihmc.DenseChains(ctx, model, runs)
    a.advance(3)
    blob = a.checkpoint(2)
    a.close()
    b = ihmc.DenseChains(ctx, model, runs)
    b.restore(2, blob)
    b.advance(5)
    same(b.result(2), want)
    b.close()
    # another choice of limb products is another force: refused
    c = ihmc.DenseChains(ctx, model, runs, products=3)
    with pytest.raises(ihmc.IhmcError):
        c.restore(2, blob)
    c.close()


def test_restore_rejects_bad_input(ctx):
    from paper_1912_03278_amd import ihmc
    lat = ihmc.Lattice((12, 10), beta=0.4, C=4.1)
    run = ihmc.Run(n_md=4, n_traj=6, seed=1, chain_id=0)
    a = ihmc.Chains(ctx, [lat], [run])
    a.advance(4)
    blob = a.checkpoint(0)
    a.close()

    def fresh(lat=lat, run=run):
        return ihmc.Chains(ctx, [lat], [run])

    bad = [
        blob[:-1],                                   # truncated
        blob + b"\0",                                # trailing bytes
        b"x" * len(blob),                            # not a checkpoint
        blob[:16],                                   # header only in part
    ]
    for data in bad:
        c = fresh()
        with pytest.raises(ihmc.IhmcError):
            c.restore(0, data)
        c.close()
    others = [
        (ihmc.Lattice((12, 10), beta=0.41, C=4.1), run),                  # other beta
        (ihmc.Lattice((10, 12), beta=0.4, C=4.1), run),                   # other shape
        (lat, ihmc.Run(n_md=4, n_traj=6, seed=2, chain_id=0)),            # other seed
        (lat, ihmc.Run(n_md=4, n_traj=6, seed=1, chain_id=1)),            # other stream
        (lat, ihmc.Run(n_md=5, n_traj=6, seed=1, chain_id=0)),            # other step count
        (lat, ihmc.Run(n_md=4, n_traj=6, seed=1, chain_id=0, precision=8)),  # other precision
        (lat, ihmc.Run(n_md=4, n_traj=3, seed=1, chain_id=0)),            # capacity below 4
    ]
    for l2, r2 in others:
        c = fresh(l2, r2)
        with pytest.raises(ihmc.IhmcError):
            c.restore(0, blob)
        c.close()
    # a failed restore leaves the chain as it was
    c = fresh()
    with pytest.raises(ihmc.IhmcError):
        c.restore(0, blob[:-1])
    c.advance(6)
    ref = fresh()
    ref.advance(6)
    same(c.result(0), ref.result(0))
    c.close()
    ref.close()


def test_n_therm_cuts_the_summary_only(ctx):
    from paper_1912_03278_amd import ihmc
    lat = ihmc.Lattice((10, 10), beta=0.44, C=4.1)
    base = dict(n_md=3, n_traj=40, seed=6, chain_id=1, precision=8)
    r0 = ihmc.Chains(ctx, [lat], [ihmc.Run(**base)])
    r0.advance(40)
    a = r0.result(0)
    r0.close()
    r1 = ihmc.Chains(ctx, [lat], [ihmc.Run(n_therm=15, **base)])
    r1.advance(40)
    b = r1.result(0)
    r1.close()
    for k in SERIES:
        assert np.array_equal(a[k], b[k]), k
    assert a["acceptance"] == pytest.approx(np.mean(a["accepted"]), abs=0)
    assert b["acceptance"] == pytest.approx(np.mean(b["accepted"][15:]), abs=1e-15)
    fin = np.isfinite(b["dH"][15:])
    assert b["mean_exp_minus_dH"] == pytest.approx(np.mean(np.exp(-b["dH"][15:][fin])), rel=1e-12)
    with pytest.raises(ihmc.IhmcError):
        ihmc.Chains(ctx, [lat], [ihmc.Run(n_therm=-1, **base)])
