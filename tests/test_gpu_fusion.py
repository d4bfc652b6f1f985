"""Two middle leap-frog steps per launch (2D tiled chains) against one per launch.

The fused launch evaluates the first step on the tile plus a 2-wide ring and the
second on the tile, with the per-site arithmetic of the one-step pass, so every
series, the summary and the final field must be bit-identical with fusion on and
off (np.array_equal): ragged lattices, lattices smaller than the halo, every 2D
tile class, FP32 and FP64, uniform and per-site fields, both integrators, flips,
and sets whose chains have uneven step counts (even and odd numbers of middle
steps, a chain with none), so that pairs, single middle steps and last passes
of different chains share launches.  Parity with the FP64 oracle is covered by
the lattice test module, which runs with fusion on (the default).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SERIES = ("dH", "H_old", "H_new", "m", "abs_m", "m2c", "beta_eps", "accepted", "flipped", "psi_final")


@pytest.fixture(scope="module")
def ctxs():
    from paper_1912_03278_amd import ihmc
    fused = ihmc.Context(arena_bytes=512 << 20, resident=0)
    plain = ihmc.Context(arena_bytes=512 << 20, resident=0, fuse_steps=False)
    yield fused, plain
    fused.close()
    plain.close()


def same(a, b):
    for k in SERIES:
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    for k in ("acceptance", "mean_exp_minus_dH", "n_nonfinite", "n_traj_done"):
        assert a[k] == b[k], k


def run_both(ctxs, lats, runs, n):
    from paper_1912_03278_amd import ihmc
    out = []
    for ctx in ctxs:
        ch = ihmc.Chains(ctx, lats, runs)
        assert all(ch.group_info(g)["cls"] >= 0 for g in range(ch.groups()))
        ch.advance(n)
        out.append([ch.result(i) for i in range(len(lats))])
        ch.close()
    return out


CASES = [
    # (L, beta, C, h, precision, integrator, flip_every, n_md, tile class)
    ((33, 17), 0.44, 4.1, "site", 4, 0, 0, 7, 1),
    ((64, 64), 0.44, 4.1, None, 4, 0, 0, 8, 0),
    ((5, 7), 0.45, 4.3, 0.05, 4, 0, 0, 6, 1),
    ((3, 3), 0.40, 4.1, None, 8, 0, 0, 5, 1),
    ((70, 21), 0.42, 4.1, "site", 4, 1, 3, 4, 0),
    ((100, 90), 0.44, 4.1, 0.02, 8, 0, 0, 9, 2),
    ((130, 35), 0.44, 4.1, "site", 4, 0, 2, 6, 2),
    ((66, 3), 0.40, 4.2, None, 4, 1, 0, 3, 0),
    ((19, 4), 0.44, 4.1, "site", 8, 1, 0, 5, 1),
]


@pytest.mark.parametrize("k", range(len(CASES)))
def test_fused_equals_one_step_per_launch(ctxs, k):
    from paper_1912_03278_amd import ihmc
    L, beta, C, h, prec, integ, flip, n_md, cls = CASES[k]
    N = int(np.prod(L))
    hv = np.random.default_rng(k).normal(0, 0.1, N) if h == "site" else h
    lat = ihmc.Lattice(L, beta=beta, C=C, h=hv)
    for ctx in ctxs:
        ctx.pin_tile(lat, cls, prec)
    run = ihmc.Run(n_md=n_md, n_traj=10, precision=prec, integrator=integ, flip_every=flip, seed=5, chain_id=k)
    a, b = run_both(ctxs, [lat], [run], 10)
    same(a[0], b[0])
    for ctx in ctxs:
        assert ctx.tile_class(lat, prec)["cls"] == cls
    assert 0.0 < a[0]["acceptance"] <= 1.0


def test_uneven_step_counts_share_launches(ctxs):
    """One launch group with step counts 1 .. 9 (leap-frog) and Omelyan chains:
    pairs, single middle steps and last passes of different chains overlap."""
    from paper_1912_03278_amd import ihmc
    rng = np.random.default_rng(7)
    lats, runs = [], []
    for i, n_md in enumerate((1, 2, 3, 4, 5, 6, 7, 8, 9, 2, 3)):
        L = (int(rng.integers(20, 90)), int(rng.integers(8, 70)))
        h = rng.normal(0, 0.05, L[0] * L[1]) if i % 3 == 0 else 0.01 * i
        lats.append(ihmc.Lattice(L, beta=float(rng.uniform(0.3, 0.5)), C=4.1, h=h))
        runs.append(ihmc.Run(n_md=n_md, n_traj=6, seed=2, chain_id=i, integrator=1 if i >= 9 else 0,
                             flip_every=2 if i == 4 else 0))
    a, b = run_both(ctxs, lats, runs, 6)
    for i in range(len(lats)):
        same(a[i], b[i])


def test_mixed_2d_3d_set(ctxs):
    from paper_1912_03278_amd import ihmc
    lats = [ihmc.Lattice((48, 40), beta=0.44, C=4.1), ihmc.Lattice((12, 10, 9), beta=0.22, C=6.1, h=0.03),
            ihmc.Lattice((17, 30), beta=0.4, C=4.1, h=0.02)]
    runs = [ihmc.Run(n_md=6 + i, n_traj=5, seed=4, chain_id=i, precision=8 if i == 2 else 4) for i in range(3)]
    a, b = run_both(ctxs, lats, runs, 5)
    for i in range(3):
        same(a[i], b[i])


def test_checkpoint_crosses_fusion(ctxs):
    """A checkpoint taken with one step per launch resumes on the fused path."""
    from paper_1912_03278_amd import ihmc
    fused, plain = ctxs
    lat = ihmc.Lattice((40, 24), beta=0.44, C=4.1, h=0.01)
    run = ihmc.Run(n_md=7, n_traj=8, seed=6, chain_id=1, flip_every=3)
    ref = ihmc.Chains(plain, [lat], [run])
    ref.advance(8)
    want = ref.result(0)
    ref.close()
    a = ihmc.Chains(plain, [lat], [run])
    a.advance(3)
    blob = a.checkpoint(0)
    a.close()
    b = ihmc.Chains(fused, [lat], [run])
    b.restore(0, blob)
    b.advance(5)
    same(b.result(0), want)
    b.close()


def test_time_pair(ctxs):
    from paper_1912_03278_amd import ihmc
    fused, _ = ctxs
    ch = ihmc.Chains(fused, [ihmc.Lattice((128, 64), beta=0.44, C=4.1)], [ihmc.Run(n_md=6, n_traj=1)])
    t1 = ch.time_pass(0, mode=ihmc.MIDDLE, reps=5)
    t2 = ch.time_pass(0, mode=ihmc.PAIR, reps=5)
    assert t1["us"] > 0 and t2["us"] > 0 and t2["sites"] == 128 * 64
    ch.close()
    short = ihmc.Chains(fused, [ihmc.Lattice((32, 32), beta=0.44, C=4.1)], [ihmc.Run(n_md=2, n_traj=1)])
    with pytest.raises(ihmc.IhmcError):
        short.time_pass(0, mode=ihmc.PAIR, reps=1)  # one middle step only
    short.close()
    cube = ihmc.Chains(fused, [ihmc.Lattice((16, 16, 16), beta=0.22, C=6.1)], [ihmc.Run(n_md=6, n_traj=1)])
    with pytest.raises(ihmc.IhmcError):
        cube.time_pass(0, mode=ihmc.PAIR, reps=1)  # 3D stays one step per launch
    cube.close()


def test_large_launch_one_thread_per_quad(ctxs):
    """A launch of more tiles than give every SIMD eight waves keeps one thread
    per tile quad; smaller launches (every case above) take two.  Both must
    equal one step per launch."""
    from paper_1912_03278_amd import ihmc
    lat = ihmc.Lattice((2048, 1040), beta=0.44, C=4.1, h=0.01)  # 2080 tiles of 64 x 16
    for ctx in ctxs:
        ctx.pin_tile(lat, 0)
    run = ihmc.Run(n_md=5, n_traj=3, seed=9, chain_id=3)
    a, b = run_both(ctxs, [lat], [run], 3)
    same(a[0], b[0])
    assert a[0]["n_traj_done"] == 3 and np.all(np.isfinite(a[0]["dH"]))
