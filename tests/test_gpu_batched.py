"""The batched form at its full size: 4096 uneven 2D chains with per-site fields.

One trajectory of every chain runs in the launch configuration the benchmark
times; sampled chains are checked against the FP64 oracle (1e-5 normwise on the
final field, FP32 state) and bitwise against the same chain run alone.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def nrm(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.fixture(scope="module")
def full_batch():
    from paper_1912_03278_amd import ihmc, inputs
    ctx = ihmc.Context(arena_bytes=6 << 30)
    ws = inputs.batched()
    lats = [ihmc.Lattice(w["L"], beta=w["beta"], C=w["C"], h=w["h"]) for w in ws]
    runs = [ihmc.Run(n_md=w["n_md"], n_traj=2, precision=ihmc.F32, seed=w["seed"], chain_id=w["chain_id"],
                     replay_accept=[1, 1]) for w in ws]
    ch = ihmc.Chains(ctx, lats, runs)
    ch.advance(2)
    yield ctx, ws, lats, runs, ch
    ch.close()
    ctx.close()


def _sample(ws):
    sizes = np.array([w["L"][0] for w in ws])
    order = np.argsort(sizes, kind="stable")
    return [int(order[0]), int(order[len(order) // 2]), int(order[-1])]


def test_sampled_chains_match_oracle(full_batch, orc):
    ctx, ws, lats, runs, ch = full_batch
    for i in _sample(ws):
        w = ws[i]
        N = w["L"][0] * w["L"][1]
        psi0 = orc.normals(w["seed"], w["chain_id"], 0, orc.TAG_INIT, N).astype(np.float32).astype(np.float64)
        r = orc.run(orc.Lattice(w["L"], beta=w["beta"], C=w["C"], h=w["h"]), 2, w["n_md"], seed=w["seed"],
                    chain_id=w["chain_id"], psi0=psi0, replay_accept=[1, 1])
        g = ch.result(i)
        assert nrm(g["psi_final"], r.psi_final) < 1e-5, (i, w["L"], w["n_md"])
        assert np.allclose(g["H_new"], r.H_new, rtol=1e-5, atol=0)
        # the estimators of the accepted field (FP64 sums of the FP32 state)
        assert np.allclose(g["beta_eps"], r.beta_eps, rtol=0, atol=1e-5)


def test_sampled_chains_bitwise_equal_alone(full_batch):
    from paper_1912_03278_amd import ihmc
    ctx, ws, lats, runs, ch = full_batch
    for i in _sample(ws)[1:]:
        alone = ctx.run_lattice(lats[i], runs[i])
        b = ch.result(i)
        for k in ("dH", "H_old", "beta_eps", "m", "psi_final"):
            assert np.array_equal(alone[k], b[k]), (i, k)


def _batched_run(ctx, ws, n_traj):
    from paper_1912_03278_amd import ihmc
    lats = [ihmc.Lattice(w["L"], beta=w["beta"], C=w["C"], h=w["h"]) for w in ws]
    runs = [ihmc.Run(n_md=w["n_md"], n_traj=n_traj, precision=ihmc.F32, seed=w["seed"], chain_id=w["chain_id"])
            for w in ws]
    ch = ihmc.Chains(ctx, lats, runs)
    ch.advance(n_traj)
    return ch, lats, runs


def test_batched_rerun_is_bitwise_deterministic():
    """Natural accept decisions over several trajectories: two runs of the full
    batch agree bit for bit (a race between concurrent launches would show here)."""
    from paper_1912_03278_amd import ihmc, inputs
    ctx = ihmc.Context(arena_bytes=6 << 30)
    ws = inputs.batched()
    a, _, _ = _batched_run(ctx, ws, 6)
    ra = [a.result(i, want_psi=False)["dH"] for i in range(0, len(ws), 97)]
    a.close()
    b, _, _ = _batched_run(ctx, ws, 6)
    rb = [b.result(i, want_psi=False)["dH"] for i in range(0, len(ws), 97)]
    b.close()
    ctx.close()
    bad = [k for k, (x, y) in enumerate(zip(ra, rb)) if not np.array_equal(x, y)]
    assert not bad, bad


def test_batched_equals_alone_natural_decisions():
    from paper_1912_03278_amd import ihmc, inputs
    ctx = ihmc.Context(arena_bytes=6 << 30)
    ws = inputs.batched()
    ch, lats, runs = _batched_run(ctx, ws, 6)
    diffs = []
    for i in (0, 1, 2, 500, 1234, 4095):
        alone = ctx.run_lattice(lats[i], runs[i], want_psi=False)
        b = ch.result(i, want_psi=False)
        if not (np.array_equal(alone["dH"], b["dH"]) and np.array_equal(alone["beta_eps"], b["beta_eps"])):
            diffs.append((i, ws[i]["L"], ws[i]["n_md"], alone["dH"].tolist(), b["dH"].tolist()))
    ch.close()
    ctx.close()
    assert not diffs, diffs
