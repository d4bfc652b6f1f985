"""The serving loop: continuous batching of lattice requests on one GPU.

Requests of mixed dimension, size, precision, field and length arrive while
others run; each served result must be bit-identical to the same request run
alone (the per-chain arithmetic does not depend on the other chains of a
launch), admission must respect the device budget, and cancellation, waiting
and error paths must behave as the C ABI states.
"""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1912_03278_amd import ihmc
    c = ihmc.Context(arena_bytes=1 << 30)
    yield c
    c.close()


def _requests(n, seed):
    from paper_1912_03278_amd import ihmc
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        d = 2 if i % 3 else 3
        L = tuple(int(v) for v in (rng.integers(5, 48, size=2) if d == 2 else rng.integers(4, 14, size=3)))
        N = int(np.prod(L))
        kind = i % 4
        h = None if kind == 0 else (float(rng.uniform(0, 0.1)) if kind < 3 else rng.normal(0, 0.05, N))
        lat = ihmc.Lattice(L, beta=float(rng.uniform(0.2, 0.6)), C=2 * d + 0.1, h=h)
        run = ihmc.Run(n_md=int(rng.integers(3, 12)), n_traj=int(rng.integers(2, 14)),
                       precision=ihmc.F64 if i % 5 == 0 else ihmc.F32, seed=17, chain_id=i,
                       integrator=ihmc.OMELYAN if i % 7 == 3 else ihmc.LEAPFROG, flip_every=3 if i % 6 == 1 else 0)
        out.append((lat, run))
    return out


def test_served_results_equal_alone_bitwise(ctx):
    from paper_1912_03278_amd import ihmc
    reqs = _requests(30, 1)
    sv = ihmc.Server(ctx, budget_bytes=6 << 20, max_active=8)
    tickets = []
    for k, (lat, run) in enumerate(reqs):
        tickets.append(sv.submit(lat, run))
        if k % 10 == 9:
            time.sleep(0.02)  # later requests arrive while earlier ones run
    served = []
    for t in tickets:
        assert sv.wait(t, 120.0) == ihmc.REQ_DONE
        served.append(sv.fetch(t))
    st = sv.stats()
    sv.close()
    assert st["completed"] == len(reqs)
    assert 1 < st["max_resident"] <= 8
    assert st["site_md_steps"] == sum(lat.N * run.n_md * run.n_traj for lat, run in reqs)
    for (lat, run), g in zip(reqs, served):
        alone = ctx.run_lattice(lat, run)
        for k in ("dH", "m", "beta_eps", "psi_final", "accepted", "flipped"):
            assert np.array_equal(g[k], alone[k]), (lat.L, k)
        assert g["n_traj_done"] == run.n_traj
        assert g["t_submit"] <= g["t_admit"] <= g["t_done"]


def test_budget_admission_and_queueing(ctx):
    """A budget that holds about one request at a time still completes every request."""
    from paper_1912_03278_amd import ihmc
    lat = ihmc.Lattice((64, 64), beta=0.4, C=4.1, h=0.02)
    sv = ihmc.Server(ctx, budget_bytes=150 << 10, max_active=64)
    tickets = [sv.submit(lat, ihmc.Run(n_md=4, n_traj=3, seed=1, chain_id=i)) for i in range(6)]
    res = [sv.fetch(t) if sv.wait(t, 60.0) == ihmc.REQ_DONE else None for t in tickets]
    st = sv.stats()
    sv.close()
    assert all(r is not None for r in res)
    assert st["max_resident"] == 1
    # admitted one after another, in arrival order
    admits = [r["t_admit"] for r in res]
    assert admits == sorted(admits)
    for a, b in zip(res, res[1:]):
        assert b["t_admit"] >= a["t_done"] - 1e-3


def test_oversized_request_is_rejected(ctx):
    from paper_1912_03278_amd import ihmc
    sv = ihmc.Server(ctx, budget_bytes=1 << 20, max_active=4)
    with pytest.raises(ihmc.IhmcError) as e:
        sv.submit(ihmc.Lattice((512, 512), beta=0.4, C=4.1), ihmc.Run(n_md=4, n_traj=2))
    assert e.value.code == -2
    with pytest.raises(ihmc.IhmcError) as e:
        sv.submit(ihmc.Lattice((16, 16), beta=0.4, C=3.9), ihmc.Run(n_md=4, n_traj=2))
    assert e.value.code == -1
    sv.close()


def test_cancel_queued_and_running(ctx):
    from paper_1912_03278_amd import ihmc
    sv = ihmc.Server(ctx, budget_bytes=64 << 20, max_active=1)
    long_run = sv.submit(ihmc.Lattice((96, 96), beta=0.4, C=4.1), ihmc.Run(n_md=10, n_traj=5000, seed=2))
    queued = sv.submit(ihmc.Lattice((16, 16), beta=0.4, C=4.1), ihmc.Run(n_md=4, n_traj=3, seed=2, chain_id=1))
    t0 = time.time()
    while sv.poll(long_run) != ihmc.REQ_RUNNING and time.time() - t0 < 30:
        time.sleep(0.005)
    assert sv.poll(queued) == ihmc.REQ_QUEUED
    sv.cancel(queued)
    assert sv.poll(queued) == ihmc.REQ_CANCELLED
    time.sleep(0.05)
    sv.cancel(long_run)
    assert sv.wait(long_run, 60.0) == ihmc.REQ_CANCELLED
    with pytest.raises(ihmc.IhmcError) as e:
        sv.fetch(long_run)
    assert e.value.code == -5
    with pytest.raises(ihmc.IhmcError) as e:
        sv.fetch(queued)
    assert e.value.code == -5
    # the server keeps serving after cancellations
    t = sv.submit(ihmc.Lattice((16, 16), beta=0.4, C=4.1), ihmc.Run(n_md=4, n_traj=3, seed=2, chain_id=2))
    assert sv.wait(t, 30.0) == ihmc.REQ_DONE
    assert sv.fetch(t)["n_traj_done"] == 3
    sv.close()


def test_fetch_before_done_and_unknown_ticket(ctx):
    from paper_1912_03278_amd import ihmc
    sv = ihmc.Server(ctx, budget_bytes=64 << 20, max_active=4)
    t = sv.submit(ihmc.Lattice((128, 128), beta=0.4, C=4.1), ihmc.Run(n_md=10, n_traj=400, seed=3))
    with pytest.raises(ihmc.IhmcError) as e:
        sv.fetch(t)
    assert e.value.code == -3
    assert sv.wait(t, 120.0) == ihmc.REQ_DONE
    assert sv.fetch(t, want_psi=False)["n_traj_done"] == 400
    with pytest.raises(ihmc.IhmcError):
        sv.poll(t)  # released by the fetch
    sv.close()


def test_destroy_with_pending_requests(ctx):
    from paper_1912_03278_amd import ihmc
    sv = ihmc.Server(ctx, budget_bytes=64 << 20, max_active=2)
    for i in range(5):
        sv.submit(ihmc.Lattice((64, 64), beta=0.4, C=4.1), ihmc.Run(n_md=8, n_traj=1000, seed=4, chain_id=i))
    time.sleep(0.05)
    sv.close()  # cancels and releases everything
    used, _ = ctx.memory()
    assert used < (1 << 20)
