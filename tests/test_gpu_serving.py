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


def _tiled_requests(n, seed):
    """Requests too large for one workgroup's LDS (2D L 72..128, 3D L 18..40), so
    they run the tiled passes: two-step 2D launches, per-request partial-sum
    tables at reused slots, last passes on the side stream beside other
    chains' passes."""
    from paper_1912_03278_amd import ihmc
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        d = 2 if i % 2 else 3
        L = tuple(int(v) for v in (rng.integers(72, 129, size=2) if d == 2 else rng.integers(18, 41, size=3)))
        N = int(np.prod(L))
        kind = i % 3
        h = None if kind == 0 else (float(rng.uniform(0, 0.1)) if kind == 1 else rng.normal(0, 0.05, N))
        lat = ihmc.Lattice(L, beta=float(rng.uniform(0.2, 0.6)), C=2 * d + 0.1, h=h)
        run = ihmc.Run(n_md=int(rng.integers(3, 12)), n_traj=int(rng.integers(2, 7)),
                       precision=ihmc.F64 if i % 4 == 0 else ihmc.F32, seed=23, chain_id=i,
                       integrator=ihmc.OMELYAN if i % 5 == 2 else ihmc.LEAPFROG, flip_every=2 if i % 3 == 1 else 0)
        out.append((lat, run))
    return out


def test_served_tiled_mix_equals_alone_bitwise(ctx):
    from paper_1912_03278_amd import ihmc
    reqs = _tiled_requests(14, 2)
    sv = ihmc.Server(ctx, budget_bytes=64 << 20, max_active=6)
    tickets = []
    for k, (lat, run) in enumerate(reqs):
        tickets.append(sv.submit(lat, run))
        if k % 4 == 3:
            time.sleep(0.01)  # later requests arrive while earlier ones run
    served = []
    for t in tickets:
        assert sv.wait(t, 300.0) == ihmc.REQ_DONE
        served.append(sv.fetch(t))
    st = sv.stats()
    sv.close()
    assert st["max_resident"] > 1
    for (lat, run), g in zip(reqs, served):
        alone = ctx.run_lattice(lat, run)
        for k in ("dH", "H_old", "H_new", "m", "beta_eps", "psi_final", "accepted", "flipped"):
            assert np.array_equal(g[k], alone[k]), (lat.L, k)


def test_served_results_against_oracle(ctx, orc):
    """Served requests of every kind (2D/3D, FP32/FP64, uniform and per-site
    field, flips, Omelyan; LDS-resident and tiled sizes), arriving together,
    against the FP64 oracle with the oracle's accept decisions replayed: final
    field and every H_old / H_new within 1e-5 (FP32) / 1e-12 (FP64)."""
    from paper_1912_03278_amd import ihmc
    rng = np.random.default_rng(7)
    specs = [((90, 75), 0.44, 4.1, None, 4, 3, 0, 0), ((21, 19, 20), 0.22, 6.1, 0.05, 4, 3, 1, 2),
             ((24, 30), 0.35, 4.1, "site", 8, 3, 0, 3), ((9, 10, 11), 0.3, 6.1, "site", 8, 4, 0, 0),
             ((80, 96), 0.5, 4.1, 0.08, 8, 4, 1, 2), ((40, 33), 0.41, 4.1, None, 4, 3, 0, 1),
             ((19, 22, 18), 0.25, 6.1, "site", 4, 2, 1, 0)]
    reqs = []
    for i, (L, beta, C, h, prec, n_traj, integ, flip) in enumerate(specs):
        N = int(np.prod(L))
        if isinstance(h, str):
            h = rng.normal(0, 0.1, N)
        psi0 = rng.standard_normal(N)
        if prec == 4:
            psi0 = psi0.astype(np.float32).astype(np.float64)
        n_md = 5 if integ == 0 else 3
        r = orc.run(orc.Lattice(L, beta=beta, C=C, h=h), n_traj, n_md, seed=31, chain_id=i, psi0=psi0,
                    flip_every=flip, integrator=integ)
        run = ihmc.Run(n_md=n_md, n_traj=n_traj, precision=prec, seed=31, chain_id=i, psi0=psi0, flip_every=flip,
                       integrator=integ, replay_accept=r.accepted)
        reqs.append((ihmc.Lattice(L, beta=beta, C=C, h=h), run, r, prec))
    sv = ihmc.Server(ctx, budget_bytes=64 << 20, max_active=4)
    tickets = [sv.submit(lat, run) for lat, run, _, _ in reqs]
    for (lat, run, r, prec), t in zip(reqs, tickets):
        assert sv.wait(t, 300.0) == ihmc.REQ_DONE
        g = sv.fetch(t)
        tol = 1e-12 if prec == 8 else 1e-5
        assert np.array_equal(g["accepted"], r.accepted)
        assert np.array_equal(g["flipped"], r.flipped), lat.L
        assert nrm(g["psi_final"], r.psi_final) < tol, (lat.L, nrm(g["psi_final"], r.psi_final))
        assert np.all(np.abs(g["H_old"] - r.H_old) <= tol * np.abs(r.H_old)), lat.L
        assert np.all(np.abs(g["H_new"] - r.H_new) <= tol * np.abs(r.H_new)), lat.L
    sv.close()


def nrm(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def _same(a, b, keys=("dH", "H_old", "H_new", "m", "abs_m", "m2c", "beta_eps", "accepted", "flipped", "psi_final")):
    for k in keys:
        assert np.array_equal(a[k], b[k]), k
    assert a["n_traj_done"] == b["n_traj_done"]
    assert a["acceptance"] == b["acceptance"]


@pytest.mark.parametrize("case", ["2d_tiled_site_field", "3d_flips_f64", "2d_resident_omelyan",
                                  "2d_shifted_site_field", "3d_shifted_uniform"])
def test_checkpoint_running_request_and_resume_elsewhere(ctx, case):
    """Kill-and-resume by ticket: checkpoint a running request, cancel it (as a
    killed server would lose it), restore the checkpoint into another server on
    another context; the resumed request's results equal the uninterrupted
    run bit for bit."""
    from paper_1912_03278_amd import ihmc
    rng = np.random.default_rng(3)
    if case == "2d_tiled_site_field":
        lat = ihmc.Lattice((96, 80), beta=0.42, C=4.1, h=rng.normal(0, 0.05, 96 * 80))
        run = ihmc.Run(n_md=6, n_traj=40, precision=ihmc.F32, seed=5, chain_id=1)
    elif case == "3d_flips_f64":
        lat = ihmc.Lattice((20, 18, 21), beta=0.25, C=6.1, h=0.03)
        run = ihmc.Run(n_md=5, n_traj=40, precision=ihmc.F64, seed=5, chain_id=2, flip_every=3)
    elif case == "2d_resident_omelyan":
        lat = ihmc.Lattice((30, 30), beta=0.44, C=4.1)
        run = ihmc.Run(n_md=3, n_traj=400, precision=ihmc.F32, seed=5, chain_id=3, integrator=ihmc.OMELYAN)
    elif case == "2d_shifted_site_field":  # the shifted form's per-site field: translated coordinates
        lat = ihmc.Lattice((72, 64), beta=0.42, C=4.1, h=rng.normal(0, 0.05, 72 * 64))
        run = ihmc.Run(n_md=6, n_traj=40, precision=ihmc.F64, seed=5, chain_id=4, form=ihmc.FORM_SHIFTED)
    else:
        lat = ihmc.Lattice((18, 16, 20), beta=0.24, C=6.1, h=0.04)
        run = ihmc.Run(n_md=5, n_traj=40, precision=ihmc.F32, seed=5, chain_id=5, form=ihmc.FORM_SHIFTED)
    whole = ctx.run_lattice(lat, run)
    sv = ihmc.Server(ctx, budget_bytes=64 << 20, max_active=4)
    t = sv.submit(lat, run)
    t0 = time.time()
    while sv.info(t)["done"] < 2 and time.time() - t0 < 60:
        time.sleep(0.001)
    blob = sv.checkpoint(t)
    sv.cancel(t)
    sv.wait(t, 60.0)
    sv.close()
    with ihmc.Context(arena_bytes=256 << 20) as ctx2:
        sv2 = ihmc.Server(ctx2, budget_bytes=64 << 20, max_active=4)
        t2 = sv2.restore(blob)
        assert sv2.wait(t2, 120.0) == ihmc.REQ_DONE
        res = sv2.fetch(t2)
        sv2.close()
    _same(res, whole)


def test_checkpoint_queued_and_finished_requests(ctx):
    """A queued request's checkpoint is the request itself (its given initial
    field included); a finished one's restores to a finished request with the
    same results."""
    from paper_1912_03278_amd import ihmc
    rng = np.random.default_rng(4)
    sv = ihmc.Server(ctx, budget_bytes=64 << 20, max_active=1)
    blocker = sv.submit(ihmc.Lattice((96, 96), beta=0.4, C=4.1), ihmc.Run(n_md=10, n_traj=3000, seed=2))
    lat = ihmc.Lattice((33, 17), beta=0.4, C=4.1, h=rng.normal(0, 0.1, 33 * 17))
    run = ihmc.Run(n_md=4, n_traj=9, seed=6, chain_id=4, psi0=rng.standard_normal(33 * 17))
    q = sv.submit(lat, run)
    t0 = time.time()
    while sv.poll(blocker) != ihmc.REQ_RUNNING and time.time() - t0 < 30:
        time.sleep(0.002)
    assert sv.poll(q) == ihmc.REQ_QUEUED
    blob_q = sv.checkpoint(q)
    sv.cancel(q)
    sv.cancel(blocker)
    whole = ctx.run_lattice(lat, run)
    sv2 = ihmc.Server(ctx, budget_bytes=64 << 20, max_active=4)
    t = sv2.restore(blob_q)
    assert sv2.wait(t, 60.0) == ihmc.REQ_DONE
    blob_done = sv2.checkpoint(t)
    _same(sv2.fetch(t), whole)
    t3 = sv2.restore(blob_done)
    assert sv2.wait(t3, 60.0) == ihmc.REQ_DONE
    assert sv2.info(t3)["done"] == run.n_traj
    _same(sv2.fetch(t3), whole)
    sv2.close()
    sv.close()


def test_restore_rejects_bad_checkpoints(ctx):
    from paper_1912_03278_amd import ihmc
    sv = ihmc.Server(ctx, budget_bytes=64 << 20, max_active=4)
    t = sv.submit(ihmc.Lattice((40, 40), beta=0.4, C=4.1, h=0.02), ihmc.Run(n_md=4, n_traj=5, seed=1))
    assert sv.wait(t, 60.0) == ihmc.REQ_DONE
    blob = sv.checkpoint(t)
    sv.fetch(t)
    for bad in (blob[:-1], blob + b"\0", b"x" * len(blob), blob[:40]):
        with pytest.raises(ihmc.IhmcError) as e:
            sv.restore(bad)
        assert e.value.code == -1
    # a chain state that does not belong to the request's parameters
    tampered = bytearray(blob)
    # the request's beta sits after the magic, version words, ndim, L and J
    import struct
    off = 8 + 4 + 4 + 4 + 12 + 8
    beta = struct.unpack_from("<d", tampered, off)[0]
    assert beta == pytest.approx(0.4)
    struct.pack_into("<d", tampered, off, 0.41)
    t2 = sv.restore(bytes(tampered))
    assert sv.wait(t2, 60.0) == ihmc.REQ_FAILED
    with pytest.raises(ihmc.IhmcError):
        sv.fetch(t2)
    with pytest.raises(ihmc.IhmcError):
        sv.checkpoint(12345)
    sv.close()
