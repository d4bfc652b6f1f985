"""Oracle parity at the single-large-chain workload's own shapes and launch
configuration, and at the paper's own shift.

* 2D 1024^2 at beta_c and 3D 128^3 at beta = 0.2216544, FP32 state, 20 MD
  steps, one chain set of both chains with tile classes from the autotuner at
  the workload's working set (the benchmark's configuration: 64x16 tiles with
  two middle steps per launch and two threads per tile quad, 32x8x8 boxes of
  512 threads; both chains close their sums in groups of 32 tiles).  One
  trajectory from an identical FP32 initial field and the Philox momenta:
  final field within 1e-5 normwise, H_old and H_new within 1e-5 relative.
* The paper's shift C = n + 1e-5 (Sec. 3, after eq. large C minima): K~ then
  has eigenvalues down to 1e-5, and in FP32 u = K~ psi on the staggered modes
  is a cancellation of O(1) terms.  The error of one FP32 trajectory against
  the FP64 oracle is measured and bounded here; FP64 state meets 1e-12.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def nrm(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def ctx():
    from paper_1912_03278_amd import ihmc
    c = ihmc.Context(arena_bytes=2 << 30)
    yield c
    c.close()


def test_large_workload_one_trajectory_fp32(ctx, orc):
    from paper_1912_03278_amd import ihmc, inputs
    ws = inputs.large()
    lats = [ihmc.Lattice(w["L"], beta=w["beta"], C=w["C"]) for w in ws]
    ctx.tune(lats)  # tile classes for the workload's working set
    classes = [ctx.tile_class(l, ihmc.F32)["cls"] for l in lats]
    psi0 = [orc.normals(w["seed"], w["chain_id"], 0, orc.TAG_INIT, int(np.prod(w["L"])))
            .astype(np.float32).astype(np.float64) for w in ws]
    refs = []
    for w, p0 in zip(ws, psi0):
        refs.append(orc.run(orc.Lattice(w["L"], beta=w["beta"], C=w["C"]), 1, w["n_md"], seed=w["seed"],
                            chain_id=w["chain_id"], psi0=p0, replay_accept=[1]))
    runs = [ihmc.Run(n_md=w["n_md"], n_traj=1, precision=ihmc.F32, seed=w["seed"], chain_id=w["chain_id"],
                     psi0=p0, replay_accept=[1]) for w, p0 in zip(ws, psi0)]
    ch = ihmc.Chains(ctx, lats, runs)
    ch.advance(1)
    infos = [ch.group_info(g) for g in range(ch.groups())]
    assert all(i["tiles"] > 256 for i in infos)  # both chains close their sums in several groups of 32 tiles
    for i, (w, r) in enumerate(zip(ws, refs)):
        g = ch.result(i)
        err = nrm(g["psi_final"], r.psi_final)
        print(f"{w['L']} class {classes[i]}: field {err:.2e}, H_old {abs(g['H_old'][0] / r.H_old[0] - 1):.2e}, "
              f"H_new {abs(g['H_new'][0] / r.H_new[0] - 1):.2e}, dH {g['dH'][0]:.4f} vs {r.dH[0]:.4f}")
        assert err < 1e-5
        assert abs(g["H_old"][0] - r.H_old[0]) <= 1e-5 * abs(r.H_old[0])
        assert abs(g["H_new"][0] - r.H_new[0]) <= 1e-5 * abs(r.H_new[0])
    ch.close()


@pytest.mark.parametrize("L", [(64, 64), (16, 16, 16)])
def test_paper_shift_c_n_plus_1e_5(ctx, orc, L):
    from paper_1912_03278_amd import ihmc
    d = len(L)
    C = 2 * d + 1e-5
    beta = 0.44 if d == 2 else 0.22
    N = int(np.prod(L))
    psi0 = np.random.default_rng(8).standard_normal(N).astype(np.float32).astype(np.float64)
    r = orc.run(orc.Lattice(L, beta=beta, C=C), 1, 12, seed=9, psi0=psi0, replay_accept=[1])
    errs = {}
    for prec in (8, 4):
        g = ctx.run_lattice(ihmc.Lattice(L, beta=beta, C=C),
                            ihmc.Run(n_md=12, n_traj=1, precision=prec, seed=9, psi0=psi0, replay_accept=[1]))
        errs[prec] = (nrm(g["psi_final"], r.psi_final), abs(g["H_new"][0] / r.H_new[0] - 1))
    print(f"C = n + 1e-5, {L}: FP64 field {errs[8][0]:.2e}, FP32 field {errs[4][0]:.2e}, "
          f"FP32 H_new {errs[4][1]:.2e}")
    assert errs[8][0] < 1e-12 and errs[8][1] < 1e-12
    # stated bound for the FP32 state at the paper's shift
    assert errs[4][0] < 1e-5 and errs[4][1] < 1e-5
