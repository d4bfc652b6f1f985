"""The oracle's checkerboard Metropolis-Hastings (the comparison method of
Sec. 4) against enumeration: the spin chain's m, m^2 and beta*eps must average
to the exact values (Gamma-method errors, 4 sigma); 2D and 3D, with and without
a field, including the smallest even lattices where both neighbours along an
axis are the same site (the coupling then counts twice, as in K)."""
import numpy as np
import pytest

from oracle import exact as E
from oracle import stats as S


@pytest.mark.parametrize("L,beta,h", [((4, 4), 0.4, 0.0), ((4, 4), 0.4, 0.1), ((2, 4), 0.3, 0.05),
                                      ((2, 2, 2), 0.2, 0.0), ((2, 2, 4), 0.25, 0.1)])
def test_mh_against_enumeration(orc, L, beta, h):
    lat = orc.Lattice(L, beta=beta, C=2 * len(L) + 0.1, h=h if h else None)
    r = orc.mh_run(lat, 120000, seed=3)
    ex = E.brute_force(E.torus_adjacency(L), beta, h=h)
    for key, series in (("be", r["beta_eps"]), ("m", r["m"]), ("m2", r["m"] ** 2)):
        g = S.gamma_method(series[100:])
        assert abs(g["mean"] - ex[key]) < 4 * g["err"] + 1e-12, (key, g, ex[key])
    assert 0.0 < r["acceptance"] < 1.0


def test_mh_determinism_and_refusals(orc):
    lat = orc.Lattice((6, 8), beta=0.44, C=4.1, h=0.02)
    a = orc.mh_run(lat, 50, seed=4, chain_id=1)
    b = orc.mh_run(lat, 50, seed=4, chain_id=1)
    assert np.array_equal(a["spins"], b["spins"]) and np.array_equal(a["beta_eps"], b["beta_eps"])
    c = orc.mh_run(lat, 50, seed=4, chain_id=2)
    assert not np.array_equal(a["spins"], c["spins"])
    # continuing from the final spins = running longer (counters restart at sweep 0 though)
    s0 = np.where(np.arange(48) % 3 == 0, 1, -1).astype(np.int8)
    d = orc.mh_run(lat, 1, seed=4, spins0=s0)
    assert d["spins"].dtype == np.int8 and set(np.unique(d["spins"])) <= {-1, 1}
    for bad in (orc.Lattice((5, 4), beta=0.4, C=4.1), orc.Lattice((4, 4), beta=0.4, C=4.1, h=np.zeros(16)),
                orc.Lattice((8,), beta=0.4, C=2.1)):
        with pytest.raises(ValueError):
            orc.mh_run(bad, 3)


def test_mh_energy_of_aligned_state(orc):
    """All spins up, beta tiny (almost every flip accepted is impossible to
    predict; instead beta = 0 accepts every flip): after one sweep at beta = 0
    every spin is flipped, so m = -1 and beta*eps = 0."""
    lat = orc.Lattice((4, 6), beta=0.0 + 1e-300, C=4.1)
    r = orc.mh_run(lat, 1, spins0=np.ones(24, dtype=np.int8))
    assert r["m"][0] == -1.0
    assert r["acceptance"] == 1.0
