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


# ---- sequential single-spin Metropolis-Hastings with an explicit coupling matrix

def _sym(rng, N, diag):
    A = rng.standard_normal((N, N)) / np.sqrt(N)
    K = 0.5 * (A + A.T)
    np.fill_diagonal(K, diag * rng.standard_normal(N) if diag else 0.0)
    return K


@pytest.mark.parametrize("case", ["sk_h0", "sk_uniform_h", "sk_site_h_diag", "infinite_range", "torus"])
def test_dense_mh_against_enumeration(orc, case):
    """m, m^2 and beta*eps of the sequential sweeps average to the exact
    Boltzmann values of H(s) = -1/2 J s^T K s - h.s (4 sigma, Gamma method).  The
    matrix with a non-zero diagonal catches a diagonal term in the local field
    (it would shift dE by a constant and break detailed balance)."""
    rng = np.random.default_rng(11)
    J, h = 1.0, None
    if case == "sk_h0":
        K, beta = _sym(rng, 8, 0.0), 1.0
    elif case == "sk_uniform_h":
        K, beta, h = _sym(rng, 8, 0.0), 0.8, np.array([0.2])
    elif case == "sk_site_h_diag":
        K, beta, h = _sym(rng, 7, 0.7), 1.2, 0.3 * rng.standard_normal(7)
    elif case == "infinite_range":
        K, beta = E.infinite_range_K(10), 1.0
    else:
        K, beta, J = E.torus_adjacency((4, 4)), 0.35, 1.0
    N = K.shape[0]
    model = orc.Dense(K, beta=beta, C=0.0, J=J, h=h)
    r = orc.dense_mh_run(model, 100000, seed=5, chain_id=2)
    hv = 0.0 if h is None else (h[0] if h.size == 1 else h)
    ex = E.brute_force(K, beta, J=J, h=hv)
    for key, series in (("be", r["beta_eps"]), ("m", r["m"]), ("m2", r["m"] ** 2)):
        g = S.gamma_method(series[100:])
        assert abs(g["mean"] - ex[key]) < 4 * g["err"] + 1e-12, (case, key, g, ex[key])
    assert 0.0 < r["acceptance"] < 1.0
    assert r["spins"].dtype == np.int8 and set(np.unique(r["spins"])) <= {-1, 1}


def test_dense_mh_energy_and_limits(orc):
    """beta*eps per sweep is beta H(s)/N of the recorded spins (checked on the
    final sweep against the quadratic form with its diagonal); at beta -> 0
    every flip is accepted, so one sweep negates every spin; at beta -> infinity
    only flips with dE <= 0 are taken, so the energy never rises."""
    rng = np.random.default_rng(12)
    N = 40
    K = _sym(rng, N, 0.5)
    h = 0.1 * rng.standard_normal(N)
    model = orc.Dense(K, beta=0.9, C=0.0, J=1.3, h=h)
    r = orc.dense_mh_run(model, 3, seed=1)
    s = r["spins"].astype(np.float64)
    H = -0.5 * 1.3 * s @ K @ s - h @ s
    assert abs(r["beta_eps"][-1] - 0.9 * H / N) < 1e-13
    assert r["m"][-1] == s.sum() / N

    s0 = np.where(rng.random(N) < 0.5, 1, -1).astype(np.int8)
    hot = orc.dense_mh_run(orc.Dense(K, beta=1e-300, C=0.0, h=h), 1, spins0=s0)
    assert np.array_equal(hot["spins"], -s0) and hot["acceptance"] == 1.0

    cold = orc.dense_mh_run(orc.Dense(K, beta=1e300, C=0.0, h=h), 6, spins0=s0)
    e = cold["beta_eps"] / 1e300
    assert np.all(np.diff(e) <= 1e-15)
    sf = cold["spins"].astype(np.float64)
    f = K @ sf - np.diag(K) * sf
    assert np.all(2.0 * sf * (f + h) >= -1e-12)  # a local minimum after the last sweep


def test_dense_mh_determinism_and_refusals(orc):
    rng = np.random.default_rng(13)
    K = _sym(rng, 16, 0.0)
    a = orc.dense_mh_run(orc.Dense(K, beta=1.0, C=0.0), 20, seed=4, chain_id=1)
    b = orc.dense_mh_run(orc.Dense(K, beta=1.0, C=0.0), 20, seed=4, chain_id=1)
    c = orc.dense_mh_run(orc.Dense(K, beta=1.0, C=0.0), 20, seed=4, chain_id=2)
    assert np.array_equal(a["spins"], b["spins"]) and np.array_equal(a["beta_eps"], b["beta_eps"])
    assert not np.array_equal(a["m"], c["m"])
    with pytest.raises(ValueError):
        orc.dense_mh_run(orc.Dense(K, beta=1.0, C=0.0, h=np.zeros(5)), 3)
