"""The FP64 oracle's HMC chains against exact spin-model results.

Pins (all independent of the auxiliary-field code): enumeration, the row
transfer matrix, the 1D closed form, the infinite-range formula of App. A, and
the exact conditional law of psi given s.  Agreement is tested at 4 sigma with
Gamma-method errors (the paper's error scheme, Sec. 4 footnote).
"""
import math

import numpy as np
import pytest

from oracle import exact as E
from oracle import stats as S

Z = 4.0


def _check(series, ref, n_therm=0):
    g = S.gamma_method(series[n_therm:])
    z = S.z_score(g["mean"], ref, g["err"])
    assert z < Z, (g, ref, z)
    return g


def test_4x4_h0_against_enumeration(orc):
    lat = orc.Lattice((4, 4), beta=0.4, C=4.1)
    ex = E.brute_force(E.torus_adjacency((4, 4)), 0.4)
    r = orc.run(lat, 30000, 10, seed=1)
    assert 0.9 < r.acceptance <= 1.0
    _check(r.beta_eps, ex["be"], 500)
    _check(r.m2c, ex["m2"], 500)


def test_4x4_field_against_enumeration(orc):
    lat = orc.Lattice((4, 4), beta=0.4, C=4.1, h=0.1)
    ex = E.brute_force(E.torus_adjacency((4, 4)), 0.4, h=0.1)
    r = orc.run(lat, 30000, 10, seed=2)
    _check(r.beta_eps, ex["be"], 500)
    _check(r.m, ex["m"], 500)
    _check(r.m2c, ex["m2"], 500)


@pytest.mark.parametrize("beta", [0.4, E.BETA_C_2D])
def test_8x8_against_transfer_matrix(orc, beta):
    """The small-lattice workload: 8x8 torus, J = 1, h = 0, C = 4.1, 10 MD steps."""
    lat = orc.Lattice((8, 8), beta=beta, C=4.1)
    ex = E.row_transfer_2d(8, 8, beta)
    r = orc.run(lat, 30000, 10, seed=3, flip_every=5)
    _check(r.beta_eps, ex["be"], 500)
    _check(r.m2c, ex["m2"], 500)


def test_ring_with_field_against_closed_form(orc):
    lat = orc.Lattice((12,), beta=0.5, C=2.1, h=0.1)
    ex = E.ring_1d(12, 0.5, h=0.1)
    r = orc.run(lat, 30000, 8, seed=4)
    _check(r.beta_eps, ex["be"], 500)
    _check(r.m, ex["m"], 500)


@pytest.mark.parametrize("N", [8, 12])
def test_infinite_range_dense_against_appendix(orc, N):
    K = E.infinite_range_K(N)
    lmin = np.linalg.eigvalsh(K).min()
    d = orc.Dense(K, beta=1.0, C=-lmin + 0.1)
    ex = E.infinite_range(N, 1.0)
    r = orc.run(d, 30000, 10, seed=5, flip_every=4)
    _check(r.beta_eps, ex["be"], 500)
    # the dense estimators of m^2 (bias 1^T Kt^-1 1 / (N^2 J') from a CG solve) and m
    _check(r.m2c, ex["m2"], 500)
    _check(r.m, ex["m"], 500)


@pytest.mark.parametrize("dC", [1e-5, 0.1, 1.0])
def test_results_independent_of_C(orc, dC):
    """Sec. 4: observables do not depend on the shift C."""
    lat = orc.Lattice((4, 4), beta=0.4, C=4 + dC, h=0.05)
    ex = E.brute_force(E.torus_adjacency((4, 4)), 0.4, h=0.05)
    r = orc.run(lat, 30000, 10, seed=6)
    _check(r.beta_eps, ex["be"], 500)
    _check(r.m, ex["m"], 500)


def test_omelyan_chain(orc):
    lat = orc.Lattice((4, 4), beta=0.4, C=4.1)
    ex = E.brute_force(E.torus_adjacency((4, 4)), 0.4)
    r = orc.run(lat, 20000, 5, seed=7, integrator=orc.OMELYAN)
    _check(r.beta_eps, ex["be"], 500)


def test_mean_exp_minus_dH_is_one(orc):
    """<exp(-dH)> = 1 for a reversible, area-preserving integrator."""
    lat = orc.Lattice((10, 10), beta=0.44, C=4.1)
    r = orc.run(lat, 6000, 4, seed=8)
    g = S.gamma_method(np.exp(-r.dH[200:]))
    assert abs(g["mean"] - 1.0) < Z * g["err"], g
    assert 0.3 < r.acceptance < 0.95


@pytest.mark.parametrize("case", ["3x3_site_field", "4x4_uniform_field"])
def test_estimators_with_exact_iid_sampler(orc, case):
    """psi | s ~ N(sqrt(J') s + Kt^-1 h'/sqrt(J'), Kt^-1) (eqs. did_HS_trafo and
    phi_psi_substitution).  Drawing s from the exact Boltzmann weights and psi from
    that law gives exact samples of psi; the oracle's estimators for m, m^2 and
    beta*eps must then average to the exact spin-model values, with no MCMC."""
    rng = np.random.default_rng(9)
    beta = 0.35
    if case == "3x3_site_field":
        L, h = (3, 3), rng.normal(0, 0.3, 9)
    else:
        L, h = (4, 4), 0.1
    Kadj = E.torus_adjacency(L)
    N = Kadj.shape[0]
    lat = orc.Lattice(L, beta=beta, C=2 * len(L) + 0.1, h=h)
    states, p = E.boltzmann_weights(Kadj, beta, h=h)
    n = 40000
    s = states[rng.choice(len(p), size=n, p=p)]
    Kt = Kadj + lat.C * np.eye(N)
    hp = beta * np.broadcast_to(h, (N,))
    psi = E.sample_psi_given_s(rng, s, Kt, beta, hp)
    est = np.array([[orc.action(lat, x)[k] for k in ("m", "m2c", "beta_eps")] for x in psi])
    hv = np.broadcast_to(h, (N,))
    ms = s.sum(axis=1) / N
    be_s = beta * (-0.5 * np.einsum("ki,ij,kj->k", s, Kadj, s) - s @ hv) / N
    ex = E.brute_force(Kadj, beta, h=h)
    for j, (key, exact) in enumerate((("m", ex["m"]), ("m2", ex["m2"]), ("be", ex["be"]))):
        mu, sd = est[:, j].mean(), est[:, j].std() / math.sqrt(n)
        assert abs(mu - exact) < Z * sd, (key, mu, exact, sd)
    # the per-sample estimator is unbiased given s, so it also tracks the spin sample mean
    assert abs(est[:, 0].mean() - ms.mean()) < Z * est[:, 0].std() / math.sqrt(n)
    assert abs(est[:, 2].mean() - be_s.mean()) < Z * (est[:, 2] - be_s).std() / math.sqrt(n)


def test_sign_flip_always_accepted_at_zero_field(orc):
    lat = orc.Lattice((6, 6), beta=0.5, C=4.1)
    r = orc.run(lat, 200, 8, seed=10, flip_every=1)
    assert r.flipped.all()


def test_sign_flip_with_field_keeps_distribution(orc):
    lat = orc.Lattice((4, 4), beta=0.5, C=4.1, h=0.02)
    ex = E.brute_force(E.torus_adjacency((4, 4)), 0.5, h=0.02)
    r = orc.run(lat, 30000, 10, seed=11, flip_every=2)
    assert 0 < r.flipped.sum() < r.flipped.size // 2
    _check(r.m, ex["m"], 500)


def test_determinism_and_replay(orc):
    lat = orc.Lattice((5, 5), beta=0.42, C=4.1, h=0.03)
    a = orc.run(lat, 200, 6, seed=12, chain_id=3)
    b = orc.run(lat, 200, 6, seed=12, chain_id=3)
    assert np.array_equal(a.dH, b.dH) and np.array_equal(a.psi_final, b.psi_final)
    c = orc.run(lat, 200, 6, seed=12, chain_id=3, replay_accept=a.accepted)
    assert np.array_equal(a.dH, c.dH) and np.array_equal(a.accepted, c.accepted)
    flipped = a.accepted.copy()
    flipped[50] ^= 1
    d = orc.run(lat, 200, 6, seed=12, chain_id=3, replay_accept=flipped)
    assert np.array_equal(d.accepted, flipped)
    assert not np.array_equal(a.psi_final, d.psi_final)
