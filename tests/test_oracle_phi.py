"""The oracle's inverse (phi) formulation (Sec. 2, eq. cosh_in_exponent),
the A/B baseline of the substitution, pinned against mathematics it does not use.

* force = -dS/dphi by central differences of the action (2D with a per-site
  field, 3D with a uniform one, a dense K);
* the estimators: phi given s is Normal(J' Kt s, J' Kt) (eq. did_HS_trafo with
  the spins held fixed), so drawing s from the exact Boltzmann weights and phi
  from that law gives exact samples; the estimators (the expectations of m,
  m^2 and beta*eps given phi) must then average to the exact spin-model values
  with no MCMC;
* leap-frog reversibility and dH ~ eps^2;
* whole chains against enumeration (4x4, h = 0 and 0.1) and App. A (dense),
  i.e. the same spin observables as the psi form, which is pinned the same way.
"""
import math

import numpy as np
import pytest

from oracle import exact as E
from oracle import stats as S


def _lat(orc, L, beta, C, h=None):
    return orc.Lattice(tuple(L), beta=beta, C=C, h=h)


@pytest.mark.parametrize("case", ["2d_site_field", "3d_uniform", "dense"])
def test_phi_force_is_minus_gradient(orc, case):
    rng = np.random.default_rng(1)
    if case == "2d_site_field":
        m = _lat(orc, (5, 4), 0.45, 4.1, rng.normal(0, 0.2, 20))
    elif case == "3d_uniform":
        m = _lat(orc, (3, 4, 3), 0.25, 6.3, 0.07)
    else:
        A = rng.normal(0, 0.3, (9, 9))
        K = np.triu(A, 1) + np.triu(A, 1).T
        m = orc.Dense(K, beta=0.8, C=-np.linalg.eigvalsh(K).min() + 0.3, h=rng.normal(0, 0.1, 9))
    phi = rng.normal(0, 1.5, m.N)
    F = orc.phi_force(m, phi)
    h = 1e-5
    fd = np.empty(m.N)
    for i in range(m.N):
        e = np.zeros(m.N)
        e[i] = h
        fd[i] = -(orc.phi_action(m, phi + e)["S"] - orc.phi_action(m, phi - e)["S"]) / (2 * h)
    assert np.max(np.abs(F - fd)) < 1e-7 * max(1.0, np.max(np.abs(F)))


def test_phi_action_closed_form_uniform_field(orc):
    """Uniform phi = c on a torus: Kt 1 = (n0 + C) 1, so S = N c^2 / (2 J' (n0 + C)) - N log cosh(h' + c)."""
    beta, C, h, c = 0.4, 4.3, 0.05, 0.7
    m = _lat(orc, (6, 5), beta, C, h)
    S_ref = 30 * c * c / (2 * beta * (4 + C)) - 30 * math.log(math.cosh(beta * h + c))
    assert orc.phi_action(m, np.full(30, c))["S"] == pytest.approx(S_ref, rel=1e-13)


@pytest.mark.parametrize("case", ["3x3_site_field", "4x4_uniform_field", "4x4_zero_field"])
def test_phi_estimators_with_exact_iid_sampler(orc, case):
    rng = np.random.default_rng(5)
    beta = 0.35
    if case == "3x3_site_field":
        L, h = (3, 3), rng.normal(0, 0.3, 9)
    elif case == "4x4_uniform_field":
        L, h = (4, 4), 0.1
    else:
        L, h = (4, 4), 0.0
    Kadj = E.torus_adjacency(L)
    N = Kadj.shape[0]
    m = _lat(orc, L, beta, 2 * len(L) + 0.1, None if case == "4x4_zero_field" else h)
    states, p = E.boltzmann_weights(Kadj, beta, h=h)
    n = 40000
    s = states[rng.choice(len(p), size=n, p=p)]
    Kt = Kadj + m.C * np.eye(N)
    Lc = np.linalg.cholesky(beta * Kt)
    phi = (beta * Kt @ s.T).T + (Lc @ rng.standard_normal((N, n))).T
    est = np.array([[orc.phi_action(m, x)[k] for k in ("m", "m2c", "beta_eps")] for x in phi])
    ex = E.brute_force(Kadj, beta, h=h)
    for j, key in enumerate(("m", "m2", "be")):
        mu, sd = est[:, j].mean(), est[:, j].std() / math.sqrt(n)
        assert abs(mu - ex[key]) < 4 * sd + 1e-12, (key, mu, ex[key], sd)


def test_phi_leapfrog_reversible_and_eps_squared(orc):
    rng = np.random.default_rng(3)
    m = _lat(orc, (5, 5), 0.44, 4.1, 0.03)
    phi, p = orc.phi_start(m, seed=2), rng.standard_normal(25)
    phi1, p1 = orc.phi_md(m, phi, p, 8)
    phi2, p2 = orc.phi_md(m, phi1, -p1, 8)
    assert np.max(np.abs(phi2 - phi)) < 1e-11 and np.max(np.abs(p2 + p)) < 1e-11
    H0 = orc.phi_hamiltonian(m, phi, p)
    d = []
    for n in (20, 40, 80, 160):
        a, b = orc.phi_md(m, phi, p, n)
        d.append(abs(orc.phi_hamiltonian(m, a, b) - H0))
    slope = np.polyfit(np.log(1.0 / np.array([20, 40, 80, 160])), np.log(d), 1)[0]
    assert abs(slope - 2.0) < 0.15, (slope, d)


def test_phi_start_is_the_substitution(orc):
    """phi0 = sqrt(J') Kt psi0 - h' with psi0 the TAG_INIT normals (the psi chain's start)."""
    m = _lat(orc, (6, 4), 0.4, 4.1, 0.02)
    psi0 = orc.normals(3, 1, 0, orc.TAG_INIT, 24)
    Kt = E.torus_adjacency((6, 4)) + 4.1 * np.eye(24)
    ref = math.sqrt(0.4) * Kt @ psi0 - 0.4 * 0.02
    assert np.max(np.abs(orc.phi_start(m, seed=3, chain_id=1) - ref)) < 1e-13


@pytest.mark.parametrize("h", [0.0, 0.1])
def test_phi_chain_against_enumeration(orc, h):
    m = _lat(orc, (4, 4), 0.4, 4.1, h if h else None)
    ex = E.brute_force(E.torus_adjacency((4, 4)), 0.4, h=h)
    r = orc.run(m, 40000, 10, seed=11, form="phi")
    assert 0.9 < r.acceptance <= 1.0
    for key, ref in (("beta_eps", ex["be"]), ("m2c", ex["m2"]), ("m", ex["m"])):
        g = S.gamma_method(getattr(r, key)[500:])
        assert abs(g["mean"] - ref) < 4 * g["err"], (key, g, ref)


def test_phi_dense_chain_against_appendix(orc):
    N = 8
    K = E.infinite_range_K(N)
    d = orc.Dense(K, beta=1.0, C=-np.linalg.eigvalsh(K).min() + 0.1)
    ex = E.infinite_range(N, 1.0)
    r = orc.run(d, 30000, 10, seed=12, form="phi")
    for key, ref in (("beta_eps", ex["be"]), ("m2c", ex["m2"])):
        g = S.gamma_method(r.__dict__[key][500:])
        assert abs(g["mean"] - ref) < 4 * g["err"], (key, g, ref)


def test_phi_chain_replay_and_refusals(orc):
    m = _lat(orc, (5, 5), 0.42, 4.1, 0.03)
    a = orc.run(m, 50, 6, seed=4, chain_id=2, form="phi")
    b = orc.run(m, 50, 6, seed=4, chain_id=2, form="phi", replay_accept=a.accepted)
    assert np.array_equal(a.dH, b.dH) and np.array_equal(a.psi_final, b.psi_final)
    with pytest.raises(ValueError):
        orc.run(m, 5, 6, form="phi", flip_every=2)
    with pytest.raises(ValueError):
        orc.run(m, 5, 6, form="phi", integrator=orc.OMELYAN)
