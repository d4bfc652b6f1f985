"""The oracle's shifted form: the substitution phi = sqrt(J') Kt psi in eq.
did_HS_trafo (Sec. 2) instead of the paper's phi = sqrt(J') Kt psi - h' (eq.
phi_psi_substitution), so that the field sits inside the log cosh:

    S(psi) = 1/2 psi.Kt psi - sum_i log cosh(sqrt(J') (Kt psi)_i + h'_i).

Pinned against mathematics it does not use:

* force = -dS/dpsi by central differences (2D with a per-site field, 3D with a
  uniform one, a dense K);
* the estimators with an exact sampler: psi given s is Normal(sqrt(J') s,
  Kt^-1) here (phi given s is Normal(J' Kt s, J' Kt) by eq. did_HS_trafo), so
  exact Boltzmann spins plus that draw give exact samples whose estimator
  averages must equal enumeration;
* the two substitutions differ by the constant translation
  psi_paper = psi_shifted + Kt^-1 h'/sqrt(J') (computed here with a dense
  numpy solve): the actions differ by h'.Kt^-1 h'/(2J'), the forces and the
  estimators agree at translated points, and whole chains started at
  translated points with the same momenta take the same decisions;
* leap-frog reversibility and dH ~ eps^2;
* a whole chain against enumeration (4x4, h = 0.1).
"""
import math

import numpy as np
import pytest

from oracle import exact as E
from oracle import stats as S


def _kt(model):
    """Kt as a dense matrix, assembled from the torus adjacency or the given K."""
    if hasattr(model, "K"):
        K = np.asarray(model.K, dtype=np.float64)
    else:
        K = E.torus_adjacency(model.L)
    return K + model.C * np.eye(K.shape[0])


def _hp(model):
    h = model.h
    if h is None:
        return np.zeros(model.N)
    return model.beta * np.broadcast_to(np.asarray(h, dtype=np.float64), (model.N,)).copy()


def _models(orc):
    rng = np.random.default_rng(21)
    A = rng.normal(0, 0.3, (10, 10))
    K = np.triu(A, 1) + np.triu(A, 1).T
    return {
        "2d_uniform": orc.Lattice((6, 5), beta=0.42, C=4.1, h=0.08),
        "2d_site_field": orc.Lattice((5, 4), beta=0.45, C=4.1, h=rng.normal(0, 0.2, 20)),
        "3d_uniform": orc.Lattice((3, 4, 3), beta=0.25, C=6.3, h=0.07),
        "dense": orc.Dense(K, beta=0.8, C=-np.linalg.eigvalsh(K).min() + 0.3, h=rng.normal(0, 0.1, 10)),
    }


@pytest.mark.parametrize("case", ["2d_site_field", "3d_uniform", "dense"])
def test_shifted_force_is_minus_gradient(orc, case):
    m = _models(orc)[case]
    rng = np.random.default_rng(2)
    psi = rng.normal(0, 1.0, m.N)
    F = orc.force(m, psi, form="shifted")
    step = 1e-5
    for i in range(m.N):
        e = np.zeros(m.N)
        e[i] = step
        num = -(orc.action(m, psi + e, form="shifted")["S"] - orc.action(m, psi - e, form="shifted")["S"]) / (2 * step)
        assert abs(num - F[i]) < 1e-7 * max(1.0, abs(F[i])), (i, num, F[i])
    # the linear term is gone: F differs from the paper form's force
    if m.h is not None:
        assert np.max(np.abs(F - orc.force(m, psi))) > 1e-3


@pytest.mark.parametrize("case", ["3x3_site_field", "4x4_uniform_field", "4x4_zero_field"])
def test_shifted_estimators_with_exact_iid_sampler(orc, case):
    rng = np.random.default_rng(6)
    beta = 0.35
    if case == "3x3_site_field":
        L, h = (3, 3), rng.normal(0, 0.3, 9)
    elif case == "4x4_uniform_field":
        L, h = (4, 4), 0.1
    else:
        L, h = (4, 4), 0.0
    Kadj = E.torus_adjacency(L)
    N = Kadj.shape[0]
    m = orc.Lattice(L, beta=beta, C=2 * len(L) + 0.1, h=None if case == "4x4_zero_field" else h)
    states, p = E.boltzmann_weights(Kadj, beta, h=h)
    n = 40000
    s = states[rng.choice(len(p), size=n, p=p)]
    Kt = Kadj + m.C * np.eye(N)
    Lc = np.linalg.cholesky(Kt)  # psi | s = sqrt(J') s + Lc^-T xi, covariance Kt^-1
    psi = math.sqrt(beta) * s + np.linalg.solve(Lc.T, rng.standard_normal((N, n))).T
    est = np.array([[orc.action(m, x, form="shifted")[k] for k in ("m", "m2c", "beta_eps")] for x in psi])
    ex = E.brute_force(Kadj, beta, h=h)
    for j, key in enumerate(("m", "m2", "be")):
        mu, sd = est[:, j].mean(), est[:, j].std() / math.sqrt(n)
        assert abs(mu - ex[key]) < 4 * sd + 1e-12, (key, mu, ex[key], sd)


@pytest.mark.parametrize("case", ["2d_uniform", "2d_site_field", "3d_uniform", "dense"])
def test_shifted_is_the_translate_of_the_paper_form(orc, case):
    m = _models(orc)[case]
    Kt, hp = _kt(m), _hp(m)
    Jp = m.beta * getattr(m, "J", 1.0)
    delta = np.linalg.solve(Kt, hp) / math.sqrt(Jp)
    c_e = hp @ np.linalg.solve(Kt, hp)
    rng = np.random.default_rng(9)
    for _ in range(3):
        psi = rng.normal(0, 1.0, m.N)
        a = orc.action(m, psi, form="shifted")
        b = orc.action(m, psi + delta)
        assert abs(a["S"] - (b["S"] + c_e / (2 * Jp))) < 1e-11 * max(1.0, abs(a["S"]))
        for k in ("m", "m2c", "beta_eps"):
            assert abs(a[k] - b[k]) < 1e-12, (k, a[k], b[k])
        assert np.max(np.abs(orc.force(m, psi, form="shifted") - orc.force(m, psi + delta))) < 1e-11
    psi0 = orc.normals(4, 3, 0, orc.TAG_INIT, m.N)
    for integ in (orc.LEAPFROG, orc.OMELYAN):
        ref = orc.run(m, 30, 6, seed=4, chain_id=3, psi0=psi0, integrator=integ)
        sh = orc.run(m, 30, 6, seed=4, chain_id=3, psi0=psi0 - delta, integrator=integ, form="shifted")
        assert np.array_equal(ref.accepted, sh.accepted) and ref.acceptance > 0.3
        assert np.max(np.abs(ref.dH - sh.dH)) < 1e-9
        for k in ("m", "m2c", "beta_eps"):
            assert np.max(np.abs(getattr(ref, k) - getattr(sh, k))) < 1e-10, k
        assert np.max(np.abs(ref.psi_final - (sh.psi_final + delta))) < 1e-10


def test_shifted_zero_field_equals_paper_form(orc):
    """At h = 0 the two substitutions coincide (flips included)."""
    m = orc.Lattice((7, 6), beta=0.44, C=4.1)
    a = orc.run(m, 40, 8, seed=2, chain_id=1, flip_every=3)
    b = orc.run(m, 40, 8, seed=2, chain_id=1, flip_every=3, form="shifted")
    for k in ("dH", "accepted", "flipped", "psi_final", "m", "m2c"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    assert np.max(np.abs(a.beta_eps - b.beta_eps)) < 1e-13
    assert b.flipped.sum() > 0


def test_shifted_leapfrog_reversible_and_eps_squared(orc):
    rng = np.random.default_rng(3)
    m = orc.Lattice((5, 5), beta=0.44, C=4.1, h=0.05)
    psi, p = rng.standard_normal(25), rng.standard_normal(25)
    psi1, p1 = orc.md(m, psi, p, 8, form="shifted")
    psi2, p2 = orc.md(m, psi1, -p1, 8, form="shifted")
    assert np.max(np.abs(psi2 - psi)) < 1e-12 and np.max(np.abs(p2 + p)) < 1e-12

    def H(x, q):
        return 0.5 * q @ q + orc.action(m, x, form="shifted")["S"]

    H0 = H(psi, p)
    d = []
    for n in (20, 40, 80, 160):
        a, b = orc.md(m, psi, p, n, form="shifted")
        d.append(abs(H(a, b) - H0))
    slope = np.polyfit(np.log(1.0 / np.array([20, 40, 80, 160])), np.log(d), 1)[0]
    assert abs(slope - 2.0) < 0.15, (slope, d)


def test_shifted_chain_against_enumeration(orc):
    m = orc.Lattice((4, 4), beta=0.4, C=4.1, h=0.1)
    ex = E.brute_force(E.torus_adjacency((4, 4)), 0.4, h=0.1)
    r = orc.run(m, 40000, 10, seed=13, form="shifted")
    assert 0.9 < r.acceptance <= 1.0
    for key, ref in (("beta_eps", ex["be"]), ("m2c", ex["m2"]), ("m", ex["m"])):
        g = S.gamma_method(getattr(r, key)[500:])
        assert abs(g["mean"] - ref) < 4 * g["err"], (key, g, ref)


def test_shifted_refusals(orc):
    m = orc.Lattice((5, 5), beta=0.42, C=4.1, h=0.03)
    with pytest.raises(ValueError):
        orc.run(m, 5, 4, flip_every=2, form="shifted")  # psi -> -psi is no symmetry at h != 0
    with pytest.raises(ValueError):
        orc.run(m, 5, 4, form="other")
    with pytest.raises(ValueError):
        orc.force(m, np.zeros(25), form="other")
    # at h = 0 flips are allowed
    orc.run(orc.Lattice((5, 5), beta=0.42, C=4.1), 4, 4, flip_every=2, form="shifted")
