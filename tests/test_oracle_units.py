"""Pins of the FP64 oracle's building blocks against mathematics it does not use.

* K~ application: the explicit K~ = K + C*1 matrix built from the torus
  adjacency (Sec. 2), and the Fourier eigenvalues C + 2 sum cos(k_mu).
* force: central finite differences of the action (EOM of Sec. 3) and the
  closed form for a uniform field.
* action: closed form for a uniform field; the large-C minima at
  psi = +-sqrt(J') (Sec. 3, eq. large C minima).
* observable constants: eq. hKh_for_constant_h and a dense solve.
* leap-frog: reversibility and dH ~ eps^2; Omelyan likewise.
* Philox / Box-Muller: distribution tests.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats as sst

from oracle import exact as E


def _lat(orc, L, beta=0.4, C=None, h=None):
    C = 2 * len(L) + 0.1 if C is None else C
    return orc.Lattice(tuple(L), beta=beta, C=C, h=h)


@pytest.mark.parametrize("L", [(5,), (3, 5), (4, 4), (7, 3), (3, 4, 5), (4, 4, 4)])
def test_stencil_equals_explicit_matrix(orc, L):
    rng = np.random.default_rng(1)
    lat = _lat(orc, L, C=2 * len(L) + 0.37)
    psi = rng.standard_normal(lat.N)
    Kt = E.torus_adjacency(L) + lat.C * np.eye(lat.N)
    assert np.max(np.abs(orc.apply_Kt(lat, psi) - Kt @ psi)) < 1e-13


@pytest.mark.parametrize("L,k", [((8, 6), (1, 2)), ((16,), (3,)), ((6, 4, 5), (1, 1, 2))])
def test_stencil_plane_wave_eigenvalue(orc, L, k):
    lat = _lat(orc, L, C=2 * len(L) + 0.25)
    grids = np.meshgrid(*[np.arange(n) for n in L[::-1]], indexing="ij")  # z, y, x
    phase = sum(2 * np.pi * k[mu] * grids[len(L) - 1 - mu] / L[mu] for mu in range(len(L)))
    psi = np.cos(phase).ravel()
    lam = lat.C + 2 * sum(math.cos(2 * math.pi * k[mu] / L[mu]) for mu in range(len(L)))
    assert np.max(np.abs(orc.apply_Kt(lat, psi) - lam * psi)) < 1e-12


def test_dense_apply(orc):
    rng = np.random.default_rng(2)
    N = 37
    A = rng.standard_normal((N, N)) / math.sqrt(N)
    K = (A + A.T) / 2
    np.fill_diagonal(K, 0)
    d = orc.Dense(K, beta=1.0, C=3.0)
    psi = rng.standard_normal(N)
    assert np.max(np.abs(orc.apply_Kt(d, psi) - (K @ psi + 3.0 * psi))) < 1e-13


def _fd_force(orc, model, psi, h=1e-5):
    F = np.empty_like(psi)
    for i in range(psi.size):
        e = np.zeros_like(psi)
        e[i] = h
        F[i] = -(orc.action(model, psi + e)["S"] - orc.action(model, psi - e)["S"]) / (2 * h)
    return F


@pytest.mark.parametrize("which", ["lattice_h0", "lattice_hsite", "lattice_3d", "dense_h"])
def test_force_is_minus_gradient_of_action(orc, which):
    rng = np.random.default_rng(3)
    if which == "lattice_h0":
        m = _lat(orc, (4, 5), beta=0.44)
    elif which == "lattice_hsite":
        m = _lat(orc, (3, 4), beta=0.3, h=rng.normal(0, 0.3, 12))
    elif which == "lattice_3d":
        m = _lat(orc, (3, 3, 4), beta=0.22, h=0.07)
    else:
        N = 10
        A = rng.standard_normal((N, N)) / math.sqrt(N)
        K = (A + A.T) / 2
        np.fill_diagonal(K, 0)
        lmin = np.linalg.eigvalsh(K).min()
        m = orc.Dense(K, beta=0.8, C=-lmin + 0.1, h=rng.normal(0, 0.2, N))
    psi = rng.standard_normal(m.N) * 0.7
    F = orc.force(m, psi)
    Ffd = _fd_force(orc, m, psi)
    assert np.max(np.abs(F - Ffd)) / np.max(np.abs(F)) < 1e-7


@pytest.mark.parametrize("L,h", [((6, 6), 0.0), ((5, 5, 3), 0.13), ((9,), -0.2)])
def test_uniform_field_closed_forms(orc, L, h):
    beta = 0.37
    lat = _lat(orc, L, beta=beta, h=h)
    n0c = 2 * len(L) + lat.C
    sq = math.sqrt(beta)
    b = beta * h / sq
    c = 0.61
    psi = np.full(lat.N, c)
    F = orc.force(lat, psi)
    y = sq * n0c * c
    F_ref = -n0c * c + b + sq * n0c * math.tanh(y)
    assert np.max(np.abs(F - F_ref)) < 1e-13
    S = orc.action(lat, psi)["S"]
    S_ref = lat.N * (0.5 * n0c * c * c - c * b - math.log(math.cosh(y)))
    assert S == pytest.approx(S_ref, rel=1e-13)


def test_large_C_minima(orc):
    """For |C| -> infinity, H/C ~ psi^2/2 - sqrt(J') sum|psi|: minima at psi = +-sqrt(J')."""
    beta = 0.45
    for C in (1e3, 1e4):
        lat = _lat(orc, (4, 4), beta=beta, C=C)
        cs = np.linspace(0.2, 1.2, 2001)
        S = [orc.action(lat, np.full(16, c))["S"] for c in cs]
        cmin = cs[int(np.argmin(S))]
        assert abs(cmin - math.sqrt(beta)) < 5.0 / C + 1e-3


def test_observable_constants(orc):
    rng = np.random.default_rng(4)
    # uniform h: h'^T Kt^-1 h' = N h0'^2 / (n0 + C)   (eq. hKh_for_constant_h)
    lat = _lat(orc, (5, 4), beta=0.4, h=0.3)
    cm, ce, cv = orc.constants(lat)
    n0c = 4 + lat.C
    hp = 0.4 * 0.3
    assert ce == pytest.approx(20 * hp * hp / n0c, rel=1e-14)
    assert cm == pytest.approx(20 * hp / n0c, rel=1e-14)
    assert cv == pytest.approx(20 / n0c, rel=1e-14)
    # per-site h: CG against a dense solve with the explicit matrix
    h = rng.normal(0, 0.5, 20)
    lat = _lat(orc, (5, 4), beta=0.4, h=h)
    Kt = E.torus_adjacency((5, 4)) + lat.C * np.eye(20)
    hp = 0.4 * h
    cm, ce, cv = orc.constants(lat)
    assert ce == pytest.approx(hp @ np.linalg.solve(Kt, hp), rel=1e-12)
    assert cm == pytest.approx(np.ones(20) @ np.linalg.solve(Kt, hp), rel=1e-12)


def test_leapfrog_reversibility(orc):
    rng = np.random.default_rng(5)
    for integ in (orc.LEAPFROG, orc.OMELYAN):
        lat = _lat(orc, (6, 6), beta=0.44, h=rng.normal(0, 0.1, 36))
        psi0, p0 = rng.standard_normal(36), rng.standard_normal(36)
        psi1, p1 = orc.md(lat, psi0, p0, 10, integrator=integ)
        psi2, p2 = orc.md(lat, psi1, -p1, 10, integrator=integ)
        assert np.max(np.abs(psi2 - psi0)) < 1e-12
        assert np.max(np.abs(p2 + p0)) < 1e-12


def _mean_abs_dH(orc, lat, n_md, integ, reps=8):
    rng = np.random.default_rng(6)
    out = []
    for _ in range(reps):
        psi, p = rng.standard_normal(lat.N), rng.standard_normal(lat.N)
        H0 = orc.hamiltonian(lat, psi, p)
        psi1, p1 = orc.md(lat, psi, p, n_md, integrator=integ)
        out.append(abs(orc.hamiltonian(lat, psi1, p1) - H0))
    return float(np.mean(out))


@pytest.mark.parametrize("integ", [0, 1])
def test_dH_scales_as_eps_squared(orc, integ):
    lat = _lat(orc, (6, 6), beta=0.44)
    steps = [10, 20, 40, 80]
    d = [_mean_abs_dH(orc, lat, n, integ) for n in steps]
    slope = np.polyfit(np.log(1.0 / np.array(steps)), np.log(d), 1)[0]
    assert abs(slope - 2.0) < 0.1, (slope, d)


def test_omelyan_beats_leapfrog_per_force(orc):
    """At equal force evaluations (leap-frog 2n steps vs Omelyan n steps) 2MN has smaller |dH|."""
    lat = _lat(orc, (6, 6), beta=0.44)
    assert _mean_abs_dH(orc, lat, 10, orc.OMELYAN) < _mean_abs_dH(orc, lat, 20, orc.LEAPFROG)


def test_philox_uniforms_and_normals(orc):
    u = np.array([orc.uniform(7, c, t, orc.TAG_ACC) for c in range(40) for t in range(250)])
    assert u.min() > 0 and u.max() < 1
    assert sst.kstest(u, "uniform").pvalue > 1e-4
    z = orc.normals(11, 3, 5, orc.TAG_MOM, 200001)
    assert abs(z.mean()) < 4 / math.sqrt(z.size)
    assert abs(z.var() - 1) < 4 * math.sqrt(2 / z.size)
    assert abs(np.mean(z ** 4) - 3) < 4 * math.sqrt(96 / z.size)
    assert sst.kstest(z, "norm").pvalue > 1e-4
    # cos/sin halves of a pair are uncorrelated
    assert abs(np.corrcoef(z[0:-1:2], z[1::2])[0, 1]) < 4 / math.sqrt(z.size / 2)


def _kat():
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    out = []
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            w = [int(v, 16) for v in line.split()]
            out.append((w[0:4], w[4:6], w[6:10]))
    return out


def test_philox_known_answer_vectors(orc):
    """The published Philox4x32-10 known-answer vectors (SC'11 / Random123)."""
    kat = _kat()
    assert len(kat) == 3
    for ctr, key, ref in kat:
        assert [int(v) for v in orc.philox4x32_10(ctr, key)] == ref, (ctr, key)


def test_philox_streams_are_distinct_and_mixing(orc):
    base = orc.normals(1, 2, 3, orc.TAG_MOM, 64)
    for other in (orc.normals(1, 2, 4, orc.TAG_MOM, 64), orc.normals(1, 3, 3, orc.TAG_MOM, 64),
                  orc.normals(1, 2, 3, orc.TAG_INIT, 64), orc.normals(2, 2, 3, orc.TAG_MOM, 64)):
        assert abs(np.corrcoef(base, other)[0, 1]) < 0.5
        assert not np.any(base == other)
    # avalanche: one flipped counter bit changes about half of the 128 output bits
    rng = np.random.default_rng(8)
    flips = []
    for _ in range(200):
        ctr = [int(v) for v in rng.integers(0, 2 ** 32, 4)]
        key = [int(v) for v in rng.integers(0, 2 ** 32, 2)]
        a = orc.philox4x32_10(ctr, key)
        w, b = int(rng.integers(0, 4)), int(rng.integers(0, 32))
        ctr[w] ^= 1 << b
        c = orc.philox4x32_10(ctr, key)
        flips.append(sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(a, c)))
    assert abs(np.mean(flips) - 64) < 2.0


def test_invalid_parameters_rejected(orc):
    with pytest.raises(ValueError):
        orc.force(orc.Lattice((4, 4), beta=0.4, C=3.9), np.zeros(16))  # C <= 2d
    with pytest.raises(ValueError):
        orc.force(orc.Lattice((2, 4), beta=0.4, C=4.1), np.zeros(8))  # L < 3
    with pytest.raises(ValueError):
        orc.force(orc.Lattice((4, 4), beta=-0.4, C=4.1), np.zeros(16))  # J' <= 0
    with pytest.raises(ValueError):
        orc.run(orc.Lattice((4, 4), beta=0.4, C=4.1), 3, 0)  # n_md < 1


def test_gamma_method_on_ar1():
    """AR(1) x_t = rho x_{t-1} + noise has tau_int = (1 + rho) / (2 (1 - rho))."""
    from oracle import stats as S
    rng = np.random.default_rng(10)
    rho, n = 0.8, 400000
    e = rng.standard_normal(n)
    x = np.empty(n)
    x[0] = e[0]
    for t in range(1, n):
        x[t] = rho * x[t - 1] + e[t]
    g = S.gamma_method(x)
    assert abs(g["tau_int"] - (1 + rho) / (2 * (1 - rho))) < 4 * g["tau_err"] + 0.05
