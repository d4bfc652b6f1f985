"""Exact references for the Ising model, independent of the HMC oracle.

TEST INFRASTRUCTURE (see ``oracle/__init__.py``).  These are the pins the HMC
oracle is checked against: they compute the spin-model expectation values
directly from the spin partition sum, never through the auxiliary field.

* ``brute_force``       -- enumerate all 2^N spin states of any symmetric K
                           (Sec. 2, partition sum Z = sum_s exp(-beta H)).
* ``row_transfer_2d``   -- row-to-row transfer matrix of an L0 x L1 torus.
* ``ring_1d``           -- closed form of the periodic chain (2x2 transfer matrix).
* ``infinite_range``    -- App. A, eq. all-to-all partition function and the
                           energy formula that follows it.
* ``onsager_energy`` / ``yang_magnetisation`` -- the textbook 2D solutions
                           (Onsager 1944, Yang 1952) cited in Sec. 1 and Sec. 4.
* ``ferdinand_fisher_leading`` -- the leading-order finite-size energy at
                           criticality quoted in Sec. 4.
* ``sample_psi_given_s`` -- the exact conditional distribution of the field:
                           eqs. did_HS_trafo and phi_psi_substitution imply
                           psi | s ~ Normal(sqrt(J') s + Kt^-1 h'/sqrt(J'), Kt^-1).

Conventions: periodic boundaries, m = sum(s)/N, beta*eps = beta*H/N.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special


def torus_adjacency(L):
    """K for the periodic nearest-neighbour lattice, multiplicities counted."""
    L = tuple(int(v) for v in L)
    N = int(np.prod(L))
    K = np.zeros((N, N))
    coords = np.array(np.unravel_index(np.arange(N), L[::-1])).T[:, ::-1]  # x fastest
    strides = [int(np.prod(L[:i])) for i in range(len(L))]
    for s in range(N):
        c = coords[s]
        for mu in range(len(L)):
            for d in (1, -1):
                cc = c.copy()
                cc[mu] = (cc[mu] + d) % L[mu]
                t = int(sum(int(cc[i]) * strides[i] for i in range(len(L))))
                K[s, t] += 1.0
    return K


def infinite_range_K(N):
    """K_ij = 1/N for i != j (App. A with J-hat = J/N)."""
    return (np.ones((N, N)) - np.eye(N)) / N


def _all_states(N):
    idx = np.arange(2 ** N, dtype=np.int64)
    bits = (idx[:, None] >> np.arange(N)) & 1
    return (2 * bits - 1).astype(np.float64)


def brute_force(K, beta, J=1.0, h=0.0):
    """Exact <beta*eps>, <m>, <m^2>, <|m|> by enumerating 2^N states.

    H(s) = -1/2 J s^T K s - h.s (eq. hamilton_matrix_notation)."""
    K = np.asarray(K, dtype=np.float64)
    N = K.shape[0]
    if N > 22:
        raise ValueError("too many sites for enumeration")
    hv = np.broadcast_to(np.asarray(h, dtype=np.float64), (N,))
    out = {}
    S = _all_states(N)
    E = -0.5 * J * np.einsum("ki,ij,kj->k", S, K, S) - S @ hv
    emin = E.min()
    w = np.exp(-beta * (E - emin))
    Z = w.sum()
    m = S.sum(axis=1) / N
    out["be"] = float((w * beta * E / N).sum() / Z)
    out["m"] = float((w * m).sum() / Z)
    out["m2"] = float((w * m * m).sum() / Z)
    out["am"] = float((w * np.abs(m)).sum() / Z)
    out["logZ"] = float(np.log(Z) - beta * emin)
    return out


def boltzmann_weights(K, beta, J=1.0, h=0.0):
    """All states and their normalised Boltzmann probabilities."""
    K = np.asarray(K, dtype=np.float64)
    N = K.shape[0]
    hv = np.broadcast_to(np.asarray(h, dtype=np.float64), (N,))
    S = _all_states(N)
    E = -0.5 * J * np.einsum("ki,ij,kj->k", S, K, S) - S @ hv
    w = np.exp(-beta * (E - E.min()))
    return S, w / w.sum()


def row_transfer_2d(L0, L1, beta, J=1.0):
    """Exact <beta*eps>, <m^2> on an L0 x L1 torus at h = 0 by the row transfer matrix.

    Rows of L0 spins; T(a, b) = exp(beta J [r(a)/2 + v(a, b) + r(b)/2]) where r is the
    intra-row bond sum and v the inter-row bond sum, so Z = Tr T^L1."""
    S = _all_states(L0)  # (2^L0, L0)
    r = (S * np.roll(S, -1, axis=1)).sum(axis=1)
    v = S @ S.T
    M = S.sum(axis=1)
    A = beta * J * (0.5 * r[:, None] + v + 0.5 * r[None, :])
    shift = A.max()
    T = np.exp(A - shift)
    lam, V = np.linalg.eigh(T)
    n = L1
    Z = float((lam ** n).sum())
    # energy: -J [sum over rows r + sum over row pairs v]; by translation
    # invariance = L1 * (<r(row0)> + <v(row0,row1)>).
    Dr = V.T @ (r[:, None] * V)
    e_r = float(np.einsum("a,aa->", lam ** n, Dr)) / Z
    Av = V.T @ ((v * T) @ V)
    e_v = float(np.einsum("a,aa->", lam ** (n - 1), Av)) / Z
    N = L0 * L1
    be = -beta * J * L1 * (e_r + e_v) / N
    # <M_total^2> = sum_{j,k} <M_j M_k> = L1 * sum_k <M_0 M_k>
    DM = V.T @ (M[:, None] * V)
    tot = 0.0
    for k in range(n):
        tot += float(np.einsum("ab,ab,a,b->", DM, DM, lam ** k, lam ** (n - k)))
    m2 = L1 * tot / Z / N ** 2
    return dict(be=be, m2=m2)


def ring_1d(N, beta, J=1.0, h=0.0):
    """Periodic chain: Z = l+^N + l-^N with
    l+- = e^{bJ}[cosh(bh) +- sqrt(sinh^2(bh) + e^{-4bJ})].
    Derivatives by complex-step differentiation of log Z (exact to rounding)."""
    def logZ(b, hh):
        a = np.exp(b * J)
        root = np.sqrt(np.sinh(b * hh) ** 2 + np.exp(-4 * b * J))
        lp = a * (np.cosh(b * hh) + root)
        lm = a * (np.cosh(b * hh) - root)
        return N * np.log(lp) + np.log(1 + (lm / lp) ** N)
    d = 1e-30
    dlogZ_db = (logZ(beta + 1j * d, h + 0j)).imag / d
    # <m> = (1/(N beta)) d logZ / dh
    dlogZ_dh = (logZ(beta + 0j, h + 1j * d)).imag / d
    return dict(be=float(-beta * dlogZ_db / N), m=float(dlogZ_dh / (N * beta)))


def infinite_range(N, betaJ, beta_h=0.0):
    """App. A: exact <beta*eps>, <m> and <m^2> of H = -(J/2N) sum_{i!=j} s_i s_j - h sum s_i.

    Z = e^{-beta J/2} sum_n C(N,n) f(beta J/N, beta h, N - 2n) with
    f(a, b, x) = exp(a x^2 / 2 + b x); the e^{-beta J/2} prefactor follows from
    H = J/2 - (J/2N)(sum s)^2 - h sum s (the appendix prints the exponent with
    the opposite sign; the prefactor cancels in <beta*eps> either way)."""
    n = np.arange(N + 1)
    x = (N - 2 * n).astype(np.float64)
    logc = np.array([math.lgamma(N + 1) - math.lgamma(k + 1) - math.lgamma(N - k + 1) for k in n])
    a = betaJ / N
    logw = logc + 0.5 * a * x * x + beta_h * x
    w = np.exp(logw - logw.max())
    Z = w.sum()
    # beta*E(x) = beta J/2 - a x^2 / 2 - beta_h x
    be = 0.5 * betaJ / N - float((w * (0.5 * a * x * x + beta_h * x)).sum() / Z) / N
    m = float((w * x).sum() / Z) / N
    # the same weights give every moment of the magnetisation x / N
    m2 = float((w * x * x).sum() / Z) / (N * N)
    return dict(be=be, m=m, m2=m2)


BETA_C_2D = 0.5 * math.log(1.0 + math.sqrt(2.0))


def onsager_energy(beta, J=1.0):
    """Onsager: energy per site of the infinite square lattice, times beta.

    u = -J coth(2K) [1 + (2/pi)(2 tanh^2(2K) - 1) K1(k)],  K = beta J,
    k = 2 sinh(2K)/cosh^2(2K), K1 the complete elliptic integral of the first kind."""
    K = beta * J
    k = 2 * math.sinh(2 * K) / math.cosh(2 * K) ** 2
    c = 2 * math.tanh(2 * K) ** 2 - 1
    # at the critical point c = 0 while K1 diverges logarithmically: the product vanishes
    term = 0.0 if abs(c) < 1e-13 else c * special.ellipk(k * k)
    u = -J / math.tanh(2 * K) * (1 + 2 / math.pi * term)
    return beta * u


def yang_magnetisation(beta, J=1.0):
    """Spontaneous magnetisation of the square lattice, (1 - sinh^-4(2 beta J))^(1/8)."""
    s = math.sinh(2 * beta * J)
    return (1 - s ** -4) ** 0.125 if beta > BETA_C_2D else 0.0


def ferdinand_fisher_leading(N):
    """Leading-order energy at criticality quoted in Sec. 4:
    -log(1+sqrt2) (sqrt2/2 + 1/(3 sqrt N))."""
    return -math.log(1 + math.sqrt(2)) * (math.sqrt(2) / 2 + 1 / (3 * math.sqrt(N)))


def sample_psi_given_s(rng, s, Kt, Jp, hp=None):
    """Draw psi | s ~ Normal(sqrt(J') s + Kt^-1 h'/sqrt(J'), Kt^-1) for a batch of
    spin states s (rows).  Follows from the joint density in eq. did_HS_trafo after
    the substitution of eq. phi_psi_substitution."""
    s = np.atleast_2d(s)
    n = s.shape[1]
    Lc = np.linalg.cholesky(Kt)  # Kt = Lc Lc^T; Kt^-1 = Lc^-T Lc^-1
    xi = rng.standard_normal(s.shape)
    noise = np.linalg.solve(Lc.T, xi.T).T
    mean = math.sqrt(Jp) * s
    if hp is not None:
        mean = mean + np.linalg.solve(Kt, np.broadcast_to(hp, (n,)))[None, :] / math.sqrt(Jp)
    return mean + noise
