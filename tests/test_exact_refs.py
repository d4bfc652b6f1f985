"""Cross-checks between independent exact references (no HMC involved).

Each reference is a different computation of the same spin-model partition
sum, so agreement pins all of them: enumeration of 2^N states, the row
transfer matrix, the 1D closed form and the appendix formula of the
infinite-range model (App. A, eq. all-to-all partition function).
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import exact as E

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "spin_model_exact.json")


@pytest.mark.parametrize("L0,L1,beta", [(4, 4, 0.4), (3, 4, 0.3), (4, 3, 0.5), (4, 4, E.BETA_C_2D)])
def test_row_transfer_matches_enumeration(L0, L1, beta):
    bf = E.brute_force(E.torus_adjacency((L0, L1)), beta)
    tm = E.row_transfer_2d(L0, L1, beta)
    assert abs(bf["be"] - tm["be"]) < 1e-12
    assert abs(bf["m2"] - tm["m2"]) < 1e-12


@pytest.mark.parametrize("N,beta,h", [(12, 0.5, 0.1), (9, 0.3, -0.2), (10, 1.0, 0.0)])
def test_ring_closed_form_matches_enumeration(N, beta, h):
    bf = E.brute_force(E.torus_adjacency((N,)), beta, h=h)
    cf = E.ring_1d(N, beta, h=h)
    assert abs(bf["be"] - cf["be"]) < 1e-12
    assert abs(bf["m"] - cf["m"]) < 1e-12


@pytest.mark.parametrize("N,betaJ,bh", [(8, 1.0, 0.0), (12, 1.0, 0.0), (10, 0.7, 0.05)])
def test_appendix_formula_matches_enumeration(N, betaJ, bh):
    bf = E.brute_force(E.infinite_range_K(N), betaJ, h=bh / betaJ)
    ap = E.infinite_range(N, betaJ, beta_h=bh)
    assert abs(bf["be"] - ap["be"]) < 1e-12
    assert abs(bf["m"] - ap["m"]) < 1e-12
    assert abs(bf["m2"] - ap["m2"]) < 1e-12


def test_torus_spectrum():
    """Spectrum of K lies in [-n, n] (eq. eigen_spectrum_K); -2d is reached for even L."""
    for L in [(4, 4), (6,), (4, 4, 4), (5, 5), (3, 3, 3)]:
        lam = np.linalg.eigvalsh(E.torus_adjacency(L))
        d = len(L)
        assert lam.max() == pytest.approx(2 * d, abs=1e-12)
        if all(v % 2 == 0 for v in L):
            assert lam.min() == pytest.approx(-2 * d, abs=1e-12)
        else:
            assert lam.min() > -2 * d + 1e-3


def test_onsager_critical_energy():
    """At beta_c the Onsager energy is -sqrt(2) J per site."""
    assert E.onsager_energy(E.BETA_C_2D) == pytest.approx(-math.sqrt(2) * E.BETA_C_2D, rel=1e-14)


def test_onsager_vs_transfer_matrix_high_temperature():
    """Finite-size corrections vanish exponentially away from beta_c: 10x10 at beta = 0.25."""
    tm = E.row_transfer_2d(10, 10, 0.25)
    assert abs(tm["be"] - E.onsager_energy(0.25)) < 2e-4


def test_ferdinand_fisher_is_leading_order_only():
    """The quoted expansion agrees with the exact 8x8 value to O(1/N)."""
    tm = E.row_transfer_2d(8, 8, E.BETA_C_2D)
    assert abs(tm["be"] - E.ferdinand_fisher_leading(64)) < 5e-3


def test_against_independent_values():
    """The exact references against values computed independently of them
    (tests/golden/spin_model_exact.json, printed to 10 decimals)."""
    with open(GOLDEN) as f:
        g = json.load(f)
    assert len(g["values"]) >= 7
    for rec in g["values"]:
        kind, args, ref = rec["kind"], rec["args"], rec["value"]
        if kind == "brute_force":
            got = E.brute_force(E.torus_adjacency(args["L"]), args["beta"], h=args["h"])
        elif kind == "row_transfer_2d":
            got = E.row_transfer_2d(args["L"][0], args["L"][1], args["beta"])
        elif kind == "ring_1d":
            got = E.ring_1d(args["N"], args["beta"], h=args["h"])
        elif kind == "infinite_range":
            got = E.infinite_range(args["N"], args["betaJ"])
        else:
            raise AssertionError(kind)
        for k, v in ref.items():
            assert abs(got[k] - v) < 1e-10, (rec, k, got[k])
