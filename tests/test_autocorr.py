"""Gamma-method analysis of the package (host side), pinned against closed forms
for autoregressive series and against the oracle's independent implementation."""
import math

import numpy as np
import pytest

from paper_1912_03278_amd import autocorr as A


def ar1(rng, phi, n, reps=1):
    """x_t = phi x_{t-1} + e_t started in equilibrium: tau_int = (1+phi)/(2(1-phi))."""
    e = rng.standard_normal((reps, n))
    x = np.empty((reps, n))
    x[:, 0] = e[:, 0] / math.sqrt(1 - phi * phi)
    for t in range(1, n):
        x[:, t] = phi * x[:, t - 1] + e[:, t]
    return x


def test_independent_series():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(40000)
    g = A.gamma_method(x)
    assert abs(g["tau_int"] - 0.5) < 3 * g["tau_err"] + 0.02
    assert g["err"] == pytest.approx(x.std() / math.sqrt(x.size), rel=0.1)
    assert g["mean"] == pytest.approx(x.mean(), abs=1e-15)


@pytest.mark.parametrize("phi", [0.5, 0.8, 0.95])
def test_ar1_tau_int_closed_form(phi):
    rng = np.random.default_rng(int(phi * 100))
    x = ar1(rng, phi, 20000, reps=8)
    g = A.gamma_method(list(x))
    exact = (1 + phi) / (2 * (1 - phi))
    assert abs(g["tau_int"] - exact) < 4 * g["tau_err"], (g["tau_int"], exact, g["tau_err"])
    # the error of the mean: sqrt(2 tau_int var / N) with the exact tau_int and variance
    var = 1.0 / (1 - phi * phi)
    assert g["err"] == pytest.approx(math.sqrt(2 * exact * var / x.size), rel=0.15)


def test_error_of_the_mean_matches_spread_of_replica_means():
    """The Gamma-method error of one run agrees with the spread of the means of
    many independent runs (AR(1), tau_int = 2.5)."""
    rng = np.random.default_rng(7)
    runs = ar1(rng, 2.0 / 3.0, 4000, reps=200)
    errs = [A.gamma_method(r)["err"] for r in runs[:20]]
    spread = runs.mean(axis=1).std(ddof=1)
    assert np.mean(errs) == pytest.approx(spread, rel=0.2)


def test_replicas_pool_like_one_long_chain():
    rng = np.random.default_rng(3)
    x = ar1(rng, 0.7, 50000, reps=1)[0]
    one = A.gamma_method(x)
    four = A.gamma_method([x[:12500], x[12500:25000], x[25000:37500], x[37500:]])
    assert four["mean"] == pytest.approx(one["mean"], abs=1e-14)
    assert four["tau_int"] == pytest.approx(one["tau_int"], abs=3 * one["tau_err"])


def test_agrees_with_oracle_implementation(orc):
    """The oracle's Gamma method (separate code) differs only in the O(1/N)
    bias correction of Gamma(0)."""
    from oracle import stats
    rng = np.random.default_rng(11)
    for phi in (0.3, 0.9):
        x = ar1(rng, phi, 30000)[0]
        a = A.gamma_method(x)
        b = stats.gamma_method(x)
        assert a["mean"] == b["mean"]
        assert a["W"] == b["W"]
        assert a["tau_int"] == pytest.approx(b["tau_int"], rel=5 * (2 * a["W"] + 1) / x.size)
        assert a["err"] == pytest.approx(b["err"], rel=5 * (2 * a["W"] + 1) / x.size)


def test_constant_and_short_series():
    g = A.gamma_method(np.ones(100))
    assert g["tau_int"] == 0.5 and g["err"] == 0.0
    with pytest.raises(ValueError):
        A.gamma_method(np.ones(3))


def test_power_fits_recover_exact_laws():
    N = np.array([16.0, 64.0, 256.0, 1024.0])
    tau = 0.3 * N ** 1.1
    f = A.fit_power(N, tau, 0.05 * tau)
    assert f["alpha"] == pytest.approx(0.3, rel=1e-10) and f["gamma"] == pytest.approx(1.1, rel=1e-10)
    g = A.fit_power(N, tau, 0.05 * tau, exponent=1.1)
    assert g["alpha"] == pytest.approx(0.3, rel=1e-10) and g["chi2_dof"] < 1e-18


def test_md_steps_rule():
    # the paper's N_step = floor(log N), natural logarithm
    assert [A.md_steps(N) for N in (16, 64, 225, 1024, 4096, 32768)] == [2, 4, 5, 6, 8, 10]
