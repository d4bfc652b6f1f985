"""Monte Carlo error analysis: the Gamma method with automatic windowing.

TEST INFRASTRUCTURE (see ``oracle/__init__.py``).  The paper computes the
integrated autocorrelation time and its error with the scheme of U. Wolff,
"Monte Carlo errors with less errors" (Comput. Phys. Commun. 156 (2004) 143),
cited in Sec. 4.  This is a plain single-observable implementation of that
scheme (S_tau = 1.5, bias-corrected Gamma, Madras-Sokal error on tau_int).
"""
from __future__ import annotations

import math

import numpy as np


def gamma_method(x, s_tau=1.5):
    """Mean, its error, tau_int and the error of tau_int for a time series."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    if n < 4:
        raise ValueError("series too short")
    mean = x.mean()
    d = x - mean
    var = d @ d / n
    if var == 0.0:
        return dict(mean=mean, err=0.0, tau_int=0.5, tau_err=0.0, W=0)
    # autocorrelation by FFT
    f = np.fft.rfft(d, n=2 * n)
    acf = np.fft.irfft(f * np.conj(f))[:n] / np.arange(n, 0, -1)
    rho = acf / acf[0]
    tau = 0.5
    W = n - 1
    for w in range(1, n):
        tau += rho[w]
        if tau <= 0:
            tau_w = 1e-6
        else:
            tau_w = s_tau / math.log((2 * tau + 1) / (2 * tau - 1)) if tau > 0.5 else 1e-6
        g = math.exp(-w / tau_w) - tau_w / math.sqrt(w * n)
        if g < 0:
            W = w
            break
    # bias correction of the summed Gamma (Wolff eq. 49)
    c_w = acf[0] + 2 * acf[1:W + 1].sum()
    c_w *= 1 + (2 * W + 1) / n
    # anticorrelated series (e.g. with sign flips) can drive C_F below Gamma(0);
    # clamp tau_int at 1/2 so the error is never below the naive one
    tau_int = max(c_w / (2 * acf[0]), 0.5)
    err = math.sqrt(2 * tau_int * acf[0] / n)
    tau_err = tau_int * math.sqrt(4 * (W + 0.5 - tau_int) / n) if W > 0 else 0.0
    return dict(mean=mean, err=err, tau_int=tau_int, tau_err=tau_err, W=W)


def z_score(a, b, err):
    return abs(a - b) / err if err > 0 else (0.0 if a == b else math.inf)
