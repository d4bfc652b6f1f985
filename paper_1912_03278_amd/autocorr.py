"""Integrated autocorrelation times of HMC observables, and the scans that
measure critical slowing down (Sec. 4, the tau_int(N) and tau_int(C) studies).

The error analysis follows the Gamma method of U. Wolff, "Monte Carlo errors
with less errors", Comput. Phys. Commun. 156 (2004) 143 -- the scheme the paper
cites for tau_int and its error:

  * the autocovariance Gamma(t) of an observable, estimated over R independent
    replicas around the common mean;
  * the integrated time tau_int(W) = 1/2 + sum_{t=1..W} Gamma(t)/Gamma(0),
    summed up to the first window W where the estimated systematic error
    exp(-W/tau) falls below the statistical one sqrt(W/N) tau (with
    tau = S / log((2 tau_int + 1) / (2 tau_int - 1)), S = 1.5);
  * Gamma corrected for the bias of the estimated mean by C_F/N, the error of
    the mean sqrt(C_F / N), and the error of tau_int from the Madras-Sokal
    formula 2 tau_int sqrt((W + 1/2 - tau_int) / N).

Host-side analysis of the series the GPU chains return (numpy); the chains
themselves run in the HIP library.
"""
from __future__ import annotations

import math
import time

import numpy as np


def _autocov(replicas, mean, t_max):
    """Gamma(t), t = 0 .. t_max, pooled over replicas (sum of lagged products
    divided by the number of pairs)."""
    num = np.zeros(t_max + 1)
    pairs = np.zeros(t_max + 1)
    for a in replicas:
        d = a - mean
        n = d.size
        m = 1 << int(math.ceil(math.log2(2 * n)))
        f = np.fft.rfft(d, m)
        c = np.fft.irfft(f * np.conj(f), m)[: min(n, t_max + 1)]
        num[: c.size] += c
        pairs[: c.size] += np.arange(n, n - c.size, -1)
    ok = pairs > 0
    g = np.zeros(t_max + 1)
    g[ok] = num[ok] / pairs[ok]
    return g[ok]


def gamma_method(series, s_tau=1.5):
    """Mean, its error, tau_int and its error for one observable.

    `series`: one 1-D array (a single Markov chain) or a list of them
    (independent replicas of the same chain, pooled).  Returns a dict with
    mean, err, tau_int, tau_err, W (the window), n (total measurements) and
    rho (the normalised autocorrelation up to W)."""
    reps = [np.asarray(series, dtype=np.float64)] if np.ndim(series[0]) == 0 else \
        [np.asarray(a, dtype=np.float64) for a in series]
    reps = [a for a in reps if a.size > 0]
    n = sum(a.size for a in reps)
    if n < 4 or max(a.size for a in reps) < 2:
        raise ValueError("series too short for the Gamma method")
    mean = sum(a.sum() for a in reps) / n
    t_max = max(a.size for a in reps) // 2
    gam = _autocov(reps, mean, t_max)
    if gam[0] <= 0.0:
        return dict(mean=mean, err=0.0, tau_int=0.5, tau_err=0.0, W=0, n=n, rho=np.ones(1))
    # automatic window
    rho = gam / gam[0]
    tau_w = 0.5 + np.cumsum(rho[1:])
    W = rho.size - 1
    for w in range(1, rho.size):
        ti = tau_w[w - 1]
        tau = s_tau / math.log((2 * ti + 1) / (2 * ti - 1)) if ti > 0.5 else 1e-12
        if math.exp(-w / tau) - tau / math.sqrt(w * n) < 0.0:
            W = w
            break
    # bias of the mean: Gamma(t) + C_F / N, then the refined C_F
    cf = gam[0] + 2.0 * gam[1:W + 1].sum()
    gam_c = gam[: W + 1] + cf / n
    cf = gam_c[0] + 2.0 * gam_c[1:].sum()
    tau_int = cf / (2.0 * gam_c[0])
    tau_err = 2.0 * tau_int * math.sqrt(max(W + 0.5 - tau_int, 0.0) / n)
    err = math.sqrt(max(cf, 0.0) / n)
    return dict(mean=mean, err=err, tau_int=tau_int, tau_err=tau_err, W=W, n=n, rho=gam_c / gam_c[0])


def fit_power(N, tau, tau_err, exponent=None):
    """Weighted least-squares fit of tau = alpha N^gamma in log space.

    With `exponent` given, gamma is fixed (the paper's fits use 2/d) and only
    alpha is fitted.  Returns dict(alpha, alpha_err, gamma, gamma_err, chi2_dof)."""
    N = np.asarray(N, dtype=np.float64)
    y = np.log(np.asarray(tau, dtype=np.float64))
    s = np.asarray(tau_err, dtype=np.float64) / np.asarray(tau, dtype=np.float64)
    w = 1.0 / np.maximum(s, 1e-12) ** 2
    x = np.log(N)
    if exponent is not None:
        r = y - exponent * x
        la = (w * r).sum() / w.sum()
        la_err = math.sqrt(1.0 / w.sum())
        chi2 = float((w * (r - la) ** 2).sum())
        dof = max(len(N) - 1, 1)
        return dict(alpha=math.exp(la), alpha_err=math.exp(la) * la_err, gamma=float(exponent), gamma_err=0.0,
                    chi2_dof=chi2 / dof)
    A = np.stack([np.ones_like(x), x], axis=1)
    Aw = A * w[:, None]
    cov = np.linalg.inv(A.T @ Aw)
    p = cov @ (Aw.T @ y)
    r = y - A @ p
    chi2 = float((w * r * r).sum())
    dof = max(len(N) - 2, 1)
    return dict(alpha=math.exp(p[0]), alpha_err=math.exp(p[0]) * math.sqrt(cov[0, 0]), gamma=float(p[1]),
                gamma_err=math.sqrt(cov[1, 1]), chi2_dof=chi2 / dof)


def md_steps(N):
    """MD steps per unit trajectory that the paper uses: floor(log N) (natural log)."""
    return max(1, int(math.floor(math.log(N))))


def run_scan(ctx, points, n_chains, n_traj, n_therm, seed=1, precision=4, observable="abs_m", flip_every=0):
    """tau_int of `observable` for several lattices, each with n_chains
    independent replicas, all advanced together as one batched chain set.

    `points`: list of dicts with L (tuple), beta, C and optionally n_md (default
    md_steps(N)) and h.  Every chain runs n_therm + n_traj unit trajectories;
    the first n_therm are discarded.  Returns one dict per point with the Gamma
    method result, the acceptance, the point's site-MD-steps and the wall time
    of the whole batched run (run_s, the same for every point)."""
    from . import ihmc
    lats, runs, owner = [], [], []
    for k, pt in enumerate(points):
        N = int(np.prod(pt["L"]))
        n_md = int(pt.get("n_md", md_steps(N)))
        for r in range(n_chains):
            lats.append(ihmc.Lattice(tuple(pt["L"]), beta=pt["beta"], C=pt["C"], h=pt.get("h")))
            runs.append(ihmc.Run(n_md=n_md, n_traj=n_therm + n_traj, precision=precision, seed=seed,
                                 chain_id=k * n_chains + r, flip_every=flip_every))
            owner.append(k)
    ch = ihmc.Chains(ctx, lats, runs)
    try:
        t0 = time.perf_counter()
        ch.advance(n_therm + n_traj)
        ctx.sync()
        run_s = time.perf_counter() - t0
        series = [[] for _ in points]
        acc = [[] for _ in points]
        for i, k in enumerate(owner):
            r = ch.result(i, want_psi=False)
            series[k].append(np.asarray(r[observable])[n_therm:])
            acc[k].append(r["acceptance"])
    finally:
        ch.close()
    out = []
    for k, pt in enumerate(points):
        N = int(np.prod(pt["L"]))
        n_md = int(pt.get("n_md", md_steps(N)))
        g = gamma_method(series[k])
        out.append(dict(L=tuple(pt["L"]), N=N, beta=pt["beta"], C=pt["C"], n_md=n_md, chains=n_chains,
                        trajectories=n_traj, mean=g["mean"], err=g["err"], tau_int=g["tau_int"],
                        tau_err=g["tau_err"], W=g["W"], acceptance=float(np.mean(acc[k])),
                        site_md_steps=N * n_md * (n_therm + n_traj) * n_chains, run_s=run_s))
    return out
