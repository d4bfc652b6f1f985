"""Seeded synthetic workloads, shared by the tests, the benchmark and the oracle runs.

This module only draws inputs (lattice shapes, couplings, fields, step counts);
it holds none of the method's arithmetic.  The method's own randomness (initial
field, momenta, accept uniforms) comes from Philox inside the library and the
oracle, keyed by the seed given here.

Workloads (the paper uses synthetic lattices only, Sec. 4):
  small      2D 8x8 torus, beta = 0.40, h = 0, C = 4.1, 10 MD steps, 2000 trajectories.
  large      2D 1024^2 at beta_c = ln(1+sqrt2)/2 and 3D 128^3 at beta = 0.2216544,
             h = 0, C = 2d + 0.1, 20 MD steps, 500 trajectories.
  batched    4096 2D tori, L log-uniform in [16, 256], beta ~ U[0.30, 0.55],
             h_x ~ N(0, 0.05^2) per site, n_md ~ U{8..32}, C = 4.1, 200 trajectories.
  dense      N = 4096, K_ij ~ N(0, 1/N) symmetric with zero diagonal, beta = 1, 256 chains.
  serving    Poisson arrivals; 2D or 3D tori, L ~ U{16..128} (3D U{16..64}),
             beta ~ U[0.2, 0.6], h ~ U[0, 0.1], n_traj ~ U{50..1000}, n_md ~ U{10..30}.
"""
from __future__ import annotations

import math

import numpy as np

BETA_C_2D = 0.5 * math.log(1.0 + math.sqrt(2.0))
BETA_3D = 0.2216544


def small():
    return dict(L=(8, 8), beta=0.40, C=4.1, h=None, n_md=10, n_traj=2000, seed=1)


def large():
    return [dict(L=(1024, 1024), beta=BETA_C_2D, C=4.1, h=None, n_md=20, n_traj=500, seed=2, chain_id=0),
            dict(L=(128, 128, 128), beta=BETA_3D, C=6.1, h=None, n_md=20, n_traj=500, seed=2, chain_id=1)]


def batched(n_chains=4096, seed=3, L_min=16, L_max=256):
    rng = np.random.Generator(np.random.PCG64(seed))
    L = np.rint(np.exp(rng.uniform(math.log(L_min), math.log(L_max), n_chains))).astype(int)
    beta = rng.uniform(0.30, 0.55, n_chains)
    n_md = rng.integers(8, 33, n_chains)
    out = []
    for i in range(n_chains):
        h = rng.normal(0.0, 0.05, int(L[i]) * int(L[i]))
        out.append(dict(L=(int(L[i]), int(L[i])), beta=float(beta[i]), C=4.1, h=h, n_md=int(n_md[i]),
                        n_traj=200, seed=seed, chain_id=i))
    return out


def dense(N=4096, n_chains=256, seed=4):
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.normal(0.0, 1.0 / math.sqrt(N), (N, N))
    K = np.triu(A, 1)
    K = K + K.T
    return dict(K=K, beta=1.0, h=None, n_chains=n_chains, n_md=16, n_traj=100, seed=seed)


def serving(rate=200.0, duration=60.0, seed=5):
    rng = np.random.Generator(np.random.PCG64(seed))
    t, reqs = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        d = 2 if rng.random() < 0.5 else 3
        L = int(rng.integers(16, 129)) if d == 2 else int(rng.integers(16, 65))
        reqs.append(dict(t=t, L=(L,) * d, beta=float(rng.uniform(0.2, 0.6)), C=2 * d + 0.1,
                         h=float(rng.uniform(0.0, 0.1)), n_traj=int(rng.integers(50, 1001)),
                         n_md=int(rng.integers(10, 31)), seed=seed, chain_id=len(reqs)))
    return reqs


def gaussian_field(rng, N, scale=1.0):
    return rng.standard_normal(N) * scale
