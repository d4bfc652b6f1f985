#!/usr/bin/env python3
"""Throughput benchmark of the fused lattice HMC path on one MI355X.

Workload (default, "large"): two single large chains, FP32 state with FP64
Hamiltonian reductions, J = 1, h = 0, 20 leap-frog steps per unit trajectory:
  * 2D 1024 x 1024 torus at beta_c = ln(1 + sqrt 2)/2, C = 4.1;
  * 3D 128^3 torus at beta = 0.2216544, C = 6.1.
Seeded Gaussian initial fields (Philox).  One step = one HMC trajectory of both
chains (21 fused passes each, Metropolis on the device); the metric is
site-MD-steps/s = (sites x MD steps) per second over the timed steps.

Besides the throughput line it reports the roofline of the dominant kernel (the
fused middle pass: 16 bytes of state per site, HIP-event timed on the library's
stream) and the FP64 CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
BYTES_MIDDLE_F32 = 16  # read psi, read p, write p, write psi' (FP32), h = 0


def large_workload():
    from paper_1912_03278_amd import inputs
    return inputs.large()


def cpu_baseline(chains):
    """The FP64 oracle, single-threaded, one trajectory of each chain."""
    import oracle
    t_total, work = 0.0, 0
    for w in chains:
        lat = oracle.Lattice(w["L"], beta=w["beta"], C=w["C"])
        t0 = time.perf_counter()
        oracle.run(lat, 1, w["n_md"], seed=w["seed"], chain_id=w["chain_id"])
        t_total += time.perf_counter() - t0
        work += int(math.prod(w["L"])) * w["n_md"]
    return dict(value=work / t_total, unit="site-MD-steps/s", cores=1, kind="oracle",
                sample="one trajectory (20 MD steps) of the 1024^2 and the 128^3 chain, FP64, "
                       f"{t_total:.1f} s on one host core")


def bench_batched(args):
    """4096 independent 2D tori of uneven size, beta, per-site field and step count,
    advanced together (one step = one trajectory of every chain), against the same
    chains run one at a time (the plain form) on a sample."""
    import numpy as np
    import torch
    from paper_1912_03278_amd import ihmc, inputs

    ws = inputs.batched(n_chains=args.chains)
    K, W = args.steps, args.warmup
    ctx = ihmc.Context(device=0, arena_bytes=6 << 30)
    lats = [ihmc.Lattice(w["L"], beta=w["beta"], C=w["C"], h=w["h"]) for w in ws]
    runs = [ihmc.Run(n_md=w["n_md"], n_traj=W + K, precision=ihmc.F32, seed=w["seed"], chain_id=w["chain_id"])
            for w in ws]
    t0 = time.perf_counter()
    chains = ihmc.Chains(ctx, lats, runs)
    t_setup = time.perf_counter() - t0
    print(f"bench: {len(ws)} chains ready in {t_setup:.1f} s", file=sys.stderr, flush=True)
    chains.advance(W)
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chains.advance(K)
    ctx.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    work = sum(int(math.prod(w["L"])) * w["n_md"] for w in ws)
    value = K * work / dt
    print(f"bench: timed {K} rounds in {dt:.3f} s", file=sys.stderr, flush=True)

    # plain form: a sample of chains, each alone, same parameters; bitwise comparison
    rng = np.random.default_rng(0)
    sample = sorted(rng.choice(len(ws), size=min(args.plain_sample, len(ws)), replace=False).tolist())
    plain_time, plain_work, identical, mismatch = 0.0, 0, True, []
    for i in sample:
        alone = ihmc.Chains(ctx, [lats[i]], [ihmc.Run(n_md=ws[i]["n_md"], n_traj=W + K, precision=ihmc.F32,
                                                      seed=ws[i]["seed"], chain_id=ws[i]["chain_id"])])
        alone.advance(W)
        ctx.sync()
        t0 = time.perf_counter()
        alone.advance(K)
        ctx.sync()
        plain_time += time.perf_counter() - t0
        plain_work += K * int(math.prod(ws[i]["L"])) * ws[i]["n_md"]
        a = alone.result(0, want_psi=False)
        b = chains.result(i, want_psi=False)
        same = bool(np.array_equal(a["dH"], b["dH"]) and np.array_equal(a["beta_eps"], b["beta_eps"]))
        if not same:
            mismatch.append(i)
        identical &= same
        alone.close()
    acc = [chains.result(i, want_psi=False)["acceptance"] for i in range(0, len(ws), max(1, len(ws) // 64))]

    kern = []
    for g in range(chains.groups()):
        mid = chains.time_pass(g, mode=1, reps=args.timing_reps)
        kern.append(dict(ndim=mid["ndim"], sites=mid["sites"], middle_us=round(mid["us"], 2),
                         middle_GBs=round(20 * mid["sites"] / (mid["us"] * 1e-6) / 1e9, 1)))
    dom = max(kern, key=lambda k: k["middle_us"])
    achieved = 20 * dom["sites"] / (dom["middle_us"] * 1e-6) / 1e9
    copy_bytes = 512 << 20
    copy_gbs = 2 * copy_bytes / (ctx.copy_bandwidth(copy_bytes, reps=10) * 1e-6) / 1e9
    line = {
        "metric": "site-MD-steps/s", "value": value, "unit": "site-MD-steps/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": 1000.0 * dt / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched: {len(ws)} 2D tori, L log-uniform [16,256], beta U[0.30,0.55], "
                               "h_x ~ N(0,0.05^2) per site, n_md U{8..32}, C=4.1, FP32 state, FP64 H; "
                               "one step = one trajectory of every chain",
                   "chains": len(ws), "sites": sum(int(math.prod(w["L"])) for w in ws)},
        "roofline": {"bound": "hbm", "kernel": "fused middle pass, 2D, per-site field (large-tile group)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_launch": 20 * dom["sites"], "avg_launch_us": dom["middle_us"],
                     "copy_kernel_GBs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)},
        "kernels": kern,
        "plain": {"chains": len(sample), "value": (plain_work / plain_time) if plain_time > 0 else None,
                  "unit": "site-MD-steps/s", "bitwise_equal_to_batched": identical if sample else None,
                  "mismatched_chains": mismatch},
        "acceptance_sample_mean": float(np.mean(acc)),
        "setup_s": round(t_setup, 2),
        "cpu_baseline": None,
    }
    chains.close()
    ctx.close()
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="large", choices=["large", "batched"],
                    help="large (default): the 1024^2 + 128^3 single chains; batched: 4096 uneven chains")
    ap.add_argument("--chains", type=int, default=4096, help="batched: number of chains")
    ap.add_argument("--plain-sample", type=int, default=16, help="batched: chains rerun alone")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle timing")
    ap.add_argument("--timing-reps", type=int, default=100)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; the multi-GPU sharding is described in "
              "DESIGN.md and is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        args.steps = 10 if args.steps is None else args.steps
        args.warmup = 2 if args.warmup is None else args.warmup
        return bench_batched(args)
    args.steps = 200 if args.steps is None else args.steps
    args.warmup = 20 if args.warmup is None else args.warmup

    import torch
    from paper_1912_03278_amd import ihmc

    ws = large_workload()
    K, W = args.steps, args.warmup
    ctx = ihmc.Context(device=0, arena_bytes=2 << 30)
    lats = [ihmc.Lattice(w["L"], beta=w["beta"], C=w["C"]) for w in ws]
    runs = [ihmc.Run(n_md=w["n_md"], n_traj=W + K, precision=ihmc.F32, seed=w["seed"], chain_id=w["chain_id"])
            for w in ws]
    chains = ihmc.Chains(ctx, lats, runs)
    print(f"bench: chains ready ({', '.join('x'.join(map(str, w['L'])) for w in ws)})", file=sys.stderr, flush=True)
    chains.advance(W)
    ctx.sync()
    print(f"bench: warmup {W} trajectories done", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    ctx.sync()
    t0 = time.perf_counter()
    chains.advance(K)
    ctx.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = t1 - t0
    site_steps = sum(int(math.prod(w["L"])) * w["n_md"] for w in ws)
    value = K * site_steps / dt
    print(f"bench: timed {K} steps in {dt:.3f} s", file=sys.stderr, flush=True)

    per = []
    for i, w in enumerate(ws):
        r = chains.result(i, want_psi=False)
        per.append(dict(lattice="x".join(map(str, w["L"])), beta=w["beta"], acceptance=round(r["acceptance"], 4),
                        n_traj_done=r["n_traj_done"], n_nonfinite=r["n_nonfinite"],
                        mean_beta_eps_last=float(r["beta_eps"][-1])))

    # ---- roofline of the dominant kernel: HIP-event timing of each fused pass kind
    kern = []
    for g in range(chains.groups()):
        mid = chains.time_pass(g, mode=1, reps=args.timing_reps)
        first = chains.time_pass(g, mode=0, reps=max(10, args.timing_reps // 5))
        n_md = ws[g]["n_md"]  # groups are ordered (precision, ndim): 2D then 3D, one chain each
        kern.append(dict(ndim=mid["ndim"], sites=mid["sites"], middle_us=mid["us"], first_us=first["us"],
                         middle_share_us=(n_md - 1) * mid["us"]))
    dom = max(kern, key=lambda k: k["middle_share_us"])
    bytes_per_launch = BYTES_MIDDLE_F32 * dom["sites"]
    achieved = bytes_per_launch / (dom["middle_us"] * 1e-6) / 1e9
    for k in kern:
        k["middle_GBs"] = round(BYTES_MIDDLE_F32 * k["sites"] / (k["middle_us"] * 1e-6) / 1e9, 1)
        k["middle_us"] = round(k["middle_us"], 3)
        k["first_us"] = round(k["first_us"], 3)
        del k["middle_share_us"]

    copy_bytes = 512 << 20
    copy_us = ctx.copy_bandwidth(copy_bytes, reps=10)
    copy_gbs = 2 * copy_bytes / (copy_us * 1e-6) / 1e9
    line = {
        "metric": "site-MD-steps/s",
        "value": value,
        "unit": "site-MD-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1000.0 * dt / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "single large chains: 2D 1024^2 at beta_c=0.4406868 (C=4.1) and 3D 128^3 at "
                        "beta=0.2216544 (C=6.1), J=1, h=0, 20 leap-frog steps per unit trajectory, FP32 "
                        "state, FP64 H/dH/Metropolis; one step = one trajectory of both chains",
            "sites": sum(int(math.prod(w["L"])) for w in ws),
            "md_steps_per_trajectory": ws[0]["n_md"],
        },
        "roofline": {
            "bound": "hbm",
            "kernel": f"fused middle pass, {dom['ndim']}D",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "bytes_per_launch": bytes_per_launch,
            "avg_launch_us": round(dom["middle_us"], 3),
            "copy_kernel_GBs": round(copy_gbs, 1),
            "frac_of_copy": round(achieved / copy_gbs, 4),
        },
        "kernels": kern,
        "chains": per,
    }
    chains.close()
    ctx.close()
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a one-trajectory sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(ws)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
