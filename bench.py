#!/usr/bin/env python3
"""Throughput benchmark of the fused lattice HMC path on one MI355X.

Default workload (the headline): 4096 independent 2D tori of uneven size, beta,
per-site field and step count (L log-uniform in [16, 256], beta ~ U[0.30, 0.55],
h_x ~ N(0, 0.05^2), n_md ~ U{8..32}, C = 4.1, 200 trajectories each), FP32 state
with FP64 Hamiltonian reductions, advanced together.  One step = one trajectory
of every chain; the metric is site-MD-steps/s = (sites x MD steps) per second
over the timed steps.  Beside it the line carries

  * the roofline of the dominant launch kind (HIP-event timed on the library's
    stream): the algorithmic fraction (20 + 8/n_md bytes per site-MD-step times
    the site-MD-steps one launch advances) and the physical one (20 bytes per
    site and launch);
  * the plain form: a sample of the same chains run one at a time, its rate and
    whether every result is bitwise equal to the batched run;
  * the FP64 CPU oracle on a 64-chain sample of the workload (5 trajectories
    each), run over the host cores in parallel processes, median of 5 runs;
  * extra keys: the single large chains (2D 1024^2 at beta_c and 3D 128^3), an
    8192^2 streaming point, the psi/phi form A/B, HMC against Metropolis-Hastings,
    the dense all-to-all workload (N = 4096, 256 chains, MFMA roofline) and 60 s
    of Poisson serving with p50/p99 latency.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload ...]
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
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 MFMA
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 matrix
BYTES_MIDDLE_F32 = 16  # read psi, read p, write p, write psi' (FP32), h = 0


# HBM traffic per launch of each workload's roofline kernel, from two rocprofv3
# --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch, median over the full
# launches), scaled by what the same counters read for the plain copy kernel of
# known size: FETCH_SIZE x 2, WRITE_SIZE x 1.  Each entry records a digest of the
# kernel sources it was measured on and the tile shape and sites of the launch;
# when any of them differs, the field is null (the batched entries instead scale
# with the launch's sites: which chains form the group varies with the tuner).
KERNEL_SOURCES = ("lattice_kernels.hip", "lattice_kernels.hpp", "chain_epilogue.hpp", "device_common.hpp",
                  "ihmc_internal.hpp", "dense_kernels.hip", "dense_kernels.hpp")
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0
TRAFFIC = {
    "large_2d_middle": {"sources": "b2a10c053ede82e0", "tiles": "64x16", "sites": 1048576,
                        "fetch_kib": 4207.0, "write_kib": 8192.0},
    "large_2d_pair": {"sources": "b2a10c053ede82e0", "tiles": "64x16", "sites": 1048576,
                      "fetch_kib": 4353.5, "write_kib": 8192.0},
    "large_3d_middle": {"sources": "b2a10c053ede82e0", "tiles": "32x8x8", "sites": 2097152,
                        "fetch_kib": 9279.0, "write_kib": 16384.0},
    "stream_2d_middle": {"sources": "b2a10c053ede82e0", "tiles": "64x16", "sites": 67108864,
                         "fetch_kib": 263729.3, "write_kib": 524288.0},
    "stream_2d_pair": {"sources": "b2a10c053ede82e0", "tiles": "64x16", "sites": 67108864,
                       "fetch_kib": 264983.6, "write_kib": 524288.0},
    # the tuner's choices set which chains form the group, so a launch of the
    # default run may hold a few more or fewer sites: per-site scaling
    "batched_middle": {"sources": "b2a10c053ede82e0", "tiles": "64x16", "sites": 28718719, "scale_by_sites": True,
                       "fetch_kib": 170626.8, "write_kib": 226601.3},
    "batched_pair": {"sources": "b2a10c053ede82e0", "tiles": "64x16", "sites": 28718719, "scale_by_sites": True,
                     "fetch_kib": 170776.5, "write_kib": 227465.4},
    "dense_gemm_bf16": {"sources": "b2a10c053ede82e0", "fetch_kib": 73752.0, "write_kib": 16384.0},
}


def kernel_digest():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1912_03278_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_bytes(key, sites=None, tiles=None):
    """Measured HBM bytes per launch of the roofline kernel, or None if the
    kernel sources, or the tile shape or sites of the launch, differ from those
    the counters were taken on."""
    t = TRAFFIC.get(key)
    if not t or t["sources"] != kernel_digest():
        return None
    if tiles is not None and t.get("tiles") not in (None, tiles):
        return None
    b = 1024 * (FETCH_SCALE * t["fetch_kib"] + WRITE_SCALE * t["write_kib"])
    if sites is not None and t.get("sites") not in (None, sites):
        if not t.get("scale_by_sites"):
            return None
        b *= sites / t["sites"]
    return int(b)


def large_workload():
    from paper_1912_03278_amd import inputs
    return inputs.large()


def tune_tiles(ctx, lats, args, sites=0):
    """Autotune the tile class of every distinct lattice shape (unless --tiles rule)
    at the workload's resident working set; returns a summary for the JSON line."""
    if args.tiles == "rule":
        return {"tile_classes": "built-in rule"}
    t0 = time.perf_counter()
    n = ctx.tune(lats, sites=sites)
    dt = time.perf_counter() - t0
    print(f"bench: tile classes tuned for {n} shapes in {dt:.1f} s", file=sys.stderr, flush=True)
    return {"tile_classes": "autotuned", "tuned_shapes": n, "tune_s": round(dt, 2)}


def group_rows(chains, reps, modes=(1,), pair=False):
    """Per launch group: tile shape, sites and HIP-event time of the pass kinds
    (with pair: also the two-step launch of the groups that have one, as
    pair_us)."""
    from paper_1912_03278_amd import ihmc
    rows = []
    for g in range(chains.groups()):
        info = chains.group_info(g)
        if info["cls"] < 0:  # LDS-resident chains: whole trajectories per launch, no passes to time
            rows.append(dict(ndim=info["ndim"], tiles="resident", chains=info["chains"], sites=info["sites"]))
            continue
        shape = ihmc.tile_shape(info["ndim"], info["cls"])
        row = dict(ndim=info["ndim"], tiles="x".join(map(str, shape if info["ndim"] == 3 else shape[:2])),
                   chains=info["chains"], sites=info["sites"])
        for m in modes:
            name = ("first_us", "middle_us", "last_us")[m]
            row[name] = chains.time_pass(g, mode=m, reps=reps if m == 1 else max(10, reps // 5))["us"]
        if pair:
            try:  # groups without two-step launches refuse the mode
                row["pair_us"] = chains.time_pass(g, mode=ihmc.PAIR, reps=reps)["us"]
            except ihmc.IhmcError:
                pass
        rows.append(row)
    return rows


def host_cpu():
    """(cores this process may run on, capped at the box's share of 16; CPU model)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return max(1, min(16, n)), model


def _oracle_warm(_):
    import oracle
    oracle.lib()
    return os.getpid()


def _oracle_job(job):
    """One oracle chain of `job` (a dict of its parameters); returns its CPU seconds."""
    import oracle
    lat = oracle.Lattice(tuple(job["L"]), beta=job["beta"], C=job["C"], h=job["h"])
    t0 = time.perf_counter()
    oracle.run(lat, job["n_traj"], job["n_md"], seed=job["seed"], chain_id=job["chain_id"])
    return time.perf_counter() - t0


def oracle_parallel(jobs, reps=5, what=""):
    """The FP64 oracle, unchanged, on `jobs` (independent chains) over the host
    cores: one process per core, chains dealt largest first; one warm-up pass
    loads the oracle in every process, then `reps` timed passes over all jobs,
    the median wall time kept.  Returns the cpu_baseline record."""
    import multiprocessing as mp
    import statistics

    import oracle
    oracle.lib()  # built once here, before the workers load it
    cores, model = host_cpu()
    work = sum(int(math.prod(j["L"])) * j["n_md"] * j["n_traj"] for j in jobs)
    order = sorted(jobs, key=lambda j: -int(math.prod(j["L"])) * j["n_md"] * j["n_traj"])
    walls, cpu_s = [], 0.0
    with mp.get_context("spawn").Pool(cores) as pool:
        pool.map(_oracle_warm, range(cores))
        for _ in range(reps):
            t0 = time.perf_counter()
            cpu_s = sum(pool.map(_oracle_job, order, chunksize=1))
            walls.append(time.perf_counter() - t0)
    wall = statistics.median(walls)
    return dict(value=work / wall, unit="site-MD-steps/s", cores=cores, kind="oracle",
                sample=f"{what}: {len(jobs)} chains, {work:.3g} site-MD-steps, FP64, each chain's set-up (field "
                       f"constants by CG) included, in {cores} processes; "
                       f"median wall time of {reps} runs {wall:.2f} s ({cpu_s:.1f} CPU-s per run)",
                cpu_model=model, runs_wall_s=[round(w, 3) for w in walls])


def streaming_point(args, copy_gbs):
    """Labelled extra point: one 2D 8192^2 chain (about 1 GiB of state, far beyond
    the 256 MB Infinity Cache), beta_c, h = 0, n_md = 20, FP32: the fused middle
    pass against the HBM peak on a single chain."""
    import torch
    from paper_1912_03278_amd import ihmc, inputs
    L = 8192
    ctx = ihmc.Context(device=0, arena_bytes=3 << 30, resident=args.resident_sites, fuse_steps=args.fuse_steps)
    lat = ihmc.Lattice((L, L), beta=inputs.BETA_C_2D, C=4.1)
    ch = ihmc.Chains(ctx, [lat], [ihmc.Run(n_md=20, n_traj=8, precision=ihmc.F32, seed=2, chain_id=2)])
    ch.advance(1)
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ch.advance(4)
    ctx.sync()
    dt = time.perf_counter() - t0
    acc = ch.result(0, want_psi=False)["acceptance"]
    mid = ch.time_pass(0, mode=1, reps=max(5, args.timing_reps // 5))
    pair = ch.time_pass(0, mode=ihmc.PAIR, reps=max(5, args.timing_reps // 5)) if args.fuse_steps else None
    ch.close()
    ctx.close()
    gbs = BYTES_MIDDLE_F32 * mid["sites"] / (mid["us"] * 1e-6) / 1e9
    print(f"bench: streaming point 8192^2 middle pass {mid['us']:.1f} us = {gbs:.0f} GB/s", file=sys.stderr,
          flush=True)
    extra = {}
    if pair:
        pgbs = BYTES_MIDDLE_F32 * pair["sites"] / (pair["us"] * 1e-6) / 1e9
        extra = {"two_step_pass_us": round(pair["us"], 2), "two_step_achieved_GBs": round(pgbs, 1),
                 "two_step_traffic": traffic_bytes("stream_2d_pair", sites=pair["sites"])}
    return {"label": "extra point, not the configured workload: one 2D 8192^2 chain at beta_c, FP32, n_md=20",
            "site_md_steps_per_s": 4 * L * L * 20 / dt, "acceptance": acc,
            "middle_pass_us": round(mid["us"], 2), "bytes_per_launch": BYTES_MIDDLE_F32 * mid["sites"],
            "traffic": traffic_bytes("stream_2d_middle", sites=mid["sites"]),
            "achieved_GBs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
            "frac_of_copy": round(gbs / copy_gbs, 4), **extra}


def bench_small(args):
    """One 2D 8x8 chain in FP64 (beta = 0.40, C = 4.1, n_md = 10, h = 0): the
    correctness configuration.  With 64 sites every pass is pure launch latency;
    the CPU oracle on the same chain is reported beside it."""
    import numpy as np
    import torch
    from paper_1912_03278_amd import ihmc, inputs
    w = inputs.small()
    K, W = args.steps, args.warmup
    ctx = ihmc.Context(device=0, arena_bytes=64 << 20, resident=args.resident_sites, fuse_steps=args.fuse_steps)
    lat = ihmc.Lattice(w["L"], beta=w["beta"], C=w["C"])
    ch = ihmc.Chains(ctx, [lat], [ihmc.Run(n_md=w["n_md"], n_traj=W + K, precision=ihmc.F64, seed=w["seed"])])
    ch.advance(W)
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ch.advance(K)
    ctx.sync()
    dt = time.perf_counter() - t0
    r = ch.result(0, want_psi=False)
    ch.close()
    ctx.close()
    N = int(math.prod(w["L"]))
    line = {
        "metric": "site-MD-steps/s", "value": K * N * w["n_md"] / dt, "unit": "site-MD-steps/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": 1000.0 * dt / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "small: one 2D 8x8 chain, beta=0.40, C=4.1, h=0, n_md=10, FP64 state; one step = "
                               "one trajectory (latency-bound by construction)", "sites": N,
                   "resident": args.resident, "fuse_steps": args.fuse},
        "observables": {"beta_eps_mean": float(np.mean(r["beta_eps"][W:])), "m2c_mean": float(np.mean(r["m2c"][W:])),
                        "acceptance": r["acceptance"],
                        "exact_beta_eps": -0.4889282573, "exact_m2": 0.4320990786},
        "roofline": None,
    }
    if not args.no_cpu_baseline:
        import oracle
        t1 = time.perf_counter()
        oracle.run(oracle.Lattice(w["L"], beta=w["beta"], C=w["C"]), W + K, w["n_md"], seed=w["seed"])
        t_cpu = time.perf_counter() - t1
        line["cpu_baseline"] = dict(value=(W + K) * N * w["n_md"] / t_cpu, unit="site-MD-steps/s", cores=1,
                                    kind="oracle", sample=f"the same chain, {W + K} trajectories, FP64, "
                                                          f"{t_cpu:.2f} s on one host core")
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


METRIC = "site-MD-steps/s & %HBM roofline, batched vs plain; p50/p99 request latency"


def run_batched(args):
    """4096 independent 2D tori of uneven size, beta, per-site field and step count,
    advanced together (one step = one trajectory of every chain), against the same
    chains run one at a time (the plain form) on a sample.  Returns the JSON line."""
    import numpy as np
    import torch
    from paper_1912_03278_amd import ihmc, inputs

    ws = inputs.batched(n_chains=args.chains)
    K, W = args.steps, args.warmup
    ctx = ihmc.Context(device=0, arena_bytes=6 << 30, resident=args.resident_sites, fuse_steps=args.fuse_steps)
    lats = [ihmc.Lattice(w["L"], beta=w["beta"], C=w["C"], h=w["h"]) for w in ws]
    runs = [ihmc.Run(n_md=w["n_md"], n_traj=W + K, precision=ihmc.F32, seed=w["seed"], chain_id=w["chain_id"])
            for w in ws]
    tiles = tune_tiles(ctx, lats, args)
    t0 = time.perf_counter()
    chains = ihmc.Chains(ctx, lats, runs)
    t_setup = time.perf_counter() - t0
    print(f"bench: {len(ws)} chains ready in {t_setup:.1f} s", file=sys.stderr, flush=True)
    chains.advance(W)
    ctx.sync()
    torch.cuda.synchronize()
    print(f"bench: warmup {W} rounds done", file=sys.stderr, flush=True)
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
        a = alone.result(0)
        b = chains.result(i)
        same = all(np.array_equal(a[k], b[k]) for k in ("dH", "H_old", "H_new", "m", "beta_eps", "accepted",
                                                         "psi_final"))
        if not same:
            mismatch.append(i)
        identical &= same
        alone.close()
    if sample:
        print(f"bench: plain form on {len(sample)} chains, bitwise equal: {identical}", file=sys.stderr, flush=True)
    acc = [chains.result(i, want_psi=False)["acceptance"] for i in range(0, len(ws), max(1, len(ws) // 64))]

    # launch groups (all chains FP32 2D): HIP-event times of the one-step and
    # two-step launches; a launch moves 20 B per site (psi, p and the field
    # read, p and psi written) for one or two MD steps
    kern = group_rows(chains, args.timing_reps, pair=args.fuse_steps)
    for k in kern:
        for name in ("middle", "pair"):
            if f"{name}_us" in k:
                k[f"{name}_physical_GBs"] = round(20 * k["sites"] / (k[f"{name}_us"] * 1e-6) / 1e9, 1)
                k[f"{name}_us"] = round(k[f"{name}_us"], 2)
    key = "pair_us" if args.fuse_steps else "middle_us"
    gi, dom = max(((g, k) for g, k in enumerate(kern) if key in k), key=lambda t: t[1]["sites"])
    steps_per_launch = 2 if args.fuse_steps else 1
    # algorithmic bytes of one launch: (20 + 8/n_md) B per site-MD-step, per
    # chain of the group, times the site-MD-steps the launch advances
    dom_chains = [ws[i] for i in chains.group_chains(gi)]
    alg_bytes = steps_per_launch * sum(int(math.prod(w["L"])) * (20.0 + 8.0 / w["n_md"]) for w in dom_chains)
    phys_bytes = 20 * dom["sites"]
    achieved = alg_bytes / (dom[key] * 1e-6) / 1e9
    achieved_phys = phys_bytes / (dom[key] * 1e-6) / 1e9
    copy_bytes = 512 << 20
    copy_gbs = 2 * copy_bytes / (ctx.copy_bandwidth(copy_bytes, reps=10) * 1e-6) / 1e9
    cls_traffic = traffic_bytes("batched_pair" if args.fuse_steps else "batched_middle", sites=dom["sites"],
                                tiles=dom["tiles"])
    line = {
        "metric": METRIC, "value": value, "unit": "site-MD-steps/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": 1000.0 * dt / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched: {len(ws)} independent 2D tori, L log-uniform [16,256], beta U[0.30,0.55], "
                               "h_x ~ N(0,0.05^2) per site, n_md U{8..32}, C=4.1, FP32 state, FP64 H/dH/Metropolis; "
                               "one step = one trajectory of every chain",
                   "chains": len(ws), "sites": sum(int(math.prod(w["L"])) for w in ws),
                   "execution_form": "one HIP graph per round (per-pass launches of every tile-class group on "
                                     "streams of their own; chains of at most 5024 sites as LDS-resident whole-"
                                     "trajectory launches beside them), replayed per round; not a single persistent "
                                     "kernel with a device work queue",
                   **tiles, "resident": args.resident, "fuse_steps": args.fuse},
        "roofline": {"bound": "hbm", "kernel": ("two-step " if args.fuse_steps else "") +
                                               f"fused middle pass, 2D, per-site field, {dom['tiles']}-tile group "
                                               f"({dom['chains']} chains, {dom['sites']} sites)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": cls_traffic,
                     "traffic_basis": None if cls_traffic is None else
                     "FETCH_SIZE x 2 + WRITE_SIZE x 1 (copy-kernel calibration) of the full-group launch, "
                     "per site of the profiled launch times this launch's sites",
                     "algorithmic_bytes_per_launch": int(alg_bytes),
                     "algorithmic_basis": f"(20 + 8/n_md) B per site-MD-step x {steps_per_launch} MD step(s) per "
                                          "site and launch, summed over the group's chains",
                     "physical_bytes_per_launch": phys_bytes, "achieved_physical": round(achieved_phys, 1),
                     "frac_physical": round(achieved_phys / HBM_PEAK_GBS, 4),
                     "avg_launch_us": dom[key], "timing": "HIP events on the library stream, launches back to back",
                     "copy_kernel_GBs": round(copy_gbs, 1), "frac_physical_of_copy": round(achieved_phys / copy_gbs, 4)},
        "kernels": kern,
        "plain": {"chains": len(sample), "value": (plain_work / plain_time) if plain_time > 0 else None,
                  "unit": "site-MD-steps/s", "batched_over_plain": (value / (plain_work / plain_time))
                  if plain_time > 0 else None,
                  "bitwise_equal_to_batched": identical if sample else None, "mismatched_chains": mismatch},
        "acceptance_sample_mean": float(np.mean(acc)),
        "setup_s": round(t_setup, 2),
    }
    chains.close()
    ctx.close()
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a 64-chain sample", file=sys.stderr, flush=True)
        pick = sorted(np.random.default_rng(1).choice(len(ws), size=min(64, len(ws)), replace=False).tolist())
        jobs = [dict(L=ws[i]["L"], beta=ws[i]["beta"], C=ws[i]["C"], h=ws[i]["h"], n_md=ws[i]["n_md"], n_traj=5,
                     seed=ws[i]["seed"], chain_id=ws[i]["chain_id"]) for i in pick]
        line["cpu_baseline"] = oracle_parallel(jobs, what="batched workload, 64 sampled chains x 5 trajectories")
    else:
        line["cpu_baseline"] = None
    return line


def bench_batched(args):
    print(json.dumps(run_batched(args)), flush=True)


_DENSE_MODEL = {}


def _oracle_dense_job(job):
    """One oracle chain of the dense workload's model (built once per process
    from the same seeded generator); returns its CPU seconds."""
    import oracle
    from paper_1912_03278_amd import inputs
    if "w" not in _DENSE_MODEL:
        _DENSE_MODEL["w"] = inputs.dense()
    w = _DENSE_MODEL["w"]
    t0 = time.perf_counter()
    oracle.run(oracle.Dense(w["K"], beta=w["beta"], C=job["C"]), job["n_traj"], w["n_md"], seed=w["seed"],
               chain_id=job["chain_id"])
    return time.perf_counter() - t0


def _oracle_dense_warm(_):
    from paper_1912_03278_amd import inputs
    import oracle
    oracle.lib()
    if "w" not in _DENSE_MODEL:
        _DENSE_MODEL["w"] = inputs.dense()
    return os.getpid()


def oracle_dense_parallel(C, n_md, N, reps=3, n_traj=1):
    """The FP64 oracle on one trajectory of each of `cores` chains of the dense
    model, one process per core; median wall time of `reps` passes."""
    import multiprocessing as mp
    import statistics

    import oracle
    oracle.lib()
    cores, model = host_cpu()
    jobs = [dict(C=C, n_traj=n_traj, chain_id=i) for i in range(cores)]
    work = len(jobs) * n_traj * N * n_md
    walls, cpu_s = [], 0.0
    with mp.get_context("spawn").Pool(cores) as pool:
        pool.map(_oracle_dense_warm, range(cores))
        for _ in range(reps):
            t0 = time.perf_counter()
            cpu_s = sum(pool.map(_oracle_dense_job, jobs, chunksize=1))
            walls.append(time.perf_counter() - t0)
    wall = statistics.median(walls)
    return dict(value=work / wall, unit="site-MD-steps/s", cores=cores, kind="oracle",
                sample=f"dense workload, {len(jobs)} chains x {n_traj} trajectory of the N={N} model: "
                       f"{work:.3g} site-MD-steps, FP64, each chain's set-up (CG constants) included, in {cores} "
                       f"processes; median wall time of {reps} runs {wall:.2f} s ({cpu_s:.1f} CPU-s per run)",
                cpu_model=model, runs_wall_s=[round(x, 3) for x in walls])


def bench_dense(args):
    print(json.dumps(run_dense(args)), flush=True)


def run_dense(args):
    """256 chains of one dense all-to-all model (N = 4096, K_ij ~ N(0, 1/N), h = 0,
    beta = 1, C from Lanczos), 16 leap-frog steps per trajectory; one step = one
    trajectory of every chain.  Both K~ applications of a force evaluation are
    4096 x 4096 by 4096 x 256 GEMMs on the MFMA units (six BF16 limb products)."""
    import numpy as np
    import torch
    from paper_1912_03278_amd import ihmc, inputs

    w = inputs.dense()
    K, W = args.steps, args.warmup
    N, B, n_md = w["K"].shape[0], w["n_chains"], w["n_md"]
    ctx = ihmc.Context(device=0, arena_bytes=2 << 30, resident=args.resident_sites, fuse_steps=args.fuse_steps)
    runs = [ihmc.Run(n_md=n_md, n_traj=W + K, precision=ihmc.F32, seed=w["seed"], chain_id=i) for i in range(B)]
    t0 = time.perf_counter()
    chains = ihmc.DenseChains(ctx, ihmc.Dense(w["K"], beta=w["beta"]), runs, products=args.products)
    t_setup = time.perf_counter() - t0
    info = chains.info()
    print(f"bench: dense chains ready in {t_setup:.2f} s (C = {info['C']:.6f}, Lanczos {info['lanczos_steps']} "
          f"steps, CG {info['cg_iters']} steps)", file=sys.stderr, flush=True)
    chains.advance(W)
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chains.advance(K)
    ctx.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = K * N * B * n_md / dt
    print(f"bench: timed {K} trajectories of {B} chains in {dt:.3f} s", file=sys.stderr, flush=True)
    res = [chains.result(i, want_psi=False) for i in range(B)]
    acc = float(np.mean([r["acceptance"] for r in res]))
    be = float(np.mean([r["beta_eps"][-1] for r in res]))

    g = chains.time(0, reps=args.timing_reps)
    f64 = chains.time(1, reps=max(5, args.timing_reps // 4))
    force = chains.time(2, reps=max(5, args.timing_reps // 4))
    m, n, k = g["m"], g["n"], g["k"]
    executed = args.products * 2.0 * m * n * k  # BF16 MFMA flops one launch executes (padded shape)
    useful = 2.0 * N * N * B  # one K~ application of every chain, FP32-equivalent
    achieved = executed / (g["us"] * 1e-6) / 1e12
    line = {
        "metric": "site-MD-steps/s", "value": value, "unit": "site-MD-steps/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": 1000.0 * dt / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16x%d->f32 (FP32 state, FP64 H)" % args.products, "data": "synthetic",
        "config": {"workload": f"dense all-to-all: N={N}, K_ij ~ N(0,1/N) symmetric, zero diagonal, h=0, beta=1, "
                               f"C=|lambda_min|+0.1 by FP64 Lanczos, {B} chains, {n_md} leap-frog steps per "
                               "trajectory; one step = one trajectory of every chain",
                   "sites": N, "chains": B, "md_steps_per_trajectory": n_md, "limb_products": args.products,
                   "C": info["C"]},
        "roofline": {"bound": "mfma", "kernel": "BF16-limb split-K GEMM (one K~ application of all chains)",
                     "achieved": round(achieved, 1), "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / BF16_PEAK_TFLOPS, 4), "traffic": traffic_bytes("dense_gemm_bf16"),
                     "flops_per_launch": executed, "avg_launch_us": round(g["us"], 2),
                     "gemm_mnk": [m, n, k], "split_k": g["split_k"],
                     "useful_fp32_equiv_TFLOPs": round(useful / (g["us"] * 1e-6) / 1e12, 1)},
        "kernels": {"gemm_bf16_us": round(g["us"], 2), "gemm_f64_us": round(f64["us"], 2),
                    "gemm_f64_TFLOPs": round(2.0 * m * B * k / (f64["us"] * 1e-6) / 1e12, 1),
                    "gemm_f64_frac": round(2.0 * m * B * k / (f64["us"] * 1e-6) / 1e12 / FP64_PEAK_TFLOPS, 4),
                    "force_evaluation_us": round(force["us"], 2)},
        "acceptance_mean": acc, "beta_eps_last_mean": be, "setup_s": round(t_setup, 2),
        "lanczos": {"theta": info["theta"], "resid": info["resid"], "steps": info["lanczos_steps"]},
    }
    chains.close()
    ctx.close()
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a sample of the dense chains", file=sys.stderr, flush=True)
        line["cpu_baseline"] = oracle_dense_parallel(info["C"], n_md, N)
    else:
        line["cpu_baseline"] = None
    return line


def run_serving(args):
    """Open-loop Poisson arrivals of lattice requests (2D or 3D, uneven size,
    beta, field and length) into the continuous-batching server; returns the
    completed site-MD-steps/s and the request latency percentiles.  A request
    still unfinished at the deadline counts in the percentiles with an unbounded
    latency (a percentile that falls on one is reported as null)."""
    import threading

    import numpy as np
    from paper_1912_03278_amd import ihmc, inputs

    reqs = inputs.serving(rate=args.rate, duration=args.serve_duration)
    ctx = ihmc.Context(device=0, arena_bytes=12 << 30, resident=args.resident_sites, fuse_steps=args.fuse_steps)
    # tile classes of every request shape, chosen before the first arrival
    shapes = {}
    for r in reqs:
        shapes.setdefault((tuple(r["L"]), r["h"] is not None and np.size(r["h"]) > 1),
                          ihmc.Lattice(r["L"], beta=r["beta"], C=r["C"], h=r["h"]))
    # the working set they are tuned for: the resident set at this load, about a
    # thousand requests of ~47k sites on average
    tiles = tune_tiles(ctx, list(shapes.values()), args, sites=1 << 25)
    sv = ihmc.Server(ctx, budget_bytes=10 << 30, max_active=2048)
    tickets = [None] * len(reqs)
    work = [int(math.prod(r["L"])) * r["n_md"] * r["n_traj"] for r in reqs]
    t_start = time.perf_counter()

    def submitter():
        for k, r in enumerate(reqs):
            delay = t_start + r["t"] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            lat = ihmc.Lattice(r["L"], beta=r["beta"], C=r["C"], h=r["h"])
            tickets[k] = sv.submit(lat, ihmc.Run(n_md=r["n_md"], n_traj=r["n_traj"], precision=ihmc.F32,
                                                 seed=r["seed"], chain_id=r["chain_id"]))

    th = threading.Thread(target=submitter)
    th.start()
    done, lat_s, next_report = {}, [], time.perf_counter() + 10
    deadline = t_start + args.serve_duration + args.drain
    while len(done) < len(reqs) and time.perf_counter() < deadline:
        for k, t in enumerate(tickets):
            if t is None or k in done:
                continue
            if sv.poll(t) >= ihmc.REQ_DONE:
                r = sv.fetch(t, want_psi=False)
                done[k] = r
                lat_s.append(r["t_done"] - r["t_submit"])
        if time.perf_counter() > next_report:
            st = sv.stats()
            print(f"bench: serving t={time.perf_counter() - t_start:.0f}s done {len(done)}/{len(reqs)} "
                  f"resident {st['resident']:.0f} queued {st['queued']:.0f}", file=sys.stderr, flush=True)
            next_report += 10
        time.sleep(0.002)
    th.join()
    t_end = time.perf_counter()
    st = sv.stats()
    incomplete = [k for k in range(len(reqs)) if k not in done]
    sv.close()
    ctx.close()
    completed_work = sum(work[k] for k in done)
    elapsed = t_end - t_start
    # every request counts: unfinished ones with an unbounded latency
    lat = np.array(lat_s + [math.inf] * len(incomplete)) if reqs else np.array([math.nan])

    def pct(q):
        v = float(np.percentile(lat, q, method="higher"))
        return v if math.isfinite(v) else None

    out = {
        "workload": f"serving: Poisson arrivals {args.rate:g}/s for {args.serve_duration:g} s; 2D or 3D (p = 1/2), "
                    "L U{16..128} (2D) / U{16..64} (3D), beta U[0.2,0.6], uniform h U[0,0.1], C = 2d + 0.1, "
                    "50-1000 trajectories of 10-30 leap-frog steps, FP32 state, FP64 H",
        "value": completed_work / elapsed, "unit": "site-MD-steps/s",
        "latency_s": {"p50": pct(50), "p99": pct(99), "mean_completed": float(np.mean(lat_s)) if lat_s else None,
                      "max_completed": float(np.max(lat_s)) if lat_s else None},
        "requests": len(reqs), "completed": len(done), "incomplete": len(incomplete), "elapsed_s": elapsed,
        "offered_site_md_steps_per_s": sum(work) / args.serve_duration,
        "server": {"rounds": st["rounds"], "busy_s": st["busy_s"], "max_resident": st["max_resident"],
                   "site_md_steps_in_rounds": st["site_md_steps"],
                   "rate_while_busy": st["site_md_steps"] / st["busy_s"] if st["busy_s"] > 0 else None},
        "resident": args.resident, "fuse_steps": args.fuse, **tiles,
    }
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a sample of the served requests", file=sys.stderr, flush=True)
        rng = np.random.default_rng(2)
        pick = sorted(rng.choice(len(reqs), size=min(64, len(reqs)), replace=False).tolist())
        jobs = [dict(L=reqs[i]["L"], beta=reqs[i]["beta"], C=reqs[i]["C"], h=reqs[i]["h"], n_md=reqs[i]["n_md"],
                     n_traj=3, seed=reqs[i]["seed"], chain_id=reqs[i]["chain_id"]) for i in pick]
        cb = oracle_parallel(jobs, reps=3, what="served requests, 64 sampled requests x 3 trajectories")
        # CPU time a whole request would take on one core, from the sample's rate
        mean_req = float(np.mean([work[i] for i in pick]))
        cb["one_core_s_per_request_mean"] = round(mean_req / (cb["value"] / cb["cores"]), 2)
        out["cpu_baseline"] = cb
    else:
        out["cpu_baseline"] = None
    return out


def bench_serving(args):
    s = run_serving(args)
    line = {"metric": METRIC, "value": s["value"], "unit": "site-MD-steps/s", "n_gpus": 1,
            "steps": s["completed"], "warmup": 0, "ms_per_step": 1000.0 * s["elapsed_s"] / max(1, s["completed"]),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": s["workload"] + "; one step = one completed request"},
            "latency_s": s["latency_s"], "serving": s, "roofline": None, "cpu_baseline": s["cpu_baseline"]}
    print(json.dumps(line), flush=True)


def run_phi_ab(args, K=20, W=2):
    """The paper's substitution measured (Sec. 2): the same chains run in the
    inverse formulation (eq. cosh_in_exponent, a CG solve of Kt per force
    evaluation) and in the substituted psi form (eq. phi_psi_substitution), both
    FP64 and LDS-resident, one workgroup per chain: 512 2D 32^2 tori at beta_c
    (C = 4.1) and 512 3D 11^3 tori at beta = 0.2216544 (C = 6.1), h = 0,
    n_md = 10.  Returns site-MD-steps/s of each form and their ratio, CG
    iterations per force evaluation, acceptance, and <beta*eps> over the timed
    trajectories (from the same start; far too few to thermalise at these
    couplings, so the two forms' values are not comparable)."""
    import numpy as np
    import torch
    from paper_1912_03278_amd import ihmc, inputs

    pts = [((32, 32), inputs.BETA_C_2D, 4.1), ((11, 11, 11), inputs.BETA_3D, 6.1)]
    R = args.phi_chains
    lats, specs = [], []
    for L, beta, C in pts:
        for r in range(R):
            lats.append(ihmc.Lattice(L, beta=beta, C=C))
            specs.append((L, beta, C))
    n_md = 10
    out = {"workload": f"{R} 2D 32^2 tori at beta_c (C=4.1) and {R} 3D 11^3 tori at beta=0.2216544 (C=6.1), "
                       f"h=0, n_md={n_md}, FP64 state, LDS-resident (one workgroup per chain); one step = one "
                       "trajectory of every chain", "steps": K, "warmup": W}
    work = sum(int(math.prod(L)) * n_md for L, _, _ in specs)
    for name, form in (("psi", ihmc.FORM_PSI), ("phi", ihmc.FORM_PHI)):
        ctx = ihmc.Context(device=0, arena_bytes=1 << 30)
        runs = [ihmc.Run(n_md=n_md, n_traj=W + K, precision=ihmc.F64, seed=21, chain_id=i, form=form)
                for i in range(len(lats))]
        ch = ihmc.Chains(ctx, lats, runs)
        ch.advance(W)
        ctx.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch.advance(K)
        ctx.sync()
        dt = time.perf_counter() - t0
        res = [ch.result(i, want_psi=False) for i in range(len(lats))]
        ch.close()
        ctx.close()
        be = {}
        for k, (L, _, _) in enumerate(pts):
            vals = np.array([r["beta_eps"][W:] for r in res[k * R:(k + 1) * R]])
            be["x".join(map(str, L))] = [float(vals.mean()), float(vals.mean(axis=1).std() / math.sqrt(R))]
        row = {"value": K * work / dt, "unit": "site-MD-steps/s", "ms_per_step": 1000.0 * dt / K,
               "acceptance": float(np.mean([r["acceptance"] for r in res])),
               "beta_eps_mean_err_unthermalised": be}
        if form == ihmc.FORM_PHI:
            cg = sum(r["cg_iterations"] for r in res)
            row["cg_iterations_per_force"] = cg / (len(res) * (W + K) * (n_md + 1))
        out[name] = row
        print(f"bench: {name} form {row['value']:.3g} site-MD-steps/s", file=sys.stderr, flush=True)
    out["psi_over_phi"] = out["psi"]["value"] / out["phi"]["value"]
    return out


def bench_phi(args):
    ab = run_phi_ab(args, K=args.steps, W=args.warmup)
    line = {"metric": "site-MD-steps/s", "value": ab["psi"]["value"], "unit": "site-MD-steps/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ab["psi"]["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "phi/psi A/B: " + ab["workload"]}, "phi_form_ab": ab, "roofline": None,
            "cpu_baseline": None}
    print(json.dumps(line), flush=True)


def run_mh_compare(args, sweeps=None):
    """Sec. 4's cost comparison on this GPU: one HMC trajectory against one
    Metropolis-Hastings sweep (checkerboard, N spin proposals) of the same
    single chain, per N_step = floor(ln N) leap-frog steps (the paper finds
    T_HMC ~ 4 N_step T_MH on its CPU code).  Single chains at the critical
    couplings, h = 0: 2D L = 64 .. 2048 at beta_c, 3D L = 16 .. 128 at
    beta = 0.2216544; HMC FP32 state on the tiled passes (no LDS-resident
    path), graph-replayed trajectories; MH int8 spins, graph-replayed sweeps
    timed with HIP events."""
    import torch
    from paper_1912_03278_amd import ihmc, inputs

    pts = [((L, L), inputs.BETA_C_2D, 4.1) for L in (64, 256, 1024, 2048)] + \
          [((L,) * 3, inputs.BETA_3D, 6.1) for L in (16, 32, 64, 128)]
    rows = []
    ctx = ihmc.Context(device=0, arena_bytes=2 << 30, resident=0, fuse_steps=args.fuse_steps)
    for L, beta, C in pts:
        N = int(math.prod(L))
        n_step = int(math.floor(math.log(N)))
        lat = ihmc.Lattice(L, beta=beta, C=C)
        n_sw = sweeps or max(20, min(400, int(4e8 // N)))
        ctx.mh_run(lat, 5, seed=1)  # warm-up (module load, graph)
        mh = ctx.mh_run(lat, n_sw, seed=1)
        t_mh = mh["seconds"] / n_sw
        K = max(10, min(200, int(4e7 // (N * n_step))))
        ch = ihmc.Chains(ctx, [lat], [ihmc.Run(n_md=n_step, n_traj=K + 3, precision=ihmc.F32, seed=1)])
        ch.advance(3)
        ctx.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch.advance(K)
        ctx.sync()
        t_hmc = (time.perf_counter() - t0) / K
        acc = ch.result(0, want_psi=False)["acceptance"]
        ch.close()
        rows.append({"lattice": "x".join(map(str, L)), "N": N, "n_step": n_step, "T_MH_us": round(1e6 * t_mh, 2),
                     "T_HMC_us": round(1e6 * t_hmc, 2), "T_HMC_over_Nstep_T_MH": round(t_hmc / (n_step * t_mh), 3),
                     "mh_acceptance": round(mh["acceptance"], 4), "hmc_acceptance": round(acc, 4),
                     "mh_spin_flips_per_s": N / t_mh})
        print(f"bench: {rows[-1]['lattice']}: T_HMC {rows[-1]['T_HMC_us']} us, T_MH {rows[-1]['T_MH_us']} us, "
              f"ratio/N_step {rows[-1]['T_HMC_over_Nstep_T_MH']}", file=sys.stderr, flush=True)
    ctx.close()
    return {"workload": "one chain per lattice, h = 0, critical couplings; HMC with N_step = floor(ln N), FP32 "
                        "state; MH checkerboard sweeps of int8 spins", "points": rows,
            "dense": run_mh_compare_dense(args)}


def run_mh_compare_dense(args):
    """The same comparison on the dense workload's all-to-all model (N = 4096,
    K_ij ~ N(0, 1/N), beta = 1, 256 chains): where every site has N - 1
    neighbours (Sec. 5 expects HMC to close the gap there).  HMC: the dense
    chains with N_step = floor(ln N) leap-frog steps (BF16-limb GEMMs over all
    chains); MH: sequential sweeps, one workgroup per chain, local fields
    carried in FP64, delayed updates per 64-site block.  T_MH from the GPU time
    of two launches of different sweep counts (their difference removes the
    set-up of the fields)."""
    import numpy as np
    import torch
    from paper_1912_03278_amd import ihmc, inputs

    w = inputs.dense()
    K, beta, B = w["K"], w["beta"], w["n_chains"]
    N = K.shape[0]
    n_step = int(math.floor(math.log(N)))
    ctx = ihmc.Context(device=0, arena_bytes=2 << 30)
    model = ihmc.Dense(K, beta=beta, C=-1.0)
    ctx.dense_mh_run(model, B, 1, seed=1)  # warm-up
    a = ctx.dense_mh_run(model, B, 2, seed=1)
    b = ctx.dense_mh_run(model, B, 6, seed=1)
    t_mh = (b["seconds"] - a["seconds"]) / 4
    Kt = 20
    ch = ihmc.DenseChains(ctx, model, [ihmc.Run(n_md=n_step, n_traj=Kt + 3, precision=ihmc.F32, seed=w["seed"],
                                                chain_id=i) for i in range(B)], products=args.products)
    ch.advance(3)
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ch.advance(Kt)
    ctx.sync()
    t_hmc = (time.perf_counter() - t0) / Kt
    acc = float(np.mean([ch.result(i, want_psi=False)["acceptance"] for i in range(B)]))
    ch.close()
    ctx.close()
    np_ = 512 * (-(-N // 512))
    # rows of K a sweep reads: one per accepted flip and chain (delayed updates),
    # plus the 64 x 64 diagonal blocks
    acc_mh = float(np.mean(b["acceptance"]))
    k_bytes = (acc_mh * N * np_ + N * 64) * 8.0 * B
    out = {"model": f"dense all-to-all N={N}, K_ij ~ N(0,1/N), beta={beta:g}, h=0, {B} chains", "N": N,
           "chains": B, "n_step": n_step, "T_MH_us": round(1e6 * t_mh, 1), "T_HMC_us": round(1e6 * t_hmc, 1),
           "T_HMC_over_Nstep_T_MH": round(t_hmc / (n_step * t_mh), 3),
           "mh_acceptance": round(acc_mh, 4), "hmc_acceptance": round(acc, 4),
           "mh_spin_flips_per_s": N * B / t_mh,
           "mh_K_row_bytes_per_s": k_bytes / t_mh,
           "mh_bound": "per 64-site block: the block's proposals in sequence on one wave, then the flipped rows "
                       "of K read four at a time by every thread (latency of the row reads)"}
    print(f"bench: dense N={N}: T_HMC {out['T_HMC_us']} us, T_MH {out['T_MH_us']} us, ratio/N_step "
          f"{out['T_HMC_over_Nstep_T_MH']}", file=sys.stderr, flush=True)
    return out


def bench_mh(args):
    cmp = run_mh_compare(args)
    line = {"metric": "T_HMC / (N_step T_MH)", "value": cmp["points"][-1]["T_HMC_over_Nstep_T_MH"],
            "unit": "ratio", "n_gpus": 1, "steps": None, "warmup": None, "ms_per_step": None,
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32/int8",
            "data": "synthetic", "config": {"workload": "HMC vs Metropolis-Hastings: " + cmp["workload"]},
            "mh_compare": cmp, "roofline": None, "cpu_baseline": None}
    print(json.dumps(line), flush=True)


def bench_tau(args):
    """Critical slowing down measured on the batched engine (Sec. 4): tau_int of
    |m| against N at the critical coupling in 2D and 3D, with the paper's fits
    tau = alpha N^(2/d) and a free exponent, and against C - n at N = 15^2 (2D).
    Every point runs `chains` independent replicas of `steps` unit trajectories
    (after `warmup` discarded ones) with floor(log N) leap-frog steps, FP32
    state, all points advanced together as one chain set."""
    from paper_1912_03278_amd import autocorr as A, ihmc, inputs

    K, W, R = args.steps, args.warmup, args.tau_chains
    pts2 = [dict(L=(L, L), beta=inputs.BETA_C_2D, C=4.1) for L in (4, 6, 8, 11, 16, 23, 32)]
    pts3 = [dict(L=(L,) * 3, beta=inputs.BETA_3D, C=6.1) for L in (3, 4, 5, 6, 8, 10)]
    dcs = (0.05, 0.25, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0)
    ptsC = [dict(L=(15, 15), beta=inputs.BETA_C_2D, C=4.0 + dc) for dc in dcs]
    ctx = ihmc.Context(device=0, arena_bytes=6 << 30, resident=args.resident_sites, fuse_steps=args.fuse_steps)
    pts = pts2 + pts3 + ptsC
    print(f"bench: tau_int scan, {len(pts)} points x {R} chains x {W + K} trajectories", file=sys.stderr,
          flush=True)
    out = A.run_scan(ctx, pts, n_chains=R, n_traj=K, n_therm=W, seed=17)
    ctx.close()
    run_s = out[0]["run_s"]
    work = sum(r["site_md_steps"] for r in out)
    r2, r3, rC = out[:len(pts2)], out[len(pts2):len(pts2) + len(pts3)], out[len(pts2) + len(pts3):]

    def fits(rows, d):
        rows = [r for r in rows if r["N"] > 10]
        N = [r["N"] for r in rows]
        tau = [r["tau_int"] for r in rows]
        err = [r["tau_err"] for r in rows]
        fixed = A.fit_power(N, tau, err, exponent=2.0 / d)
        free = A.fit_power(N, tau, err)
        return {"alpha_at_2_over_d": fixed["alpha"], "alpha_err": fixed["alpha_err"],
                "chi2_dof_at_2_over_d": fixed["chi2_dof"], "free_gamma": free["gamma"],
                "free_gamma_err": free["gamma_err"], "z": d * free["gamma"], "z_err": d * free["gamma_err"]}

    def rowfmt(rows, key):
        return [{key: r[key] if key != "C_minus_n" else round(r["C"] - 2 * len(r["L"]), 4), "N": r["N"],
                 "n_md": r["n_md"], "tau_int": round(r["tau_int"], 4), "tau_err": round(r["tau_err"], 4),
                 "abs_m": round(r["mean"], 6), "abs_m_err": round(r["err"], 6),
                 "acceptance": round(r["acceptance"], 4)} for r in rows]

    t0 = rC[0]
    c_crit = next((round(r["C"] - 4.0, 4) for r in rC[1:]
                   if r["tau_int"] > t0["tau_int"] + 3 * math.hypot(t0["tau_err"], r["tau_err"])), None)
    line = {
        "metric": "site-MD-steps/s", "value": work / run_s, "unit": "site-MD-steps/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": 1000.0 * run_s / (K + W), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"tau_int scans at the critical coupling, h = 0, {R} replicas per point, "
                               f"{K} trajectories after {W}, n_md = floor(log N): 2D L 4..32 (C = 4.1), "
                               "3D L 3..10 (C = 6.1), 2D 15^2 with C - n from 0.05 to 4; one step = one "
                               "trajectory of every chain", "chains": R * len(pts), "resident": args.resident,
                   "fuse_steps": args.fuse},
        "tau_2d": {"points": rowfmt(r2, "L"), "fit": fits(r2, 2)},
        "tau_3d": {"points": rowfmt(r3, "L"), "fit": fits(r3, 3)},
        "tau_vs_C": {"points": rowfmt(rC, "C_minus_n"), "first_C_minus_n_above_plateau": c_crit},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def run_large(args, K=None, W=None):
    """Single large chains: 2D 1024^2 at beta_c and 3D 128^3 at beta = 0.2216544,
    FP32 state, FP64 H, h = 0, 20 MD steps; one step = one trajectory of both.
    Returns the JSON line (extra keys included)."""
    import torch
    from paper_1912_03278_amd import ihmc

    ws = large_workload()
    K = args.steps if K is None else K
    W = args.warmup if W is None else W
    ctx = ihmc.Context(device=0, arena_bytes=2 << 30, resident=args.resident_sites, fuse_steps=args.fuse_steps)
    lats = [ihmc.Lattice(w["L"], beta=w["beta"], C=w["C"]) for w in ws]
    runs = [ihmc.Run(n_md=w["n_md"], n_traj=W + K, precision=ihmc.F32, seed=w["seed"], chain_id=w["chain_id"])
            for w in ws]
    tiles = tune_tiles(ctx, lats, args)
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
    # groups are ordered (precision, ndim, tile class): the 2D chain, then the 3D one
    # per group, the launch kind that carries most of its middle steps: the
    # two-step launch of a fused 2D group (plus one single step for an odd
    # number of middle steps), else the one-step pass; both move 16 B per site
    kern = group_rows(chains, args.timing_reps, modes=(1, 0, 2), pair=args.fuse_steps)
    for g, k in enumerate(kern):
        n_mid = ws[g]["n_md"] - 1
        if "pair_us" in k:
            k["kind"], k["kind_us"] = "two-step middle pass", k["pair_us"]
            k["middle_share_us"] = (n_mid // 2) * k["pair_us"] + (n_mid % 2) * k["middle_us"]
            k["steps_per_launch"] = 2
        else:
            k["kind"], k["kind_us"] = "middle pass", k["middle_us"]
            k["middle_share_us"] = n_mid * k["middle_us"]
            k["steps_per_launch"] = 1
    dom = max(kern, key=lambda k: k["middle_share_us"])
    n_md = ws[0]["n_md"]
    phys_bytes = BYTES_MIDDLE_F32 * dom["sites"]
    alg_bytes = dom["steps_per_launch"] * dom["sites"] * (16.0 + 4.0 / n_md)
    achieved = alg_bytes / (dom["kind_us"] * 1e-6) / 1e9
    achieved_phys = phys_bytes / (dom["kind_us"] * 1e-6) / 1e9
    dom_kind, dom_us, dom_steps = dom["kind"], dom["kind_us"], dom["steps_per_launch"]
    for k in kern:
        for name in ("middle", "pair"):
            if f"{name}_us" in k:
                k[f"{name}_physical_GBs"] = round(BYTES_MIDDLE_F32 * k["sites"] / (k[f"{name}_us"] * 1e-6) / 1e9, 1)
                k[f"{name}_us"] = round(k[f"{name}_us"], 3)
        k["first_us"] = round(k["first_us"], 3)
        k["last_us"] = round(k["last_us"], 3)
        for name in ("middle_share_us", "kind", "kind_us", "steps_per_launch"):
            del k[name]

    copy_bytes = 512 << 20
    copy_us = ctx.copy_bandwidth(copy_bytes, reps=10)
    copy_gbs = 2 * copy_bytes / (copy_us * 1e-6) / 1e9
    line = {
        "metric": "site-MD-steps/s", "value": value, "unit": "site-MD-steps/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": 1000.0 * dt / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {
            "workload": "single large chains: 2D 1024^2 at beta_c=0.4406868 (C=4.1) and 3D 128^3 at "
                        "beta=0.2216544 (C=6.1), J=1, h=0, 20 leap-frog steps per unit trajectory, FP32 "
                        "state, FP64 H/dH/Metropolis; one step = one trajectory of both chains",
            "sites": sum(int(math.prod(w["L"])) for w in ws),
            "md_steps_per_trajectory": n_md, "fuse_steps": args.fuse, **tiles,
        },
        "roofline": {
            "bound": "hbm", "kernel": f"fused {dom_kind}, {dom['ndim']}D",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_bytes(("large_3d_" if dom["ndim"] == 3 else "large_2d_") +
                                     ("pair" if dom_kind.startswith("two") else "middle"),
                                     sites=dom["sites"], tiles=dom["tiles"]),
            "algorithmic_bytes_per_launch": int(alg_bytes),
            "algorithmic_basis": f"(16 + 4/n_md) B per site-MD-step x {dom_steps} MD step(s) "
                                 "per site and launch",
            "physical_bytes_per_launch": phys_bytes, "achieved_physical": round(achieved_phys, 1),
            "frac_physical": round(achieved_phys / HBM_PEAK_GBS, 4),
            "avg_launch_us": round(dom_us, 3),
            "copy_kernel_GBs": round(copy_gbs, 1), "frac_physical_of_copy": round(achieved_phys / copy_gbs, 4),
        },
        "kernels": kern,
        "chains": per,
    }
    chains.close()
    ctx.close()
    if not args.no_streaming_point:
        line["extra_streaming_point"] = streaming_point(args, copy_gbs)
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on one trajectory of each large chain", file=sys.stderr, flush=True)
        jobs = [dict(L=w["L"], beta=w["beta"], C=w["C"], h=None, n_md=w["n_md"], n_traj=1, seed=w["seed"],
                     chain_id=w["chain_id"]) for w in ws]
        line["cpu_baseline"] = oracle_parallel(jobs, reps=3, what="one trajectory of the 1024^2 and of the "
                                                                    "128^3 chain")
    else:
        line["cpu_baseline"] = None
    return line


def bench_large(args):
    print(json.dumps(run_large(args)), flush=True)


def bench_headline(args):
    """The batched workload's line, with the single large chains, the streaming
    point and the serving run as extra keys."""
    line = run_batched(args)
    if args.extras in ("all", "large"):
        print("bench: extra key: single large chains", file=sys.stderr, flush=True)
        lg = run_large(args, K=max(args.steps, 20), W=max(args.warmup, 5))
        line["extra_large_chains"] = {k: lg[k] for k in ("value", "unit", "ms_per_step", "steps", "warmup", "config",
                                                         "roofline", "kernels", "chains", "cpu_baseline")}
        if "extra_streaming_point" in lg:
            line["extra_streaming_point"] = lg["extra_streaming_point"]
    if args.extras in ("all", "phi"):
        print("bench: extra key: phi/psi form A/B", file=sys.stderr, flush=True)
        line["extra_phi_form_ab"] = run_phi_ab(args)
    if args.extras in ("all", "mh"):
        print("bench: extra key: HMC trajectory against Metropolis-Hastings sweep", file=sys.stderr, flush=True)
        line["extra_mh_compare"] = run_mh_compare(args)
    if args.extras in ("all", "dense"):
        print("bench: extra key: dense all-to-all chains", file=sys.stderr, flush=True)
        dargs = argparse.Namespace(**vars(args))
        dargs.steps, dargs.warmup = 100, 5
        dn = run_dense(dargs)
        line["extra_dense"] = {k: dn[k] for k in ("value", "unit", "ms_per_step", "steps", "warmup", "dtype", "config",
                                                  "roofline", "kernels", "acceptance_mean", "cpu_baseline")}
    if args.extras in ("all", "serving"):
        print("bench: extra key: serving", file=sys.stderr, flush=True)
        sv = run_serving(args)
        line["extra_serving"] = sv
        line["latency_s"] = sv["latency_s"]
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "batched", "large", "dense", "serving", "small", "tau", "phi", "mh"],
                    help="headline (default): the batched workload with the large chains, the streaming point and "
                         "serving as extra keys; batched: 4096 uneven chains only; large: the 1024^2 + 128^3 single "
                         "chains; dense: 256 chains of an N=4096 all-to-all model; serving: Poisson request arrivals")
    ap.add_argument("--extras", default="all", choices=["all", "large", "dense", "serving", "phi", "mh", "none"],
                    help="headline: which extra keys to run")
    ap.add_argument("--rate", type=float, default=200.0, help="serving: arrivals per second")
    ap.add_argument("--serve-duration", type=float, default=60.0, help="serving: seconds of arrivals")
    ap.add_argument("--drain", type=float, default=120.0, help="serving: seconds allowed after the last arrival")
    ap.add_argument("--products", type=int, default=6, choices=[3, 6], help="dense: BF16 limb products")
    ap.add_argument("--chains", type=int, default=4096, help="batched: number of chains")
    ap.add_argument("--plain-sample", type=int, default=16, help="batched: chains rerun alone")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle timing")
    ap.add_argument("--no-streaming-point", action="store_true", help="large: skip the extra 8192^2 point")
    ap.add_argument("--timing-reps", type=int, default=100)
    ap.add_argument("--tau-chains", type=int, default=128, help="tau: replicas per scan point")
    ap.add_argument("--phi-chains", type=int, default=512, help="phi: chains per lattice shape of the A/B")
    ap.add_argument("--resident", default="on", choices=["on", "off"],
                    help="chains that fit one workgroup's LDS run whole trajectories per launch (on) or the "
                         "tiled passes (off); results are bit-identical")
    ap.add_argument("--fuse", default="on", choices=["on", "off"],
                    help="2D chains on the tiled passes run two middle leap-frog steps per launch (on) or one "
                         "(off); results are bit-identical")
    ap.add_argument("--tiles", default="tuned", choices=["tuned", "rule"],
                    help="tile classes: autotuned per lattice shape before the run (default), or the built-in rule")
    args = ap.parse_args()
    args.resident_sites = -1 if args.resident == "on" else 0
    args.fuse_steps = args.fuse == "on"
    if args.gpus != 1:
        print("bench.py: runs on one GPU only; sharding chains or a lattice over several GPUs is a design, "
              "not implemented here", file=sys.stderr)
        sys.exit(2)
    if args.workload in ("headline", "batched"):
        args.steps = 10 if args.steps is None else args.steps
        args.warmup = 2 if args.warmup is None else args.warmup
        return bench_headline(args) if args.workload == "headline" else bench_batched(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "mh":
        return bench_mh(args)
    if args.workload == "phi":
        args.steps = 20 if args.steps is None else args.steps
        args.warmup = 2 if args.warmup is None else args.warmup
        return bench_phi(args)
    if args.workload == "tau":
        args.steps = 8000 if args.steps is None else args.steps
        args.warmup = 1000 if args.warmup is None else args.warmup
        return bench_tau(args)
    if args.workload == "small":
        args.steps = 2000 if args.steps is None else args.steps
        args.warmup = 200 if args.warmup is None else args.warmup
        return bench_small(args)
    if args.workload == "dense":
        args.steps = 100 if args.steps is None else args.steps
        args.warmup = 5 if args.warmup is None else args.warmup
        return bench_dense(args)
    args.steps = 200 if args.steps is None else args.steps
    args.warmup = 20 if args.warmup is None else args.warmup
    return bench_large(args)


if __name__ == "__main__":
    main()
