#!/usr/bin/env python3
"""Benchmark of the ensemble flood hot path on one MI355X.

Workload (default): 2000 x 2000 cells (4.0 M, 3 m), 96 members, FP32 state,
urban synthetic DEM, Chicago storm, per-member lognormal Manning scales and
rain multipliers, particle filter every 600 s on 10 depth gauges.

One benchmark step = one assimilation cycle: every member advances 600 s of
simulated time (adaptive Eq. 4 steps, one fused kernel launch per step for
all members) followed by the filter update (gauge gather, weights, N_eff,
systematic resampling and member copy when N_eff < 0.8 N).  Observations
come from a hidden truth member run beforehand plus N(0, 0.05^2) noise.

Metric: member-cell-updates per second (MCU/s) over the timed steps,
counted from the per-member step counters.  The JSON line also carries the
roofline of the step kernel (HIP-event durations of every step launch in the
timed region) and the FP64 oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_MCU = 24.0    # h, qx, qy read + written once per member-cell-step (FP32)


def _cpu_worker(args):
    """Run one member of the workload with the oracle for n_steps from the dry start."""
    cfg, member, n_steps = args
    import oracle
    import workloads as W
    wl = W.CONFIGS[cfg["config"]](cfg["ny"], cfg["nx"], cfg["members"])
    c = wl.catchments[0]
    m = oracle.Model.from_workload(wl)
    mem = oracle.Member.dry(m, s=c.n_scale[member], mu=c.rain_mult[member])
    t0 = time.perf_counter()
    n = oracle.advance(m, mem, wl.t_end, max_steps=n_steps)
    el = time.perf_counter() - t0
    return n * c.ny * c.nx, el


def cpu_baseline(cfg, cores, n_steps):
    ctx = mp.get_context("spawn")
    jobs = [(cfg, i % cfg["members"], n_steps) for i in range(cores)]
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_cpu_worker, jobs)
    wall = time.perf_counter() - t0
    mcu = sum(r[0] for r in res)
    busy = max(r[1] for r in res)
    return {"value": mcu / busy, "unit": "MCU/s", "cores": cores, "kind": "oracle",
            "sample": "FP64 serial oracle, one process per core, each running one member of the same "
                      "workload for its first %d steps from the dry start (%d member-runs, %.1f s per "
                      "process, %.1f s wall incl. start-up)" % (n_steps, cores, busy, wall)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=5)
    ap.add_argument("--ny", type=int, default=2000)
    ap.add_argument("--nx", type=int, default=2000)
    ap.add_argument("--members", type=int, default=96)
    ap.add_argument("--window", type=float, default=600.0, help="simulated seconds per assimilation cycle")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=60)
    ap.add_argument("--cpu-cores", type=int, default=0)
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--mi", type=int, default=0)
    ap.add_argument("--rows", type=int, default=0)
    ap.add_argument("--cpb", type=int, default=0)
    ap.add_argument("--kernel", type=int, default=0, help="0 autotune, 1 tiled, 2 row-marching")
    ap.add_argument("--kernel-only", type=int, default=0,
                    help="after the warm-up, time this many single steps in which every member steps")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the run, copy a 1 GiB device buffer (counter calibration for profiling)")
    ap.add_argument("--march-rows", type=int, default=0)
    ap.add_argument("--march-members", type=int, default=0)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: members shard across GPUs without communication between "
              "filter updates, and this build measures the single-GPU path (see DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    cfg = {"config": args.config, "ny": args.ny, "nx": args.nx, "members": args.members}
    cpu = None
    if not args.no_cpu:
        cores = args.cpu_cores or min(16, os.cpu_count() or 1)
        cpu = cpu_baseline(cfg, cores, args.cpu_steps)

    import torch
    import workloads as W
    from paper_2302_08341_amd import FloodEnsemble

    torch.cuda.set_device(0)
    wl = W.CONFIGS[args.config](args.ny, args.nx, args.members)
    c = wl.catchments[0]
    N = c.n_members
    ncell = c.ny * c.nx
    K = c.gauges.shape[0]
    sigma = np.full(K, wl.obs_sigma)
    n_cycles = args.warmup + args.steps
    rng = np.random.default_rng(wl.seed + 7)

    # observations: hidden truth member drawn from the same prior
    truth = FloodEnsemble([dict(dem=c.dem, manning=c.manning, dx=c.dx, edge_kind=c.edge_kind,
                                edge_slope=c.edge_slope, n_members=1, n_scale=[c.truth_n_scale],
                                rain_mult=[c.truth_rain_mult])], wl.rain, real_bytes=wl.real_bytes)
    obs = []
    for k in range(n_cycles):
        truth.step((k + 1) * args.window)
        hv = truth.field(0)[c.gauges[:, 0], c.gauges[:, 1]]
        obs.append(W.obs_noise(rng, hv, wl.obs_sigma))
    truth.close()
    draws = [W.pf_draws(rng, N) for _ in range(n_cycles)]

    ens = FloodEnsemble.from_workload(wl, member_interleave=args.mi, tile_rows=args.rows,
                                      chunks_per_block=args.cpb, step_kernel=args.kernel,
                                      march_rows=args.march_rows, march_members=args.march_members)
    conf = ens.config()
    resampled = []

    def cycle(k):
        ens.step((k + 1) * args.window)
        u0, beta = draws[k]
        neff, anc, res = ens.assimilate(0, c.gauges, obs[k], sigma, 0.8, u0, beta)
        resampled.append(bool(res))

    for k in range(args.warmup):
        cycle(k)
    torch.cuda.synchronize()
    if args.kernel_only:
        # every launch steps every member: single steps of 0.02 s, shorter than Eq. 4 allows here
        t = args.warmup * args.window
        l0 = ens.ledger()
        ens.timing(True)
        for i in range(args.kernel_only):
            ens.step(t + 0.02 * (i + 1))
        ens.timing(False)
        l1 = ens.ledger()
        avg_ms, launches = ens.get_timing()
        steps = int((l1["steps"] - l0["steps"]).sum())
        full = steps // args.kernel_only
        gbs = BYTES_PER_MCU * full * ncell / (avg_ms * 1e-3) / 1e9 if launches == args.kernel_only else None
        # attainable streaming bandwidth: one elementwise kernel reading and writing 2 GiB each
        x = torch.ones(1 << 29, dtype=torch.float32, device="cuda")
        ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        y = x + 1.0
        torch.cuda.synchronize()
        ea.record()
        for _ in range(5):
            y = x + 1.0
        eb.record()
        torch.cuda.synchronize()
        copy_gbs = 5 * 2 * x.numel() * 4 / (ea.elapsed_time(eb) * 1e-3) / 1e9
        del x, y
        print(json.dumps({"kernel_only": True, "members_per_launch": full, "real_launches": args.kernel_only,
                          "timed_launches": launches, "avg_launch_ms": avg_ms, "algorithmic_GBps": gbs,
                          "elementwise_copy_GBps": copy_gbs,
                          "config": ens.config()}))
        return
    led0 = ens.ledger()
    if not args.no_kernel_timing:
        ens.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.warmup, n_cycles):
        cycle(k)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if not args.no_kernel_timing:
        ens.timing(False)
    led1 = ens.ledger()
    avg_ms, launches = ens.get_timing()

    member_steps = int((led1["steps"] - led0["steps"]).sum())
    mcu = member_steps * ncell
    value = mcu / elapsed
    mass = float(np.max(np.abs(led1["storage"] - (led1["rain_in"] - led1["outflow"] + led1["clamp"]))
                        / np.maximum(led1["rain_in"], 1e-30)))

    roof = None
    if launches:
        mcu_per_launch = mcu / launches
        achieved = BYTES_PER_MCU * mcu_per_launch / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_march (row-marching fused step)" if conf["step_kernel"] == 2
                          else "k_step (tiled fused step)",
                "avg_launch_ms": round(avg_ms, 4), "launches": launches,
                "algorithmic_bytes_per_launch": round(BYTES_PER_MCU * mcu_per_launch)}

    out = {
        "metric": "member-cell-updates/s fwd & fwd+adj; % HBM peak; batched vs plain, 96x4M",
        "value": value,
        "unit": "MCU/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if wl.real_bytes == 4 else "f64",
        "data": "synthetic",
        "config": {"workload": "urban %dx%d cells x %d members, FP32, PF every %.0f s (%d gauges); one step = "
                               "one %.0f s assimilation cycle" % (c.ny, c.nx, N, args.window, K, args.window),
                   "cells": ncell, "members": N, "window_s": args.window,
                   "sim_time_s": [args.warmup * args.window, n_cycles * args.window],
                   "member_interleave": conf["member_interleave"], "tile_rows": conf["tile_rows"],
                   "chunks_per_block": conf["chunks_per_block"], "step_kernel": conf["step_kernel"],
                   "march_rows": conf["march_rows"], "march_members": conf["march_members"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "detail": {"member_steps": member_steps, "mcu": mcu, "elapsed_s": elapsed,
                   "resampled": resampled[args.warmup:], "mass_balance_rel": mass,
                   "paper_context": "8x P100: 4.69e10 MCU/s (96 x 4.0 M cells x 14,400 steps in 118 s)"},
    }
    if args.copy_calibration:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        y = x + 1.0          # one elementwise kernel: reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del y
        out["detail"]["copy_calibration_bytes"] = 2 * x.numel() * 4
    print(json.dumps(out))


if __name__ == "__main__":
    main()
