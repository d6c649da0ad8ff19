#!/usr/bin/env python3
"""Throughput of the KPZ octahedron sweep on one MI355X.

Workload (default): L = 65536 periodic lattice (2^32 sites, 1 GiB of packed
slopes), p = 1, q = 0, flat start, Philox seed 1, 256 x 256 dead-border
blocks with 4 x 4 double tiles; W^2 is sampled every 10 MCS.  One "step" =
10 MCS followed by one exact W^2 sample (the full hot path: init once, then
sweep + roughness).  Value = site-update attempts per second over the timed
steps, with the lattice already resident in HBM.

Prints one JSON line.  Besides the contract fields it carries
  roofline      the sweep kernel's integer-ALU roofline (HIP events on the
                sweep's stream give its mean launch time), plus its HBM view
  cpu_baseline  the CPU oracle timed on a bounded sample of the same workload
                (single blocks of the same lattice, same draws)
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peak rates of MI355X used for the roofline (public figures): HBM3E 8 TB/s;
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 32-bit integer VALU lane
# operations per second (the fp32 vector peak of 157.3 TFLOP/s counts packed
# FMAs as 4 flops per lane-cycle).
HBM_PEAK_GBS = 8000.0
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic cost of one attempt (bytes and integer operations); derivation
# in the design doc (sweep roofline).
BYTES_PER_ATTEMPT = 0.5
OPS_PER_ATTEMPT = 9.0


def cpu_baseline(L, block, p, q, seed, budget_s):
    """Oracle on single blocks of MCS 0 of the same lattice: block after
    block until the time budget is used; attempts/s = blocks * Bx*By / time."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    Bx, By = block
    ox, oy = oracle.dd_origin(seed, 0, block)
    y, x = np.mgrid[0:By, 0:Bx]
    n_done = 0
    t0 = time.perf_counter()
    nbx = L // Bx
    b = 0
    while True:
        bx, by = b % nbx, b // nbx
        # flat start: the block's slopes depend only on the parity of its corner
        gx0, gy0 = (ox + bx * Bx) % L, (oy + by * By) % L
        par = (x + y + gx0 + gy0) & 1
        sx = np.where(par == 0, 1, -1).astype(np.int8)
        sy = sx.copy()
        oracle.dd_block_mcs(L, p, q, seed, block, 0, bx, by, sx, sy)
        n_done += 1
        b += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": n_done * Bx * By / dt, "unit": "attempts/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_done} dead-border blocks of {Bx}x{By} sites, MCS 0 of the L={L} "
                      f"lattice (p={p}, q={q}, seed {seed}), plain single-threaded C oracle, "
                      f"{dt:.1f} s on {platform.processor() or platform.machine()}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--L", type=int, default=65536)
    ap.add_argument("--block", type=int, nargs=2, default=[256, 256])
    ap.add_argument("--mcs-per-step", type=int, default=10)
    ap.add_argument("--p", type=float, default=1.0)
    ap.add_argument("--q", type=float, default=0.0)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on exactly one GPU (one lattice per device); "
              "--gpus N with N > 1 is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1204_5072_amd as kpz

    L, M = args.L, args.mcs_per_step
    block = tuple(args.block)
    print(f"bench: L={L} block={block} p={args.p} q={args.q} seed={args.seed} "
          f"steps={args.steps} warmup={args.warmup} mcs/step={M}", file=sys.stderr, flush=True)
    sim = kpz.Sim(L, args.p, args.q, args.seed, block)
    stream = sim.stream
    for _ in range(args.warmup):
        sim.sweep(M)
        sim.roughness()
    torch.cuda.synchronize()

    n = args.steps * M
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(n)]
    rev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    w2 = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        for m in range(M):
            e0, e1 = ev[s * M + m]
            e0.record(stream)
            sim.sweep(1)
            e1.record(stream)
        rev[s][0].record(stream)
        w2.append(sim.roughness().W2)
        rev[s][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    sweep_ms = sum(a.elapsed_time(b) for a, b in ev) / n
    rough_ms = sum(a.elapsed_time(b) for a, b in rev) / args.steps
    attempts = float(L) * L * n
    value = attempts / elapsed
    per_launch_attempts = float(L) * L
    sweep_s = sweep_ms / 1e3
    achieved_tops = OPS_PER_ATTEMPT * per_launch_attempts / sweep_s / 1e12
    achieved_gbs = BYTES_PER_ATTEMPT * per_launch_attempts / sweep_s / 1e9
    line = {
        "metric": "site-update attempts/s at L=2^16",
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": f"KPZ octahedron L={L} periodic, p={args.p} q={args.q}, flat start, "
                        f"Philox seed {args.seed}, dead-border blocks {block[0]}x{block[1]}, "
                        f"4x4 double tiles; step = {M} MCS + one exact W^2 sample",
            "L": L, "block": list(block), "tile": [4, 4], "mcs_per_step": M,
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved_tops,
            "peak": VALU_PEAK_TOPS,
            "unit": "Tops/s",
            "frac": achieved_tops / VALU_PEAK_TOPS,
            "traffic": None,
            "kernel": "kpz_sweep_kernel",
            "mean_launch_ms": sweep_ms,
            "ops_per_attempt": OPS_PER_ATTEMPT,
            "hbm_achieved_gbs": achieved_gbs,
            "hbm_frac": achieved_gbs / HBM_PEAK_GBS,
        },
        "roughness_ms": rough_ms,
        "w2_last": w2[-1] if w2 else None,
        "t_final": sim.state()[0],
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(L, block, args.p, args.q, args.seed, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
