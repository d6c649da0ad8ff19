#!/usr/bin/env python3
"""Throughput of the KPZ octahedron sweep on one MI355X.

Workload (default): L = 65536 periodic lattice (2^32 sites, 1 GiB of packed
slopes), p = 1, q = 0, flat start, Philox seed 1, 1024 x 32 dead-border
blocks (the fastest shape at this L) with 4 x 4 double tiles; W^2 is sampled
every 10 MCS.  One "step" = 10 MCS followed by one exact W^2 sample (the
full hot path: init once, then sweep + roughness).  Value = site-update
attempts per second over the timed steps, with the lattice already resident
in HBM.

Prints one JSON line.  Besides the contract fields it carries
  roofline      the sweep launch (one MCS) against the vector-ALU issue
                ceiling measured in the same run by kpz_valu_probe (the
                kernel's VALU instruction count per launch comes from the
                committed rocprofv3 counter summary of the same code), and
                its HBM view at the algorithmic 0.5 B per attempt
  cpu_baseline  the CPU oracle (the same decomposed schedule and draws) on a
                smaller lattice with the same block shape, on all host cores
                and on one
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

# HBM3E peak of MI355X (public figure).
HBM_PEAK_GBS = 8000.0
# Algorithmic traffic of one attempt: the packed lattice (2 bits per site)
# is read once and written once per MCS.
BYTES_PER_ATTEMPT = 0.5


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(block, p, q, seed, budget_s):
    """The oracle's decomposed schedule (or_dd_run_par, the plain C runner
    with the blocks of a residency spread over OpenMP threads) on an L = 2048
    lattice with the benchmark's block shape, p, q and seed, from the flat
    start, MCS after MCS until half the budget is used: once on all host
    cores, once on one.  attempts/s = MCS * L^2 / time."""
    import oracle
    oracle.build(force=False)
    L = 2048
    threads = os.cpu_count() or 1

    def run(nthreads, budget):
        st = oracle.SlopeState(L)
        t0 = time.perf_counter()
        n = 0
        while True:
            st.run_dd(1, p, q, seed, block=block, tile=(4, 4), threads=nthreads)
            n += 1
            if time.perf_counter() - t0 > budget:
                break
        return n, time.perf_counter() - t0

    n_all, t_all = run(threads, budget_s / 2)
    n_one, t_one = run(1, budget_s / 2)
    return {"value": n_all * L * L / t_all, "unit": "attempts/s", "cores": threads,
            "kind": "oracle",
            "single_core": n_one * L * L / t_one,
            "cpu_model": cpu_model(),
            "sample": f"L={L} lattice, {block[0]}x{block[1]} dead-border blocks, p={p} q={q} "
                      f"seed {seed}, flat start: {n_all} MCS on {threads} threads in {t_all:.1f} s "
                      f"and {n_one} MCS on one thread in {t_one:.1f} s (plain C oracle, "
                      f"or_dd_run_par), {cpu_model()}"}


def valu_ceiling(reps: int = 3):
    """Vector-ALU issue ceiling of this device for the sweep's instruction
    mix: kpz_valu_probe (8192 waves, exactly counted bitwise instructions),
    best of `reps` timings with HIP events; wave instructions per second."""
    import ctypes
    import torch
    import paper_1204_5072_amd as kpz
    groups, iters = 2048, 1000
    out = torch.empty(groups * 256, dtype=torch.int32, device="cuda")
    ops = ctypes.c_int32()
    st = torch.cuda.current_stream()
    best = None
    for _ in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        rc = kpz.lib().kpz_valu_probe(ctypes.c_void_p(out.data_ptr()), groups, iters,
                                      ctypes.byref(ops), ctypes.c_void_p(st.cuda_stream))
        e1.record(st)
        torch.cuda.synchronize()
        if rc != 0:
            return None
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return groups * 4 * iters * ops.value / (best * 1e-3)


def log_times(n=64, t_max=10_000):
    """n log-spaced sampling times ending at t_max: t_k = max(t_{k-1} + 1,
    round(t_max^(k/(n-1))))."""
    out = []
    for k in range(n):
        t = max((out[-1] + 1) if out else 1, round(t_max ** (k / (n - 1))))
        out.append(int(t))
    return out


# Block shape per lattice size of the ensemble leg: the autotuner's pick on
# MI355X (autotune.tune_ensemble: the first candidate within 3 % of the
# fastest).  Fixed here because the shape is part of the dynamics and the
# candidates lie within the run-to-run timing noise of each other;
# --ens-autotune tunes afresh and reports the timings.
ENS_BLOCKS = {256: (128, 128), 512: (128, 256), 1024: (128, 256), 2048: (512, 64)}


def ensemble_leg(args):
    """The batched ensemble: 512 lattices, L uniform over {256,...,2048},
    p = 1, q uniform over {0, 1/4, 1/2}, seeds 1000 + r (job table from numpy
    default_rng(0)), 10^4 MCS with W^2 at 64 log-spaced times, run as one
    captured graph (per MCS: one launch over every member's blocks and one
    straddling-word merge); compared with plain single-lattice launches of a
    subset of the same members, one after another."""
    import numpy as np
    import torch
    import paper_1204_5072_amd as kpz
    from paper_1204_5072_amd import autotune

    rng = np.random.default_rng(0)
    n = args.ens_members
    Ls = rng.choice([256, 512, 1024, 2048], size=n)
    qs = rng.choice([0.0, 0.25, 0.5], size=n)
    base = [kpz.make_params(int(L), 1.0, float(q), 1000 + r) for r, (L, q) in enumerate(zip(Ls, qs))]
    tuned = None
    if args.ens_block:
        blocks = {int(L): tuple(args.ens_block) for L in set(Ls)}
    elif args.ens_autotune:
        tuned = autotune.tune_ensemble(base)
        blocks = tuned["blocks"]
        print(f"bench: ensemble blocks {blocks} (tuned per L)", file=sys.stderr, flush=True)
    else:
        blocks = dict(ENS_BLOCKS)
    members = [kpz.make_params(m.L, m.p, m.q, m.seed, blocks[int(m.L)]) for m in base]
    times = log_times(64, args.ens_mcs)
    ens = kpz.Ensemble(members)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S1, S2, W2 = ens.run(times)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    attempts = float(sum(int(L) ** 2 for L in Ls)) * times[-1]
    print(f"bench: ensemble run {elapsed:.2f} s", file=sys.stderr, flush=True)
    ens.close()
    # sequential plain launches: a subset of members, each on its own
    m_seq = min(args.ens_seq_members, n)
    seq_mcs = 5
    sims = [kpz.Sim(m.L, m.p, m.q, m.seed, blocks[int(m.L)]) for m in members[:m_seq]]
    for sim in sims:
        sim.sweep(1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for sim in sims:
        sim.sweep(seq_mcs)
    torch.cuda.synchronize()
    seq_elapsed = time.perf_counter() - t1
    seq_attempts = float(sum(m.L ** 2 for m in members[:m_seq])) * seq_mcs
    final = {}
    for L in (256, 512, 1024, 2048):
        sel = Ls == L
        if sel.any():
            final[str(L)] = float(np.mean(W2[-1][sel]))
    return {
        "metric": "site-update attempts/s, batched ensemble",
        "value": attempts / elapsed,
        "unit": "attempts/s",
        "seconds": elapsed,
        "members": n,
        "mcs": times[-1],
        "samples": len(times),
        "blocks_by_L": {str(L): list(b) for L, b in sorted(blocks.items())},
        "autotune_ms_per_mcs": ({str(L): {f"{k[0]}x{k[1]}": v for k, v in t.items()}
                                 for L, t in tuned["ms_per_mcs"].items()} if tuned else None),
        "sequential_plain_launches": {"value": seq_attempts / seq_elapsed, "unit": "attempts/s",
                                      "members": m_seq, "mcs": seq_mcs},
        "speedup_vs_sequential": (attempts / elapsed) / (seq_attempts / seq_elapsed),
        "mean_w2_final_by_L": final,
        # each member's lattice is read and written once per MCS (0.5 B per
        # attempt); the members' lattices (about 180 MB) stay in the 256 MB
        # last-level cache, so the HBM figure is nominal
        "roofline": {"bound": "alu", "hbm_achieved_gbs": 0.5 * attempts / elapsed / 1e9,
                     "hbm_peak_gbs": HBM_PEAK_GBS,
                     "hbm_frac": 0.5 * attempts / elapsed / 1e9 / HBM_PEAK_GBS,
                     "bytes_per_attempt": 0.5},
    }


def growth_leg(args):
    """The L = 4096 growth runs: p = 1, q = 0 (KPZ) and p = q = 1/2 (EW),
    seeds 1..8 each, flat start, 10^4 MCS with W^2 at 64 log-spaced times,
    all 16 realisations as one ensemble graph with the default block shape.
    Reports the rate and, per (p, q), the seed-mean W^2 at the last time and
    the slope of log W^2 against log t over the last decade (2 beta for KPZ,
    about 0.48 in 2+1 d; EW grows like log t, so its slope falls)."""
    import numpy as np
    import torch
    import paper_1204_5072_amd as kpz

    L, n_seeds = 4096, 8
    runs = [(1.0, 0.0), (0.5, 0.5)]
    members = [kpz.make_params(L, p, q, seed) for p, q in runs for seed in range(1, n_seeds + 1)]
    times = log_times(64, args.growth_mcs)
    ens = kpz.Ensemble(members)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, W2 = ens.run(times)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ens.close()
    W2 = np.asarray(W2, dtype=np.float64)
    t = np.asarray(times, dtype=np.float64)
    late = t >= t[-1] / 10
    out = {}
    for k, (p, q) in enumerate(runs):
        w = W2[:, k * n_seeds:(k + 1) * n_seeds].mean(axis=1)
        slope = float(np.polyfit(np.log(t[late]), np.log(w[late]), 1)[0])
        out[f"p={p},q={q}"] = {"w2_final_mean": float(w[-1]), "slope_log_w2_last_decade": slope}
    attempts = float(L) * L * len(members) * times[-1]
    return {
        "metric": "site-update attempts/s, L=4096 growth runs (KPZ and EW, 8 seeds each)",
        "value": attempts / elapsed,
        "unit": "attempts/s",
        "seconds": elapsed,
        "members": len(members),
        "mcs": times[-1],
        "samples": len(times),
        "runs": out,
    }


def latency_leg(args):
    """The small workload: L = 64, p = 1, q = 0, seed 1, one 64 x 64 block
    (periodic, no dead border), 1000 MCS with the exact moments after every
    MCS.  Eager: each MCS is sweep(1) + roughness() (which waits for the
    result); per-MCS latency p50/p99.  Graph: the whole run (1000 sweeps and
    1000 samples) as one captured graph, through a one-member ensemble."""
    import numpy as np
    import torch
    import paper_1204_5072_amd as kpz

    L, n_mcs = 64, 1000
    sim = kpz.Sim(L, 1.0, 0.0, 1, (64, 64))
    sim.sweep(1)
    sim.roughness()
    lat = []
    for _ in range(n_mcs):
        t0 = time.perf_counter()
        sim.sweep(1)
        sim.roughness()
        lat.append((time.perf_counter() - t0) * 1e3)
    sim.close()
    ens = kpz.Ensemble([kpz.make_params(L, 1.0, 0.0, 1, (64, 64))])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, W2 = ens.run(list(range(1, n_mcs + 1)))
    graph_s = time.perf_counter() - t0
    ens.close()
    lat = np.array(lat)
    return {
        "metric": "per-MCS latency (sweep + exact W^2 on the host), L=64",
        "eager_p50_ms": float(np.percentile(lat, 50)),
        "eager_p99_ms": float(np.percentile(lat, 99)),
        "graph_run_ms": graph_s * 1e3,
        "graph_ms_per_mcs": graph_s * 1e3 / n_mcs,
        "mcs": n_mcs,
        "w2_final": float(W2[-1, 0]),
    }


def ring_leg(args, ceiling):
    """The 1+1-d ring (the rooftop reduction) at L = 2^30 sites (128 MiB of
    packed bonds), p = 1, q = 0, seed 1, default blocks: attempts/s over 20
    MCS timed with HIP events on the ring's stream, and its HBM roofline at
    0.25 B per attempt (each bond bit read and written once per MCS)."""
    import torch
    import paper_1204_5072_amd as kpz
    L, n = 1 << 30, 20
    r = kpz.Ring(L, 1.0, 0.0, 1)
    r.sweep(2)
    r.roughness()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(r.stream)
    r.sweep(n)
    e1.record(r.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / n
    m = r.roughness()
    block = int(r.params.block) or 128
    r.close()
    gbs = 0.25 * L / (ms * 1e-3) / 1e9
    valu = ring_valu_per_mcs()
    if valu is None or ceiling is None:
        roof = {"bound": "alu", "achieved": None,
                "peak": ceiling / 1e9 if ceiling else None,
                "unit": "G wave-instr/s", "frac": None,
                "note": "VALU count not measured for this source"}
    else:
        rate = valu / (ms * 1e-3)
        roof = {"bound": "alu", "achieved": rate / 1e9, "peak": ceiling / 1e9,
                "unit": "G wave-instr/s", "frac": rate / ceiling,
                "valu_wave_instr_per_mcs": valu}
    roof.update({"hbm_achieved_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
                 "bytes_per_attempt": 0.25})
    return {
        "metric": "site-update attempts/s, 1+1-d ring L=2^30",
        "value": L / (ms * 1e-3),
        "unit": "attempts/s",
        "ms_per_mcs": ms,
        "block": block,
        "roofline": roof,
        "w2_t22": m.W2,
    }


def code_sha256(names):
    """sha256 of the code of the named sources under paper_1204_5072_amd/csrc:
    comments (// to the line end, /* ... */) and blank lines removed, trailing
    blanks stripped, lines joined by newlines.  Counters taken on one code
    stay valid across comment edits; any change to the code invalidates
    them."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in names:
        text = open(os.path.join(ROOT, "paper_1204_5072_amd", "csrc", f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for line in text.splitlines():
            line = re.sub(r"//.*", "", line).rstrip()
            if line:
                h.update(line.encode() + b"\n")
    return h.hexdigest()


def ring_valu_per_mcs():
    """VALU wave instructions per ring MCS (sweep + merge launch) from the
    committed counter summary, or None when kpz_ring.hip or the device
    helpers changed since the counters were taken."""
    import re
    path = os.path.join(ROOT, "profiles", "kpz_ring_L2p30_kernel_trace.md")
    try:
        text = open(path).read()
        sha = code_sha256(("kpz_ring.hip", "kpz_device.h"))
    except OSError:
        return None
    m = re.search(r"code_sha256 = ([0-9a-f]{64})", text)
    if not m or m.group(1) != sha:
        return None
    m = re.search(r"valu_wave_instr_per_mcs = (\d+)", text)
    return float(m.group(1)) if m else None


def kmc_leg(args):
    """The paper's KMC quench benchmark configuration: fcc lattice of
    512^3/2 sites, c = 0.325, eps = 1.5, 32^3 device-layer blocks: attempts/s
    over 20 MCS timed with HIP events on the simulation's stream, plus the
    oracle's random-sequential dynamics on a 128^3/2 sample for scale."""
    import time
    import torch
    import paper_1204_5072_amd as kpz
    L, n = 512, 20
    sim = kpz.Kmc(L, c=0.325, eps=1.5, seed=1, block=32)
    nb0, bonds0 = sim.counts()
    sim.sweep(2)
    torch.cuda.synchronize()
    t0, m0 = sim.state()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.sweep(n)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / n
    t1, m1 = sim.state()
    nb1, bonds1 = sim.counts()
    sim.close()
    N = L ** 3 // 2
    out = {
        "metric": "update attempts/s, KMC binary alloy fcc 512^3/2, c=0.325, eps=1.5",
        "value": N / (ms * 1e-3),
        "unit": "attempts/s",
        "ms_per_mcs": ms,
        "launches_per_mcs": 8,
        "block": 32,
        "accepted_per_attempt": (m1 - m0) / (N * n),
        "bonds_initial": bonds0,
        "bonds_final": bonds1,
        "n_b": nb1,
        "t_final": t1,
    }
    if not args.no_cpu_baseline:
        from oracle import kmc as okmc
        occ = okmc.init(128, 0.325, 1)
        t = time.perf_counter()
        okmc.rs_run(occ, 1.5, 1, 0, 2)
        dt = time.perf_counter() - t
        out["cpu_oracle_rs"] = {"value": 2 * 128 ** 3 // 2 / dt, "unit": "attempts/s", "cores": 1,
                                "kind": "oracle", "sample": "random-sequential, 128^3/2 sites, 2 MCS"}
    return out


def serving_leg(args):
    """Serving: a Poisson stream of jobs (2000 at 50 jobs/s by default), L =
    64 round(2^U / 64) with U uniform on [8, 13], p = 1, q uniform on [0, 0.5],
    MCS log-uniform on 10^2..10^4, admitted into a device job pool by HBM
    budget and run with continuous batching; p50/p99 of arrival -> result
    latency.  Two shorter streams report the latencies at half that rate
    (below the pool's capacity) and at a rate above it."""
    from paper_1204_5072_amd import serve

    def run(n_jobs, rate):
        jobs = serve.poisson_jobs(n_jobs=n_jobs, rate=rate, seed=0)

        def progress(done, total, resident):
            print(f"bench: serving {done}/{total} done, {resident} resident", file=sys.stderr,
                  flush=True)

        kw = {"block": tuple(args.serve_block)} if args.serve_block else {}
        rep = serve.serve(jobs, hbm_bytes=int(args.serve_hbm_gib * (1 << 30)),
                          quantum=args.serve_quantum, progress=progress, **kw)
        return {
            "p50_ms": rep.latency_p50_ms,
            "p99_ms": rep.latency_p99_ms,
            "max_ms": rep.latency_max_ms,
            "throughput_attempts_per_s": rep.attempts_per_s,
            "jobs": rep.jobs,
            "rate_jobs_per_s": rate,
            "seconds": rep.seconds,
            "offered_attempts_per_s": rep.attempts / max(j.arrival for j in jobs),
            "steps": rep.steps,
            "max_resident_jobs": rep.max_resident,
        }

    out = {"metric": "job latency p50/p99 (arrival -> result), serving",
           "sizes": "L = 64 round(2^U / 64), U ~ U(8, 13)",
           "hbm_budget_gib": args.serve_hbm_gib, "quantum_mcs": args.serve_quantum}
    out.update(run(args.serve_jobs, args.serve_rate))
    if args.serve_low_jobs > 0:
        out["below_saturation"] = run(args.serve_low_jobs, args.serve_low_rate)
    if args.serve_sat_jobs > 0:
        out["saturated"] = run(args.serve_sat_jobs, args.serve_sat_rate)
    return out


def sweep_counters(block, in_place=False, device_dt=False):
    """(HBM bytes per MCS, VALU wave instructions per MCS) of this block shape
    and mode from the committed hardware-counter summary, each None when the
    sweep's source (kpz.hip and the device headers it includes) has changed
    since the counters were taken or the shape was not measured."""
    import re
    path = os.path.join(ROOT, "profiles", "kpz_sweep_L65536_hbm_counters.md")
    try:
        text = open(path).read()
        sha = code_sha256(("kpz.hip", "kpz_slice.h", "kpz_device.h"))
    except OSError:
        return None, None
    m = re.search(r"code_sha256 = ([0-9a-f]{64})", text)
    if not m or m.group(1) != sha:
        return None, None
    key = "%dx%d%s" % (block[0], block[1],
                       ",device_dt" if device_dt else (",in_place" if in_place else ""))
    out = []
    for name in ("traffic_bytes_per_mcs", "valu_wave_instr_per_mcs"):
        m = re.search(r"%s\[%s\] = (\d+)" % (name, re.escape(key)), text)
        out.append(float(m.group(1)) if m else None)
    return tuple(out)


def copy_probe(mib: int) -> None:
    """A plain copy of known size (mib MiB read, mib MiB written per call):
    hardware byte counters read on it give the scale between the counters'
    units and bytes."""
    import torch
    n = mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n, "calls": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--L", type=int, default=65536)
    ap.add_argument("--block", type=int, nargs=2, default=None,
                    help="block shape (default 1024 x 32, the fastest shape at L = 2^16 for "
                         "dead borders and for --device-dt, whose 256-byte block rows leave "
                         "fewest cache lines shared with idle blocks)")
    ap.add_argument("--mcs-per-step", type=int, default=10)
    ap.add_argument("--p", type=float, default=1.0)
    ap.add_argument("--q", type=float, default=0.0)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--device-dt", action="store_true",
                    help="double tiling at the device layer instead of dead borders")
    ap.add_argument("--dt-ahead", action="store_true",
                    help="device-layer double tiling with a set and its diagonal partner "
                         "sharing a launch where they follow each other (implies --device-dt)")
    ap.add_argument("--in-place", action="store_true",
                    help="update the lattice in place (no second lattice buffer)")
    ap.add_argument("--moves", type=int, default=1,
                    help="dead-border origin moves per MCS (block residency 1/moves MCS)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--ens-members", type=int, default=512)
    ap.add_argument("--ens-mcs", type=int, default=10_000)
    ap.add_argument("--ens-block", type=int, nargs=2, default=None)
    ap.add_argument("--ens-autotune", action="store_true",
                    help="tune the ensemble's block shape per L instead of the recorded table")
    ap.add_argument("--ens-seq-members", type=int, default=32)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-low-jobs", type=int, default=500)
    ap.add_argument("--serve-low-rate", type=float, default=25.0)
    ap.add_argument("--serve-sat-jobs", type=int, default=400)
    ap.add_argument("--serve-sat-rate", type=float, default=200.0)
    ap.add_argument("--no-latency", action="store_true")
    ap.add_argument("--no-growth", action="store_true")
    ap.add_argument("--growth-mcs", type=int, default=10_000)
    ap.add_argument("--no-ring", action="store_true")
    ap.add_argument("--no-kmc", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=2000)
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--serve-hbm-gib", type=float, default=16.0)
    ap.add_argument("--serve-quantum", type=int, default=64)
    ap.add_argument("--serve-block", type=int, nargs=2, default=None,
                    help="common block shape of the job pool (default: the pool's own)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (3 times) "
                         "and exit: the known-size reference for HBM byte counters")
    args = ap.parse_args()
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on exactly one GPU (one lattice per device); "
              "--gpus N with N > 1 is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1204_5072_amd as kpz

    L, M = args.L, args.mcs_per_step
    args.device_dt = args.device_dt or args.dt_ahead
    block = tuple(args.block) if args.block else (1024, 32)
    print(f"bench: L={L} block={block} p={args.p} q={args.q} seed={args.seed} "
          f"steps={args.steps} warmup={args.warmup} mcs/step={M}", file=sys.stderr, flush=True)
    sim = kpz.Sim(L, args.p, args.q, args.seed, block, moves=args.moves, in_place=args.in_place,
                  device_dt=args.device_dt or args.dt_ahead, dt_ahead=args.dt_ahead)
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
    achieved_gbs = BYTES_PER_ATTEMPT * per_launch_attempts / sweep_s / 1e9
    traffic, valu = (sweep_counters(block, args.in_place, args.device_dt)
                     if (L == 65536 and args.moves == 1 and not args.dt_ahead) else (None, None))
    ceiling = valu_ceiling()
    valu_rate = valu / sweep_s if valu else None
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
            "origin_moves_per_mcs": args.moves,
            "lattice_buffers": 1 if (args.in_place or args.device_dt) else 2,
            "device_layer": "double tiling" if args.device_dt else "dead border",
        },
        "roofline": {
            # bound by vector-ALU issue: the kernel's VALU wave instructions per
            # launch (rocprofv3 SQ_INSTS_VALU, committed summary of this code)
            # over the mean launch time, against the issue rate kpz_valu_probe
            # measures on this device for the same instruction mix
            "bound": "alu",
            "achieved": valu_rate / 1e9 if valu_rate else None,
            "peak": ceiling / 1e9 if ceiling else None,
            "unit": "G wave-instr/s",
            "frac": valu_rate / ceiling if (valu_rate and ceiling) else None,
            "traffic": traffic,
            "traffic_unit": "HBM bytes per MCS (all launches of one MCS; rocprofv3 FETCH_SIZE "
                            "and WRITE_SIZE scaled by a 1 GiB copy probe)",
            # one MCS = one sweep launch (two-buffer mode), or the sweep launch
            # plus the straddling-word merge launch (in place), bracketed
            # together by the events
            "kernel": ("kpz_dt_kernel, 2-4 launches per MCS" if args.dt_ahead else
                       "kpz_dt_kernel x4 phases" if args.device_dt else
                       "kpz_sweep_kernel+kpz_merge_kernel" if args.in_place else "kpz_sweep_kernel"),
            "mean_launch_ms": sweep_ms,
            "valu_wave_instr_per_launch": valu,
            "hbm": {"achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved_gbs / HBM_PEAK_GBS, "bytes_per_attempt": BYTES_PER_ATTEMPT},
        },
        "roughness_ms": rough_ms,
        "w2_last": w2[-1] if w2 else None,
        "t_final": sim.state()[0],
    }
    # after the timed region: the final surface must satisfy the slope
    # constraints everywhere (open plaquettes, row-0 and column-0 sums)
    line["final_surface_check"] = dict(zip(("open_plaquettes", "row0_sum", "col0_sum"),
                                           sim.check_invariants()))
    sim.close()
    del sim
    if not args.no_ensemble:
        print("bench: ensemble leg", file=sys.stderr, flush=True)
        line["ensemble"] = ensemble_leg(args)
    if not args.no_growth:
        print("bench: growth leg", file=sys.stderr, flush=True)
        line["growth"] = growth_leg(args)
    if not args.no_latency:
        print("bench: latency leg", file=sys.stderr, flush=True)
        line["latency"] = latency_leg(args)
    if not args.no_ring:
        print("bench: ring leg", file=sys.stderr, flush=True)
        line["ring"] = ring_leg(args, ceiling)
    if not args.no_kmc:
        print("bench: kmc leg", file=sys.stderr, flush=True)
        line["kmc"] = kmc_leg(args)
    if not args.no_serve:
        print("bench: serving leg", file=sys.stderr, flush=True)
        line["serving"] = serving_leg(args)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(block, args.p, args.q, args.seed, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
