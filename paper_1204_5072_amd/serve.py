"""Serving loop: simulation jobs arrive over time, are admitted into a
device job pool by HBM budget, run with continuous batching, and leave with
their exact final W^2.  Reports p50/p99 job latency (arrival -> result) and
throughput."""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import POOL_BLOCK, Pool, make_params


@dataclass
class Job:
    arrival: float       # seconds after the start of the run
    L: int
    p: float
    q: float
    seed: int
    n_mcs: int
    jid: Optional[int] = None
    admitted: Optional[float] = None
    finished: Optional[float] = None
    result: object = None


def poisson_jobs(n_jobs: int = 2000, rate: float = 50.0, seed: int = 0,
                 log2L=(8, 13), log10_mcs=(2.0, 4.0), q_max: float = 0.5,
                 sizes: str = "multiple64") -> List[Job]:
    """Poisson arrivals (exponential gaps, mean 1/rate); MCS = round(10^U), U
    uniform on log10_mcs; p = 1, q uniform on [0, q_max]; seed = job number.
    Lattice sizes, log-uniform between 2^log2L[0] and 2^log2L[1]:
      "multiple64": L = 64 round(2^U / 64), U uniform on log2L (sizes that
                    are not powers of two run with the largest power-of-two
                    blocks dividing them);
      "pow2":       L = 2^k, k uniform on the integers of log2L."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_jobs)
    arrivals = np.cumsum(gaps) - gaps[0]
    if sizes == "pow2":
        Ls = 2 ** rng.integers(log2L[0], log2L[1] + 1, size=n_jobs)
    elif sizes == "multiple64":
        Ls = 64 * np.maximum(1, np.round(2.0 ** rng.uniform(log2L[0], log2L[1], size=n_jobs) / 64))
    else:
        raise ValueError(f"unknown size distribution {sizes!r}")
    mcs = np.round(10.0 ** rng.uniform(log10_mcs[0], log10_mcs[1], size=n_jobs)).astype(int)
    qs = rng.uniform(0.0, q_max, size=n_jobs)
    return [Job(float(arrivals[i]), int(Ls[i]), 1.0, float(qs[i]), i, int(mcs[i]))
            for i in range(n_jobs)]


@dataclass
class ServeReport:
    jobs: int
    seconds: float
    attempts: float
    latency_p50_ms: float
    latency_p99_ms: float
    latency_max_ms: float
    steps: int
    max_resident: int
    extra: Dict = field(default_factory=dict)

    @property
    def attempts_per_s(self) -> float:
        return self.attempts / self.seconds


def serve(jobs: List[Job], hbm_bytes: int, quantum: int = 64, block=POOL_BLOCK,
          max_jobs: int = 1024, clock=time.perf_counter, progress=None,
          progress_every_s: float = 10.0) -> ServeReport:
    """Runs the jobs in real time: a job becomes visible at its arrival time,
    waits FIFO until it fits into the pool, and is done when its result is
    back on the host.  ``progress(done, total, resident)`` is called about
    every ``progress_every_s`` seconds when given."""
    pool = Pool(hbm_bytes, max_jobs=max_jobs, max_quantum=quantum, block=block)
    pending = deque(sorted(jobs, key=lambda j: j.arrival))
    waiting: deque = deque()
    by_id: Dict[int, Job] = {}
    t0 = clock()
    steps = 0
    resident = 0
    max_resident = 0
    done = 0
    next_report = progress_every_s
    while done < len(jobs):
        now = clock() - t0
        if progress is not None and now >= next_report:
            progress(done, len(jobs), resident)
            next_report = now + progress_every_s
        while pending and pending[0].arrival <= now:
            waiting.append(pending.popleft())
        while waiting:
            j = waiting[0]
            jid = pool.submit(make_params(j.L, j.p, j.q, j.seed, block), j.n_mcs)
            if jid is None:
                break
            j.jid, j.admitted = jid, clock() - t0
            by_id[jid] = j
            waiting.popleft()
            resident += 1
        if resident == 0:
            # idle until the next arrival
            if pending:
                delay = pending[0].arrival - (clock() - t0)
                if delay > 0:
                    time.sleep(min(delay, 0.01))
            continue
        max_resident = max(max_resident, resident)
        resident = pool.step(quantum)
        steps += 1
        now = clock() - t0
        for jid, mom in pool.poll():
            j = by_id.pop(jid)
            j.finished, j.result = now, mom
            done += 1
        if pool.failures:
            bad = list(pool.failures)
            pool.close()
            raise RuntimeError(f"serving: {len(bad)} job(s) failed (job id, kpz_status): {bad[:8]}")
    seconds = clock() - t0
    pool.close()
    lat = np.array([(j.finished - j.arrival) * 1e3 for j in jobs])
    attempts = float(sum(j.L * j.L * j.n_mcs for j in jobs))
    return ServeReport(len(jobs), seconds, attempts, float(np.percentile(lat, 50)),
                       float(np.percentile(lat, 99)), float(lat.max()), steps, max_resident)
