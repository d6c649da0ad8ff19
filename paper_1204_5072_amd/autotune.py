"""Block-shape autotuner for the sweep.

The dead-border block shape (the device layer of the decomposition) is a
free parameter of the method: any valid shape gives a correct decomposed
schedule, but the shape changes the sequence of updates, so the chosen shape
is returned and must be recorded with the results (runs are reproducible for
identical parameters and shape only).  The tuner times each candidate with
HIP events on the device and keeps the fastest, counting shapes within a few
per cent of it as ties (the first in a fixed order wins, so that timing noise
does not change the dynamics between runs); the launch shape (threads per
block) is chosen by the library and does not affect results.
"""
from __future__ import annotations

from typing import Dict, Iterable, List, Optional, Sequence, Tuple

from . import Ensemble, KPZError, Sim, make_params, workspace_bytes

# Candidate shapes (block_x, block_y): one wave per block, so the full
# shapes hold 64 lanes of (row group of 128 sites, tile row): 128 x 256,
# 256 x 128, 512 x 64; the half and quarter shapes keep the dead-border
# fraction 1/Bx + 1/By at or below about 3 %.
CANDIDATES: Tuple[Tuple[int, int], ...] = (
    (128, 256), (256, 128), (512, 64), (128, 128), (256, 64), (512, 32), (64, 256),
    (128, 64), (64, 64), (1024, 32), (1024, 16),
)


def valid_shapes(L: int, candidates: Iterable[Tuple[int, int]] = CANDIDATES) -> List[Tuple[int, int]]:
    out = []
    for bx, by in candidates:
        if L % bx or L % by:
            continue
        try:
            workspace_bytes(make_params(L, 1.0, 0.0, 1, (bx, by)))
        except KPZError:
            continue
        out.append((bx, by))
    return out


# Shapes whose times lie within this fraction of the fastest count as ties;
# the first of them in CANDIDATES order is chosen, so that run-to-run timing
# noise of a few per cent does not change the chosen shape (and with it the
# dynamics) from one run to the next.
TIE = 0.03


def pick(timings: Dict[Tuple[int, int], float]) -> Tuple[int, int]:
    """The first shape, in the order of `timings` (candidate order), whose
    time is within TIE of the fastest."""
    best = min(timings.values())
    return next(s for s, t in timings.items() if t <= best * (1.0 + TIE))


def _time(fn, reps: int, trials: int = 3) -> float:
    """Median over `trials` of the mean time of `reps` calls of fn (ms)."""
    import torch
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()                      # warm-up (first launch of this kernel variant)
    torch.cuda.synchronize()
    out = []
    for _ in range(trials):
        start.record()
        for _ in range(reps):
            fn()
        stop.record()
        torch.cuda.synchronize()
        out.append(start.elapsed_time(stop) / reps)
    return sorted(out)[len(out) // 2]


def tune_lattice(L: int, p: float = 1.0, q: float = 0.0, mcs: int = 2,
                 candidates: Optional[Sequence[Tuple[int, int]]] = None,
                 verbose: bool = False) -> Dict:
    """Fastest block shape for one lattice of size L; returns
    {"block": (bx, by), "ms_per_mcs": {shape: ms}}."""
    shapes = valid_shapes(L, candidates or CANDIDATES)
    if not shapes:
        raise ValueError(f"no valid block shape for L={L}")
    timings, failed = {}, {}
    for shape in shapes:
        try:
            sim = Sim(L, p, q, 12345, shape)
        except KPZError as e:          # recorded, not fatal: other shapes may run
            failed[shape] = str(e)
            continue
        timings[shape] = _time(lambda: sim.sweep(mcs), 1) / mcs
        sim.close()
        del sim
        if verbose:
            print(f"autotune: {shape[0]}x{shape[1]} {timings[shape]:.3f} ms/MCS", flush=True)
    if not timings:
        raise RuntimeError(f"no block shape ran for L={L}: {failed}")
    return {"block": pick(timings), "ms_per_mcs": timings, "failed": failed}


def tune_ensemble(members, mcs: int = 4,
                  candidates: Optional[Sequence[Tuple[int, int]]] = None) -> Dict:
    """Fastest block shape for each lattice size of an ensemble (list of
    kpz_params with block 0): for every distinct L the members of that size
    run as one ensemble with each candidate shape (median of three timings
    of `mcs` MCS).  Returns {"blocks": {L: (bx, by)}, "ms_per_mcs": {L:
    {shape: ms}}}; every member then runs the shape chosen for its L."""
    by_L: Dict[int, list] = {}
    for m in members:
        by_L.setdefault(int(m.L), []).append(m)
    blocks, timings = {}, {}
    for L, group in sorted(by_L.items()):
        shapes = valid_shapes(L, candidates or CANDIDATES)
        if not shapes:
            raise ValueError(f"no valid block shape for L={L}")
        t = {}
        for shape in shapes:
            ens = Ensemble([make_params(m.L, m.p, m.q, m.seed, shape) for m in group])
            t[shape] = _time(lambda: ens.sweep(mcs), 1) / mcs
            ens.close()
            del ens
        blocks[L] = pick(t)
        timings[L] = t
    return {"blocks": blocks, "ms_per_mcs": timings}


def main(argv=None) -> None:
    import argparse
    import json
    ap = argparse.ArgumentParser(description="time the sweep for each candidate block shape")
    ap.add_argument("--L", type=int, default=65536)
    ap.add_argument("--p", type=float, default=1.0)
    ap.add_argument("--q", type=float, default=0.0)
    ap.add_argument("--mcs", type=int, default=5)
    args = ap.parse_args(argv)
    res = tune_lattice(args.L, args.p, args.q, args.mcs, verbose=True)
    rows = {f"{s[0]}x{s[1]}": {"ms_per_mcs": ms, "attempts_per_s": args.L * args.L / ms * 1e3}
            for s, ms in sorted(res["ms_per_mcs"].items(), key=lambda kv: kv[1])}
    print(json.dumps({"L": args.L, "p": args.p, "q": args.q, "best": list(res["block"]),
                      "shapes": rows,
                      "failed": {f"{s[0]}x{s[1]}": m for s, m in res["failed"].items()}}),
          flush=True)


if __name__ == "__main__":
    main()
