"""Writes l4096_seed1.json: the L = 4096 workload (flat start, seed 1, 256 x 128
dead-border blocks, 4 x 4 tiles) for p = 1, q = 0 and p = q = 1/2, run by the
CPU oracle's block-parallel runner to t = 1000 and t = 10^4 MCS.  Stored per
checkpoint: sha256 of the packed slope words (uint32, little-endian, the
documented layout), the exact S1 = sum h and S2 = sum h^2 (as decimal
strings), h(0, 0) and the net flip count.  Calls only the oracle.

    python tests/golden/make_l4096_seed1.py [threads]
"""
import hashlib
import json
import os
import sys

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))

import numpy as np  # noqa: E402

import oracle  # noqa: E402

L, SEED, BLOCK = 4096, 1, (256, 128)
CHECKPOINTS = (1000, 10_000)


def state_record(st, t):
    words = oracle.pack(st.sx, st.sy).astype("<u4")
    S1, S2 = st.moments()
    return {"t": t, "words_sha256": hashlib.sha256(words.tobytes()).hexdigest(),
            "S1": str(int(S1)), "S2": str(int(S2)), "h00": int(st.h00[0]),
            "net": int(st.net[0])}


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    runs = []
    out = {"L": L, "seed": SEED, "block": list(BLOCK), "tile": [4, 4], "runs": runs,
           "written_by": "tests/golden/make_l4096_seed1.py (CPU oracle only)"}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "l4096_seed1.json")
    for p, q in ((1.0, 0.0), (0.5, 0.5)):
        st = oracle.SlopeState(L)
        recs, t = [], 0
        runs.append({"p": p, "q": q, "checkpoints": recs})
        for c in CHECKPOINTS:
            st.run_dd(c - t, p, q, SEED, block=BLOCK, threads=threads)
            t = c
            recs.append(state_record(st, t))
            with open(path, "w") as f:   # rewritten after every checkpoint
                json.dump(out, f, indent=1)
            print(f"p={p} q={q} t={t} written", flush=True)


if __name__ == "__main__":
    main()
