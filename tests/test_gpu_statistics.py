"""Statistical agreement of the decomposed schedule with random-sequential
dynamics (Sec. 3: the decomposition deviates from the original model only at
domain boundaries; Sec. 3.1: single-hit updates make that error negligible).

W^2(t) from the GPU's decomposed schedule, averaged over independent seeds,
must match the oracle's true random-sequential W^2(t) within the combined
standard errors; a schedule with 1x1 cells (deterministic sublattice sweeps),
run on the oracle, must fail the same comparison.
"""
import numpy as np
import pytest

TIMES = [1, 2, 4, 8, 16, 32, 64]


def _rs_w2(oracle_lib, L, p, q, seeds):
    out = np.zeros((len(seeds), len(TIMES)))
    for i, seed in enumerate(seeds):
        h = oracle_lib.flat_heights(L)
        t = 0
        for k, T in enumerate(TIMES):
            h = oracle_lib.rs_heights_run(h, t, T - t, p, q, 50_000 + seed)
            t = T
            S1, S2 = oracle_lib.moments(h)
            out[i, k] = oracle_lib.w2(S1, S2, L * L)
    return out


def _dd_w2_oracle(oracle_lib, L, p, q, seeds, block, tile):
    out = np.zeros((len(seeds), len(TIMES)))
    for i, seed in enumerate(seeds):
        st = oracle_lib.SlopeState(L)
        for k, T in enumerate(TIMES):
            st.run_dd(T - st.t, p, q, 70_000 + seed, block=block, tile=tile)
            S1, S2 = st.moments()
            out[i, k] = oracle_lib.w2(S1, S2, L * L)
    return out


def _z(a, b):
    se = np.sqrt(a.var(axis=0, ddof=1) / len(a) + b.var(axis=0, ddof=1) / len(b))
    return (a.mean(axis=0) - b.mean(axis=0)) / se


@pytest.fixture(scope="module")
def rs_reference(oracle_lib):
    return _rs_w2(oracle_lib, 256, 1.0, 0.0, range(64))


@pytest.mark.gpu
@pytest.mark.parametrize("block", [(256, 256), (128, 128), (64, 64)])
def test_gpu_dd_agrees_with_rs(oracle_lib, rs_reference, block):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1204_5072_amd as kpz
    L = 256
    dd = np.zeros((64, len(TIMES)))
    sims = [kpz.Sim(L, 1.0, 0.0, 90_000 + s, block) for s in range(64)]
    t = 0
    for k, T in enumerate(TIMES):
        for sim in sims:
            sim.sweep(T - t)
        for i, sim in enumerate(sims):
            dd[i, k] = sim.roughness().W2
        t = T
    z = _z(dd, rs_reference)
    print("z-scores", block, np.round(z, 2), flush=True)
    assert np.all(np.abs(z) < 4.0), z


def test_checkerboard_like_cells_fail(oracle_lib):
    """Negative control on the CPU: 1x1 cells (2x2 tiles) bias W^2(t)."""
    L = 64
    rs = _rs_w2(oracle_lib, L, 1.0, 0.0, range(48))
    bad = _dd_w2_oracle(oracle_lib, L, 1.0, 0.0, range(48), (L, L), (2, 2))
    good = _dd_w2_oracle(oracle_lib, L, 1.0, 0.0, range(48), (L, L), (4, 4))
    assert np.max(np.abs(_z(bad, rs))) > 6.0
    assert np.all(np.abs(_z(good, rs)) < 4.0), _z(good, rs)
