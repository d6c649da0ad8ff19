"""Statistical agreement of the decomposed schedule with random-sequential
dynamics (Sec. 3: the decomposition deviates from the original model only at
domain boundaries; Sec. 3.1: single-hit updates with small cells).

W^2(t) is averaged over 64 independent seeds per schedule at L = 256, and
every comparison is stated with its standard error:

* the GPU's decomposed schedule against the CPU oracle's decomposed schedule
  with other seeds (two samples of one distribution): per-time z-scores
  within +-4 (seven times, so a false alarm has probability below 1e-3);
* the schedule against random-sequential dynamics: the per-time amplitude
  offset rel(t) = <W^2>_DD / <W^2>_RS - 1 and its standard error are
  reported; the offset is a property of the schedule, measured on the
  oracle with many seeds (tests/test_oracle_schedule_bias.py: -3.4 to -6 %
  with 4 x 4 tiles, about 60 % of it from the exact per-tile attempt count),
  and the test states the band -8 % < rel(t) < +3 sigma; the growth exponent
  fitted on t = 8..64 agrees within 0.03;
* a schedule with 1x1 cells (every step a deterministic sublattice sweep),
  run on the oracle, fails grossly (W^2 off by more than 30 %).
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


AMPLITUDE_BAND = -0.08
BETA_TOL = 0.03
Z_MAX = 4.0


def _rel_err(a, b):
    """Offset <a>/<b> - 1 per time and its standard error (independent
    samples a, b of shape (seeds, times))."""
    ma, mb = a.mean(axis=0), b.mean(axis=0)
    ea = a.std(axis=0, ddof=1) / np.sqrt(len(a))
    eb = b.std(axis=0, ddof=1) / np.sqrt(len(b))
    return ma / mb - 1.0, np.sqrt((ea / mb) ** 2 + (ma * eb / mb ** 2) ** 2)


def _z(a, b):
    ea = a.std(axis=0, ddof=1) / np.sqrt(len(a))
    eb = b.std(axis=0, ddof=1) / np.sqrt(len(b))
    return (a.mean(axis=0) - b.mean(axis=0)) / np.sqrt(ea ** 2 + eb ** 2)


def _rel(a, b):
    return a.mean(axis=0) / b.mean(axis=0) - 1.0


def _beta(w):
    sel = [i for i, t in enumerate(TIMES) if 8 <= t <= 64]
    return np.polyfit(np.log([TIMES[i] for i in sel]), np.log(w.mean(axis=0)[sel]), 1)[0] / 2


def _agrees(dd, rs):
    rel, err = _rel_err(dd, rs)
    ok = bool(np.all(rel > AMPLITUDE_BAND) and np.all(rel < 3 * err)
              and abs(_beta(dd) - _beta(rs)) < BETA_TOL)
    return ok, rel, err


def _dd_w2_oracle_par(oracle_lib, L, p, q, seeds, block, moves=1):
    import os
    out = np.zeros((len(seeds), len(TIMES)))
    for i, seed in enumerate(seeds):
        st = oracle_lib.SlopeState(L)
        for k, T in enumerate(TIMES):
            st.run_dd(T - st.t, p, q, seed, block=block, moves=moves,
                      threads=min(16, os.cpu_count() or 1))
            S1, S2 = st.moments()
            out[i, k] = oracle_lib.w2(S1, S2, L * L)
    return out


@pytest.fixture(scope="module")
def rs_reference(oracle_lib):
    return _rs_w2(oracle_lib, 256, 1.0, 0.0, range(64))


def _gpu_w2(kpz, L, seeds, block, moves=1):
    dd = np.zeros((len(seeds), len(TIMES)))
    sims = [kpz.Sim(L, 1.0, 0.0, s, block, moves=moves) for s in seeds]
    t = 0
    for k, T in enumerate(TIMES):
        for sim in sims:
            sim.sweep(T - t)
        for i, sim in enumerate(sims):
            dd[i, k] = sim.roughness().W2
        t = T
    for sim in sims:
        sim.close()
    return dd


@pytest.mark.gpu
@pytest.mark.parametrize("block", [(256, 128), (128, 128), (64, 64)])
def test_gpu_dd_agrees_with_rs(oracle_lib, rs_reference, block):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1204_5072_amd as kpz
    L = 256
    dd = _gpu_w2(kpz, L, [90_000 + s for s in range(64)], block)
    cpu = _dd_w2_oracle_par(oracle_lib, L, 1.0, 0.0, [190_000 + s for s in range(64)], block)
    z = _z(dd, cpu)
    ok, rel, err = _agrees(dd, rs_reference)
    print("block", block, "GPU vs oracle schedule z", np.round(z, 2),
          "| offset to RS %", np.round(100 * rel, 2), "+-", np.round(100 * err, 2),
          "| beta", round(_beta(dd), 4), round(_beta(rs_reference), 4), flush=True)
    assert np.all(np.abs(z) < Z_MAX), z
    assert ok, (rel, err, _beta(dd), _beta(rs_reference))


@pytest.mark.gpu
@pytest.mark.parametrize("moves", [4, 16])
def test_gpu_dd_origin_moves_agree_with_rs(oracle_lib, rs_reference, moves):
    """Block residency below one MCS (the origin moved 4 or 16 times per
    MCS): the same statements; the printed offset is the fidelity figure for
    that residency (on the oracle it is slightly larger than with one move
    per MCS, not smaller)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1204_5072_amd as kpz
    L, block = 256, (64, 64)
    dd = _gpu_w2(kpz, L, [95_000 + s for s in range(64)], block, moves=moves)
    cpu = _dd_w2_oracle_par(oracle_lib, L, 1.0, 0.0, [195_000 + s for s in range(64)], block,
                            moves=moves)
    z = _z(dd, cpu)
    ok, rel, err = _agrees(dd, rs_reference)
    print("moves", moves, "GPU vs oracle schedule z", np.round(z, 2),
          "| offset to RS %", np.round(100 * rel, 2), "+-", np.round(100 * err, 2),
          "| beta", round(_beta(dd), 4), round(_beta(rs_reference), 4), flush=True)
    assert np.all(np.abs(z) < Z_MAX), z
    assert ok, (rel, err, _beta(dd), _beta(rs_reference))


def test_checkerboard_like_cells_fail(oracle_lib):
    """Negative control on the CPU: 1x1 cells (2x2 tiles) bias W^2(t)."""
    L = 64
    rs = _rs_w2(oracle_lib, L, 1.0, 0.0, range(48))
    bad = _dd_w2_oracle(oracle_lib, L, 1.0, 0.0, range(48), (L, L), (2, 2))
    good = _dd_w2_oracle(oracle_lib, L, 1.0, 0.0, range(48), (L, L), (4, 4))
    ok, rel, err = _agrees(good, rs)
    assert ok, (rel, err, _beta(good), _beta(rs))
    rel_bad = _rel(bad, rs)
    assert np.min(rel_bad[[i for i, t in enumerate(TIMES) if t >= 16]]) < -0.3, rel_bad
