"""Host logic (no GPU): the serving loop's job stream (sizes, rates and the
mean work per job of the two lattice-size distributions) and the
autotuner's choice among near-tied block shapes."""
import numpy as np
import pytest

from paper_1204_5072_amd import serve


def test_multiple64_sizes():
    jobs = serve.poisson_jobs(n_jobs=20000, rate=50.0, seed=0)
    Ls = np.array([j.L for j in jobs])
    assert np.all(Ls % 64 == 0) and Ls.min() >= 256 and Ls.max() <= 8192
    assert np.mean(Ls & (Ls - 1) != 0) > 0.5          # mostly not powers of two
    # log-uniform on [2^8, 2^13]: E[L^2] = (2^26 - 2^16) / (5 * 2 ln 2)
    e_l2 = (2.0 ** 26 - 2.0 ** 16) / (5 * 2 * np.log(2))
    assert abs(np.mean(Ls.astype(float) ** 2) / e_l2 - 1) < 0.05
    # MCS log-uniform on [10^2, 10^4]: E = (10^4 - 10^2) / (2 ln 10)
    mcs = np.array([j.n_mcs for j in jobs])
    assert abs(mcs.mean() / (9900 / (2 * np.log(10))) - 1) < 0.05
    gaps = np.diff([j.arrival for j in jobs])
    assert abs(gaps.mean() * 50.0 - 1) < 0.03
    assert all(j.p == 1.0 and 0.0 <= j.q <= 0.5 and j.seed == i for i, j in enumerate(jobs))


def test_pow2_sizes():
    jobs = serve.poisson_jobs(n_jobs=3000, seed=1, sizes="pow2")
    Ls = np.array([j.L for j in jobs])
    assert set(Ls.tolist()) == {2 ** k for k in range(8, 14)}


def test_unknown_size_distribution():
    with pytest.raises(ValueError):
        serve.poisson_jobs(n_jobs=3, sizes="square")


def test_autotune_pick_breaks_near_ties_by_candidate_order():
    from paper_1204_5072_amd.autotune import pick
    t = {(128, 256): 1.02, (256, 128): 1.00, (512, 64): 1.01}
    assert pick(t) == (128, 256)                    # within 3 % of the fastest: first wins
    t = {(128, 256): 1.10, (256, 128): 1.00, (512, 64): 1.01}
    assert pick(t) == (256, 128)
