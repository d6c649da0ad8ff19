"""The block-parallel runner of the decomposed schedule equals the plain
step-by-step runner (blocks of one residency never touch each other's
slopes, Sec. 3), and the 32-level acceptance uniform reproduces the exact
law with thresholds that need every level (Sec. 2.1 eq. ``rule`` with
generic p, q).  CPU only."""
import numpy as np
import pytest

from oracle import exact_small

CASES = [
    # L, block, p, q, seed, n, moves
    (64, (32, 16), 1.0, 0.0, 1, 3, 1),
    (64, (64, 64), 1.0, 0.25, 2, 3, 1),       # one periodic block
    (64, (16, 64), 0.7, 0.3, 3, 2, 1),        # one block along y
    (64, (64, 16), 0.5, 0.5, 4, 2, 2),        # one block along x, two residencies
    (48, (16, 16), 1.0, 0.0, 5, 3, 1),        # non-power-of-two L
    (128, (128, 32), 0.3, 0.9, 6, 2, 16),
    (96, (32, 32), 1.0, 0.999999, 7, 2, 4),
]


@pytest.mark.parametrize("L,block,p,q,seed,n,moves", CASES)
def test_parallel_runner_equals_plain(oracle_lib, L, block, p, q, seed, n, moves):
    a = oracle_lib.SlopeState(L).run_dd(n, p, q, seed, block=block, moves=moves, check=True)
    b = oracle_lib.SlopeState(L).run_dd(n, p, q, seed, block=block, moves=moves, threads=4)
    assert np.array_equal(a.sx, b.sx) and np.array_equal(a.sy, b.sy)
    assert int(a.net[0]) == int(b.net[0]) and int(a.h00[0]) == int(b.h00[0])
    oracle_lib.check_invariants(b.sx, b.sy)


def test_parallel_runner_rejects_bad_threads(oracle_lib):
    st = oracle_lib.SlopeState(16)
    assert oracle_lib.lib().or_dd_run_par(16, 1.0, 0.0, 1, 16, 16, 4, 4, 1, 0, 1, st.sx, st.sy,
                                          st.h00, st.net, 0) == oracle_lib.OR_EINVAL


@pytest.fixture(scope="module")
def chain4():
    return exact_small.SmallChain(4)


@pytest.mark.parametrize("p,q", [(0.7, 0.3), (0.9, 0.6)])
def test_generic_thresholds_match_exact_law(oracle_lib, chain4, p, q):
    """P and Q need all 32 levels of the uniform (neither is a short binary
    fraction): the oracle's mean W^2 after t MCS agrees with the exact law of
    the same schedule (one periodic 4x4 block, 4x4 tiles)."""
    t, block = 3, (4, 4)
    exact = chain4.expected_w2(chain4.dd_mcs(p, q, block, (4, 4)), [t])[t]
    n = 3000
    vals = np.empty(n)
    for i in range(n):
        st = oracle_lib.SlopeState(4).run_dd(t, p, q, 7000 + i, block=block, tile=(4, 4))
        S1, S2 = st.moments()
        vals[i] = oracle_lib.w2(S1, S2, 16)
    z = (vals.mean() - exact) / (vals.std(ddof=1) / np.sqrt(n))
    assert abs(z) < 4.0, (vals.mean(), exact, z)
