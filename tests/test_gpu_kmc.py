"""GPU parity of the KMC binary alloy (Sec. 2.2 "Kinetic Monte Carlo";
Sec. 3.2 "Implementation of KMC") against the oracle's doubly tiled schedule:
every site byte, the accepted-jump count and the B / bond counts after each
call, bit for bit, from small lattices with one block per set up to the
512^3 / 2 quench benchmark (c = 0.325, eps = 1.5)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1204_5072_amd as kpz
    kpz.lib()
    return kpz


@pytest.fixture(scope="module")
def kmc(oracle_lib):
    from oracle import kmc as k
    return k


@pytest.mark.parametrize("L,c,seed", [(16, 0.325, 1), (32, 0.5, 7), (64, 0.0, 3), (64, 1.0, 4),
                                      (128, 0.325, 9)])
def test_init_matches_oracle(gpu, kmc, L, c, seed):
    _log(f"kmc init L={L} c={c} seed={seed}")
    sim = gpu.Kmc(L, c=c, eps=1.5, seed=seed)
    ref = kmc.init(L, c, seed)
    assert np.array_equal(sim.occ_host(), kmc.to_fcc(ref))
    assert sim.counts() == kmc.counts(ref)
    assert sim.state() == (0, 0)


CASES = [  # L, block, c, eps, seed, calls of n MCS
    (16, 8, 0.325, 1.5, 1, (1, 2)),
    (32, 8, 0.325, 1.5, 2, (2,)),
    (32, 16, 0.5, 0.7, 3, (1, 1)),
    (64, 32, 0.325, 1.5, 4, (1,)),
    (64, 16, 0.1, 3.0, 5, (2,)),
    (64, 8, 0.3, 0.0, 6, (1,)),
    (128, 32, 0.6, 1.2, 7, (1,)),
    (32, 16, 1.0, 1.5, 8, (1,)),     # all B: nothing can move
]


@pytest.mark.parametrize("L,B,c,eps,seed,calls", CASES)
def test_sweep_matches_oracle(gpu, kmc, L, B, c, eps, seed, calls):
    sim = gpu.Kmc(L, c=c, eps=eps, seed=seed, block=B)
    ref = kmc.init(L, c, seed)
    t = 0
    moves = 0
    for n in calls:
        _log(f"kmc sweep L={L} B={B} c={c} eps={eps} seed={seed} t={t} n={n}")
        sim.sweep(n)
        moves += kmc.dt_run(ref, eps, seed, B, t, n)
        t += n
        got = sim.occ_host()
        exp = kmc.to_fcc(ref)
        bad = np.flatnonzero(got != exp)
        assert bad.size == 0, f"{bad.size} sites differ, first {bad[:8]}"
        assert sim.state() == (t, moves)
        assert sim.counts() == kmc.counts(ref)
    if c in (0.0, 1.0):
        assert moves == 0
    else:
        assert moves > 0


def test_load_resumes_the_schedule(gpu, kmc):
    L, B, eps, seed = 32, 16, 1.5, 11
    ref = kmc.init(L, 0.4, 5)
    m0 = kmc.dt_run(ref, eps, seed, B, 0, 3)
    sim = gpu.Kmc(L, c=0.0, eps=eps, seed=seed, block=B)
    sim.load(kmc.to_fcc(ref), t=3, moves=m0)
    _log("kmc load at t=3, sweep 2")
    sim.sweep(2)
    m1 = kmc.dt_run(ref, eps, seed, B, 3, 2)
    assert np.array_equal(sim.occ_host(), kmc.to_fcc(ref))
    assert sim.state() == (5, m0 + m1)


def test_quench_benchmark_size_one_mcs(gpu, kmc):
    """The 512^3/2-site quench (c = 0.325, eps = 1.5) with 32^3 blocks, the
    configuration the benchmark times: one full MCS, every site."""
    L, B, c, eps, seed = 512, 32, 0.325, 1.5, 2024
    _log("kmc L=512 init + 1 MCS on the GPU")
    sim = gpu.Kmc(L, c=c, eps=eps, seed=seed, block=B)
    sim.sweep(1)
    got = sim.occ_host()
    _log("kmc L=512 oracle (about half a minute)")
    ref = kmc.init(L, c, seed)
    moves = kmc.dt_run(ref, eps, seed, B, 0, 1)
    exp = kmc.to_fcc(ref)
    del ref
    bad = np.flatnonzero(got != exp)
    assert bad.size == 0, f"{bad.size} sites differ, first {bad[:8]}"
    assert sim.state() == (1, moves)


def test_quench_orders_the_alloy(gpu):
    """Spinodal decomposition at c = 0.325, eps = 1.5: B-B bonds grow from
    the random-mixture value and the B count never changes."""
    L = 64
    sim = gpu.Kmc(L, c=0.325, eps=1.5, seed=3)
    nb0, b0 = sim.counts()
    N = L ** 3 // 2
    assert abs(b0 - 6 * nb0 * (nb0 - 1) / (N - 1)) < 0.03 * b0
    sim.sweep(20)
    nb1, b1 = sim.counts()
    assert nb1 == nb0
    assert b1 > 1.3 * b0
