"""The device-side surface check (kpz_check_invariants, Sec. 2.1: slopes
close around every plaquette and sum to zero along every periodic row and
column) against the oracle's counts of the same surface.

Valid surfaces from the GPU's own runs must give (0, 0, 0); surfaces broken
on the host (single flipped bonds at the word, row and lattice edges, random
flips, a tilted plane) must give exactly the oracle's counts of open
plaquettes and of the row-0 / column-0 slope sums.
"""
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


def _counts_of(gpu, L, words):
    sim = gpu.Sim(L, 1.0, 0.0, 1)
    sim.load_words(words)
    c = sim.check_invariants()
    sim.close()
    return c


@pytest.mark.parametrize("L", [16, 48, 64, 256, 1024])
def test_valid_surfaces_after_sweeps(gpu, oracle_lib, L):
    """Flat start and after a few MCS (two-buffer mode, rotated storage) for
    one- and multi-word rows, W = L/16 a multiple of 4 or not."""
    _log(f"check after sweeps L={L}")
    sim = gpu.Sim(L, 0.7, 0.3, 5)
    assert sim.check_invariants() == (0, 0, 0)
    for _ in range(3):
        sim.sweep(2)
        assert sim.check_invariants() == (0, 0, 0)
        sx, sy = oracle_lib.unpack(sim.words_host(), L)
        assert oracle_lib.invariant_counts(sx, sy) == (0, 0, 0)
    sim.close()


@pytest.mark.parametrize("L", [16, 48, 128])
def test_single_flips_match_oracle(gpu, oracle_lib, L):
    """One flipped sigma_x or sigma_y bond at interior sites, at the last site
    of a word (the right neighbour's sigma_y comes from the next word), in the
    last column and row (periodic wrap) and in row / column 0."""
    _log(f"single flips L={L}")
    st = oracle_lib.SlopeState(L)
    st.run_dd(3, 1.0, 0.3, 2, block=(16, 16), tile=(4, 4))
    base = oracle_lib.pack(st.sx, st.sy)
    sites = [(0, 0), (0, 15), (5, 15), (5, 16 % L), (L - 1, L - 1), (L - 1, 0), (3, L - 1),
             (7, 9)]
    for y, x in sites:
        for bit in (0, 1):
            w = base.copy()
            w[y, x // 16] ^= np.uint32(1 << (2 * (x % 16) + bit))
            sx, sy = oracle_lib.unpack(w, L)
            want = oracle_lib.invariant_counts(sx, sy)
            assert want[0] == 2
            assert _counts_of(gpu, L, w) == want, (y, x, bit)


def test_random_flips_match_oracle(gpu, oracle_lib):
    """Many flipped bonds at random places of a 256 x 256 surface."""
    L = 256
    rng = np.random.default_rng(11)
    st = oracle_lib.SlopeState(L)
    st.run_dd(2, 1.0, 0.0, 3, block=(64, 64), tile=(4, 4))
    base = oracle_lib.pack(st.sx, st.sy)
    for n in (1, 2, 17, 300):
        w = base.copy().reshape(-1)
        idx = rng.integers(0, w.size, n)
        bits = rng.integers(0, 32, n).astype(np.uint32)
        for i, b in zip(idx, bits):
            w[i] ^= np.uint32(1) << b
        w = w.reshape(L, L // 16)
        sx, sy = oracle_lib.unpack(w, L)
        assert _counts_of(gpu, L, w) == oracle_lib.invariant_counts(sx, sy), n


def test_tilted_planes(gpu, oracle_lib):
    """Planes tilted along y and along x: every plaquette closed, one slope
    sum equal to L."""
    L = 64
    x = np.arange(L)
    alt = np.tile(np.where(x % 2 == 0, 1, -1), (L, 1)).astype(np.int8)
    ones = np.ones((L, L), np.int8)
    for sx, sy in ((alt, ones), (ones.T.copy(), alt.T.copy())):
        w = oracle_lib.pack(sx, sy)
        assert _counts_of(gpu, L, w) == oracle_lib.invariant_counts(sx, sy)


def test_large_lattice_after_sweeps(gpu):
    """L = 16384 after 20 MCS of the default schedule with acceptance: still a
    valid surface, and one flipped bond is seen."""
    import torch
    L = 16384
    _log("check L=16384")
    sim = gpu.Sim(L, 0.7, 0.3, 9)
    sim.sweep(20)
    assert sim.check_invariants() == (0, 0, 0)
    sim.sync_words()
    t, net = sim.state()
    w = sim.words.view(L, L // 16)
    with torch.cuda.stream(sim.stream):
        w[1234, 77] ^= 1 << 6        # sigma_x of site (16*77 + 3, 1234)
    sim.set_state(t, net)            # `words` holds the lattice from here on
    c = sim.check_invariants()
    assert c[0] == 2 and c[2] == 0
    sim.close()
