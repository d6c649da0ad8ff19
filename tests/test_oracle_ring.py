"""Pins of the oracle's 1+1-d decomposed schedule (the rooftop ring of
Sec. 2.1 under the decomposition of Sec. 3 / 3.1 reduced to one dimension):
packing, invariants, the no-neighbours property of each step, conjugation
symmetry, the block runner, the exact law on tiny rings (70 states at L = 8),
and the KPZ / EW growth exponents."""
import numpy as np
import pytest

from oracle import exact_small


def test_flat_ring_and_packing(oracle_lib):
    r = oracle_lib.RingState(64)
    assert list(oracle_lib.pack1d(r.s)) == [0x55555555, 0x55555555]
    assert r.moments() == (32, 32)           # h = i mod 2
    rng = np.random.default_rng(1)
    s = (2 * rng.integers(0, 2, 256) - 1).astype(np.int8)
    assert np.array_equal(oracle_lib.unpack1d(oracle_lib.pack1d(s)), s)


@pytest.mark.parametrize("L,B,p,q", [(64, 16, 1.0, 0.0), (256, 64, 0.7, 0.2), (128, 128, 0.5, 0.5),
                                     (96, 32, 1.0, 0.4)])
def test_ring_dd_invariants_and_mass_balance(oracle_lib, L, B, p, q):
    r = oracle_lib.RingState(L)
    for _ in range(6):
        r.run_dd(3, p, q, 11, B, check=True)
        assert int(r.s.sum()) == 0
        S1, _ = r.moments()
        assert S1 == L // 2 + 2 * int(r.net[0])
        h = r.heights()
        assert np.all((h - np.arange(L) - int(r.h0[0])) % 2 == 0)


def test_ring_dd_invalid_blocks_rejected(oracle_lib):
    r = oracle_lib.RingState(64)
    for B in (0, 6, 48, 128):
        with pytest.raises(RuntimeError):
            r.run_dd(1, 1.0, 0.0, 1, B)


@pytest.mark.parametrize("p,q", [(1.0, 0.0), (0.7, 0.2)])
def test_ring_dd_conjugation_symmetry(oracle_lib, p, q):
    L, B = 128, 32
    a = oracle_lib.RingState(L).run_rs(3, 0.9, 0.1, 5)
    b = a.copy()
    b.s = (-b.s).astype(np.int8)
    b.h0, b.net = -b.h0, -b.net
    a.run_dd(7, p, q, 12, B)
    b.run_dd(7, q, p, 12, B)
    assert np.array_equal(b.s, -a.s) and b.h0[0] == -a.h0[0] and b.net[0] == -a.net[0]


@pytest.mark.parametrize("p,q", [(1.0, 0.0), (0.6, 0.3)])
def test_ring_block_runner_equals_full_run(oracle_lib, p, q):
    L, B, seed = 512, 128, 9
    st = oracle_lib.RingState(L).run_dd(2, p, q, seed, B)
    before = st.copy()
    t = st.t
    st.run_dd(1, p, q, seed, B)
    o = oracle_lib.dd1d_origin(seed, t, B)
    total = 0
    for b in range(L // B):
        idx = (o + b * B + np.arange(B)) % L
        bs = np.ascontiguousarray(before.s[idx])
        total += oracle_lib.dd1d_block_mcs(L, p, q, seed, B, t, b, bs)
        assert np.array_equal(bs, st.s[idx]), b
    assert total == int(st.net[0] - before.net[0])


def test_exact_ring_single_tile_is_rs():
    c = exact_small.RingChain(4)
    assert np.allclose(c.dd_mcs(1.0, 0.0, 4), c.rs_mcs(1.0, 0.0))
    assert np.allclose(c.dd_mcs(0.7, 0.2, 4), c.rs_mcs(0.7, 0.2))


def test_exact_ring_symmetric_rates_uniform():
    c = exact_small.RingChain(8)
    for T in (c.dd_mcs(0.5, 0.5, 8), c.dd_mcs(0.5, 0.5, 4)):
        w, v = np.linalg.eig(T.T)
        pi = np.real(v[:, np.argmin(np.abs(w - 1))])
        pi /= pi.sum()
        assert np.allclose(pi, 1.0 / c.n)


@pytest.fixture(scope="module")
def ring8():
    return exact_small.RingChain(8)


@pytest.mark.parametrize("B,p,q,t", [(8, 1.0, 0.0, 2), (4, 1.0, 0.0, 2), (8, 1.0, 0.375, 3)])
def test_ring_dd_matches_exact_law(oracle_lib, ring8, B, p, q, t):
    pi_t = ring8.distribution(ring8.dd_mcs(p, q, B), t)
    n = 4000
    counts = np.zeros(ring8.n)
    for i in range(n):
        r = oracle_lib.RingState(8).run_dd(t, p, q, 20_000 + i, B)
        counts[ring8.index[tuple(int(v) for v in r.s)]] += 1
    exp = pi_t * n
    big = exp >= 5
    o2 = np.append(counts[big], counts[~big].sum())
    e2 = np.append(exp[big], exp[~big].sum())
    keep = e2 > 0
    chi2 = (((o2[keep] - e2[keep]) ** 2) / e2[keep]).sum()
    dof = keep.sum() - 1
    assert chi2 < dof + 4.5 * np.sqrt(2 * dof) + 10, (chi2, dof)


def test_exact_ring_dead_border_changes_the_law(ring8):
    a = ring8.distribution(ring8.dd_mcs(1.0, 0.0, 8), 2)
    b = ring8.distribution(ring8.dd_mcs(1.0, 0.0, 4), 2)
    assert np.abs(a - b).sum() > 0.1


def _beta_ring_dd(oracle_lib, p, q, L=1 << 14, B=1 << 11, seeds=4,
                  times=(64, 128, 256, 512, 1024)):
    w2 = np.zeros(len(times))
    for seed in range(seeds):
        r = oracle_lib.RingState(L)
        for i, T in enumerate(times):
            r.run_dd(T - r.t, p, q, 700 + seed, B)
            h = r.heights().astype(np.float64)
            w2[i] += h.var() / seeds
    return np.polyfit(np.log(times), np.log(w2), 1)[0] / 2


def test_ring_dd_kpz_and_ew_beta(oracle_lib):
    b_kpz = _beta_ring_dd(oracle_lib, 1.0, 0.0)
    b_ew = _beta_ring_dd(oracle_lib, 0.5, 0.5)
    assert 0.28 <= b_kpz <= 0.36, b_kpz
    assert 0.21 <= b_ew <= 0.28, b_ew


def _ring_w2_at(oracle_lib, L, T, block, seeds):
    vals = []
    for s in range(seeds):
        r = oracle_lib.RingState(L)
        if block is None:
            r.run_rs(T, 1.0, 0.0, 40 + s)
        else:
            r.run_dd(T, 1.0, 0.0, 40 + s, block)
        vals.append(r.heights().astype(np.float64).var())
    return float(np.mean(vals))


def test_ring_block_size_changes_the_amplitude(oracle_lib):
    """Every block draws one cell set per step for all its tiles, which
    correlates the block's updates: in one dimension the W^2 amplitude at
    t = 256 (L = 8192, p = 1) stays within 10 % of random-sequential
    dynamics for 128-site blocks, and falls by more than 15 % for a single
    block spanning the ring -- the reason the ring's blocks are small."""
    L, T, seeds = 8192, 256, 12
    rs = _ring_w2_at(oracle_lib, L, T, None, seeds)
    small = _ring_w2_at(oracle_lib, L, T, 128, seeds)
    whole = _ring_w2_at(oracle_lib, L, T, L, seeds)
    assert abs(small / rs - 1) < 0.10, (small, rs)
    assert whole / rs - 1 < -0.15, (whole, rs)
