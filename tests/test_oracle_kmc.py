"""Pins of the KMC binary-alloy oracle (Sec. 2.2 "Kinetic Monte Carlo",
eqs. ``fcc`` and ``metropolis``; Sec. 3.2 "Implementation of KMC").

What fixes the oracle here, independently of its own code:

* fcc geometry (eq. ``fcc``): a lone B reaches exactly twelve distinct fcc
  positions, each two unit steps away along two axes, and can jump back;
* the Metropolis rule (eq. ``metropolis``, Gamma = 1) for the energy
  -eps * (number of B-B bonds): every exchange is accepted exactly for
  u < floor(min(1, exp(eps * delta_bonds)) 2^32), with the bond change
  counted here with numpy;
* the exact stationary law of random-sequential dynamics on the smallest
  fcc torus (L = 4) with three B atoms, enumerated by brute force;
* the double-tiled schedule: no two attempts of a step interact, every MCS
  makes N attempts that hit each site once on average, the set orderings are
  the permutations of 0..7 in lexicographic numbering, and the schedule
  reaches the same equilibrium as random-sequential dynamics.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import kmc

HALF = [(1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1)]


def np_bonds(occ):
    """B-B nearest-neighbour bonds of a cubic (z, y, x) array, fcc offsets
    (two coordinates +-1, one 0), each bond counted once."""
    o = occ.astype(np.int64)
    tot = 0
    for dx, dy, dz in HALF:
        tot += int((o * np.roll(o, shift=(-dz, -dy, -dx), axis=(0, 1, 2))).sum())
    return tot


def fcc_sites(L):
    return [(x, y, z) for z in range(L) for y in range(L) for x in range(L) if not (x ^ y ^ z) & 1]


def cyc(d, L):
    d %= L
    return min(d, L - d)


def test_thresholds_are_floor_of_exp():
    for eps in (0.0, 0.5, 1.5, 30.0):
        T = kmc.thresholds(eps)
        assert int(T[0]) == 2 ** 32
        for d in range(1, 13):
            assert int(T[d]) == min(2 ** 32, math.floor(math.exp(-d * eps) * 2 ** 32))


@pytest.mark.parametrize("L", [4, 6])
def test_lone_b_reaches_twelve_fcc_neighbours_and_returns(L):
    p = (2, 1, 1) if L == 4 else (3, 2, 1)
    dests = []
    for nb in range(12):
        occ = np.zeros((L, L, L), np.uint8)
        occ[p[2], p[1], p[0]] = 1
        assert kmc.attempt(occ, 1.5, *p, nb, 0) == 1
        (z,), (y,), (x,) = np.nonzero(occ)
        q = (int(x), int(y), int(z))
        assert not (q[0] ^ q[1] ^ q[2]) & 1
        steps = sorted(cyc(q[i] - p[i], L) for i in range(3))
        assert steps == [0, 1, 1]
        dests.append(q)
        # some neighbour choice at q brings it back
        back = 0
        for nb2 in range(12):
            occ2 = occ.copy()
            kmc.attempt(occ2, 1.5, *q, nb2, 0)
            back += occ2[p[2], p[1], p[0]]
        assert back == 1
    assert len(set(dests)) == 12


def test_a_site_pulls_b_from_neighbour_both_species_active():
    L = 6
    occ = np.zeros((L, L, L), np.uint8)
    occ[1, 1, 2] = 1                       # B at (2, 1, 1)
    moved = 0
    for nb in range(12):
        o = occ.copy()
        # i = (1, 0, 1) is an A site next to the B: (2,1,1) - (1,0,1) = (1,1,0)
        moved += kmc.attempt(o, 1.5, 1, 0, 1, nb, 0)
        if o[1, 0, 1]:
            assert o.sum() == 1 and o[1, 1, 2] == 0
    assert moved == 1


@pytest.mark.parametrize("L,eps,seed", [(4, 0.0, 1), (4, 0.7, 2), (4, 1.5, 3), (6, 1.5, 4),
                                        (6, 0.35, 5)])
def test_metropolis_threshold_equals_bond_change(L, eps, seed):
    rng = np.random.default_rng(seed)
    sites = fcc_sites(L)
    checked = 0
    for _ in range(3):
        occ = np.zeros((L, L, L), np.uint8)
        for (x, y, z) in sites:
            occ[z, y, x] = rng.random() < 0.4
        E0 = np_bonds(occ)
        for idx in rng.choice(len(sites), size=min(len(sites), 40), replace=False):
            x, y, z = sites[idx]
            for nb in range(12):
                o = occ.copy()
                if kmc.attempt(o, eps, x, y, z, nb, 0) == 0:
                    # u = 0 rejects only when the two sites hold the same species
                    assert np.array_equal(o, occ)
                    continue
                diff = np.argwhere(o != occ)
                assert len(diff) == 2 and o.sum() == occ.sum()
                dE = np_bonds(o) - E0
                Texp = 2 ** 32 if dE >= 0 else math.floor(math.exp(eps * dE) * 2 ** 32)
                if Texp > 0:
                    o2 = occ.copy()
                    assert kmc.attempt(o2, eps, x, y, z, nb, Texp - 1) == 1
                    assert np.array_equal(o2, o)
                if Texp < 2 ** 32:
                    o3 = occ.copy()
                    assert kmc.attempt(o3, eps, x, y, z, nb, Texp) == 0
                    assert np.array_equal(o3, occ)
                checked += 1
    assert checked > 100


def test_counts_match_numpy():
    for L, c, seed in ((4, 0.5, 1), (8, 0.325, 2), (10, 0.7, 3)):
        occ = kmc.init(L, c, seed)
        nB, bonds = kmc.counts(occ)
        assert nB == int(occ.sum())
        assert bonds == np_bonds(occ)


def test_init_is_bernoulli_on_fcc_sites():
    L = 16
    occ = kmc.init(L, 0.325, 7)
    mask = kmc.fcc_mask(L)
    assert occ[~mask].sum() == 0
    N = L ** 3 // 2
    frac = occ.sum() / N
    assert abs(frac - 0.325) < 5 * math.sqrt(0.325 * 0.675 / N)
    assert kmc.init(8, 0.0, 1).sum() == 0
    assert kmc.init(8, 1.0, 1).sum() == 8 ** 3 // 2
    assert np.array_equal(kmc.from_fcc(kmc.to_fcc(occ), L), occ)


def test_rs_conserves_species():
    occ = kmc.init(8, 0.3, 11)
    n0 = int(occ.sum())
    moves = kmc.rs_run(occ, 1.5, 12, 0, 5)
    assert int(occ.sum()) == n0 and moves > 0
    assert occ[~kmc.fcc_mask(8)].sum() == 0


def exact_bond_law_three_b(L, eps):
    """P(#bonds = E) for three B atoms on the L^3/2-site torus under
    exp(eps * #bonds), by enumerating all triples."""
    sites = fcc_sites(L)
    n = len(sites)
    adj = np.zeros((n, n), bool)
    for a in range(n):
        for b in range(n):
            d = sorted(cyc(sites[a][i] - sites[b][i], L) for i in range(3))
            adj[a, b] = d == [0, 1, 1]
    g = np.zeros(4)
    for a, b, c in itertools.combinations(range(n), 3):
        g[int(adj[a, b]) + int(adj[a, c]) + int(adj[b, c])] += 1
    w = g * np.exp(eps * np.arange(4))
    return g, w / w.sum()


def test_rs_stationary_law_three_b_on_smallest_torus():
    L, eps = 4, 1.0
    g, law = exact_bond_law_three_b(L, eps)
    assert g.sum() == math.comb(32, 3)
    occ = np.zeros((L, L, L), np.uint8)
    occ[0, 0, 0] = occ[0, 2, 0] = occ[2, 2, 2] = 1
    hist = np.zeros(4)
    kmc.rs_run(occ, eps, 99, 0, 200)
    for t in range(200, 200 + 30000, 5):
        kmc.rs_run(occ, eps, 99, t, 5)
        hist[kmc.counts(occ)[1]] += 1
    emp = hist / hist.sum()
    # about 6000 samples, correlated over a few samples
    assert np.all(np.abs(emp - law) < 0.03), (emp, law)
    # a rule that counted b among e's B neighbours would bias towards bonds
    assert abs(emp @ np.arange(4) - law @ np.arange(4)) < 0.05


@pytest.mark.parametrize("L,B", [(16, 8), (32, 8), (32, 16), (64, 32)])
def test_dt_steps_never_interact_and_hit_each_site_once_per_mcs(L, B):
    occ = kmc.init(L, 0.325, 3)
    n0 = int(occ.sum())
    N = L ** 3 // 2
    nmcs = 1 if L == 64 else 3
    cnt = np.zeros(N, np.int32)
    kmc.dt_run(occ, 1.5, 5, B, 0, nmcs, check=True, counts=cnt)
    assert int(cnt.sum()) == nmcs * N
    assert int(occ.sum()) == n0
    assert occ[~kmc.fcc_mask(L)].sum() == 0


def test_dt_site_attempts_are_uniform():
    L, B, n = 16, 8, 20
    N = L ** 3 // 2
    cnt = np.zeros(N, np.int32)
    occ = kmc.init(L, 0.3, 1)
    kmc.dt_run(occ, 1.0, 8, B, 0, n, counts=cnt)
    # each attempt hits a given site with probability 1/256 within its
    # tile: Binomial(256, 1/256) per MCS, variance about 1 per MCS
    assert cnt.mean() == n
    assert 0.75 * n < cnt.var() < 1.25 * n


def lehmer_index(perm):
    idx = 0
    rest = list(range(8))
    for i, v in enumerate(perm):
        k = rest.index(v)
        idx += k * math.factorial(7 - i)
        rest.pop(k)
    return idx


def test_dt_order_is_lexicographic_permutation_number():
    from oracle import draw
    seed = 77
    first = np.zeros(8)
    for t in range(3000):
        p = kmc.order(seed, t)
        assert sorted(p) == list(range(8))
        w0 = int(draw(seed, kmc.TAG_ORDER, t, 0, 0)[0])
        assert lehmer_index(p) == (w0 * 40320) >> 32
        first[p[0]] += 1
    assert np.all(np.abs(first - 375) < 90)


def test_dt_origin_is_scaled_draw():
    from oracle import draw
    for t in range(50):
        w = draw(3, kmc.TAG_ORIGIN, t, 0, 0)
        assert kmc.origin(3, t, 32) == tuple((int(w[i]) * 32) >> 32 for i in range(3))


def _mean_bonds(run, occ, t0, burn, n, every):
    run(occ, t0, burn)
    vals = []
    t = t0 + burn
    for _ in range(n):
        run(occ, t, every)
        t += every
        vals.append(kmc.counts(occ)[1])
    v = np.array(vals, float)
    # batch means of 10 for the standard error
    bm = v[: len(v) // 10 * 10].reshape(10, -1).mean(axis=1)
    return v.mean(), bm.std(ddof=1) / math.sqrt(len(bm))


def test_dt_and_rs_reach_the_same_equilibrium():
    L, c, eps = 16, 0.3, 0.6
    occ_rs = kmc.init(L, c, 21)
    occ_dt = occ_rs.copy()
    m_rs, e_rs = _mean_bonds(lambda o, t, n: kmc.rs_run(o, eps, 31, t, n), occ_rs, 0, 100, 200, 3)
    m_dt, e_dt = _mean_bonds(lambda o, t, n: kmc.dt_run(o, eps, 32, 8, t, n), occ_dt, 0, 100,
                             200, 3)
    assert abs(m_rs - m_dt) < 5 * math.hypot(e_rs, e_dt) + 2.0, (m_rs, e_rs, m_dt, e_dt)
    # the interaction is felt: more bonds than a random mixture
    nB = int(occ_rs.sum())
    random_mix = 6 * nB * (nB - 1) / (L ** 3 // 2 - 1)
    assert m_rs > random_mix + 20


def test_dt_rejects_bad_shapes():
    occ = np.zeros((16, 16, 16), np.uint8)
    for B in (4, 12, 16):          # not a multiple of 8, or L/B odd
        with pytest.raises(RuntimeError):
            kmc.dt_run(occ, 1.0, 1, B, 0, 1)
