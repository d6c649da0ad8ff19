"""Pins for the oracle's model code against what the paper and the mathematics
fix (Sec. 2.1 rule and observables, Sec. 3 / 3.1 decomposition):

* t = 0 values of the flat start and the packed words it implies,
* random-sequential heights == random-sequential slopes, draw for draw,
* the slope-field invariants after any dynamics,
* mass balance S1(t) - S1(0) = 2 (deposits - desorptions),
* height reconstruction independent of the path,
* up-down conjugation symmetry (exact, bit level),
* the decomposed schedule never updates two neighbours in one step,
* exact 4x4 master-equation law (enumerated independently) vs Monte Carlo of
  both the random-sequential and the decomposed oracle modes.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact_small


# ------------------------------------------------------------------ t = 0

@pytest.mark.parametrize("L", [2, 4, 16, 64])
def test_flat_start_values(oracle_lib, L):
    s = oracle_lib.SlopeState(L)
    oracle_lib.check_invariants(s.sx, s.sy)
    h = s.heights()
    assert np.array_equal(h, oracle_lib.flat_heights(L))
    S1, S2 = oracle_lib.moments(h)
    N = L * L
    assert S1 == N // 2 and S2 == N // 2
    assert oracle_lib.w2_exact(S1, S2, N) == Fraction(1, 4)


def test_flat_words(oracle_lib):
    # even rows: sites x even have sigma_x = sigma_y = +1 (h = 0 below h = 1
    # neighbours), x odd both -1 -> 2-bit fields 11,00,11,.. = 0x33333333;
    # odd rows the complement 0xCCCCCCCC.
    L = 64
    s = oracle_lib.SlopeState(L)
    w = oracle_lib.pack(s.sx, s.sy)
    assert (w[0::2] == 0x33333333).all() and (w[1::2] == 0xCCCCCCCC).all()
    sx, sy = oracle_lib.unpack(w, L)
    assert np.array_equal(sx, s.sx) and np.array_equal(sy, s.sy)


def test_pack_roundtrip_random(oracle_lib):
    L = 32
    s = oracle_lib.SlopeState(L).run_rs(3, 1.0, 0.3, 5)
    w = oracle_lib.pack(s.sx, s.sy)
    sx, sy = oracle_lib.unpack(w, L)
    assert np.array_equal(sx, s.sx) and np.array_equal(sy, s.sy)
    # bit 2k of word w = sigma_x of site x = 16 w + k
    for y, x in [(0, 0), (3, 17), (31, 31), (7, 16)]:
        word = int(w[y, x // 16])
        assert ((word >> (2 * (x % 16))) & 1) == (s.sx[y, x] > 0)
        assert ((word >> (2 * (x % 16) + 1)) & 1) == (s.sy[y, x] > 0)


# ------------------------------------------------- rule / encoding (P2)

@pytest.mark.parametrize("p,q,seed", [(1.0, 0.0, 1), (0.5, 0.5, 2), (1.0, 0.25, 3), (0.3, 0.7, 4)])
def test_rs_heights_equal_rs_slopes(oracle_lib, p, q, seed):
    L = 24
    h = oracle_lib.flat_heights(L)
    s = oracle_lib.SlopeState(L)
    for t in range(6):
        h = oracle_lib.rs_heights_run(h, t, 1, p, q, seed)
        s.run_rs(1, p, q, seed)
        assert np.array_equal(s.heights(), h), t


# ------------------------------------------------------- invariants (P3, P4)

DD_SHAPES = [((16, 16), (4, 4)), ((32, 16), (4, 4)), ((64, 64), (4, 4)),
             ((16, 32), (4, 4)), ((8, 8), (2, 2)), ((64, 16), (4, 4))]


@pytest.mark.parametrize("block,tile", DD_SHAPES)
@pytest.mark.parametrize("p,q", [(1.0, 0.0), (0.5, 0.5), (1.0, 0.5)])
def test_dd_invariants_and_mass_balance(oracle_lib, block, tile, p, q):
    L = 64
    s = oracle_lib.SlopeState(L)
    S1_0, _ = s.moments()
    for _ in range(4):
        s.run_dd(3, p, q, 7, block=block, tile=tile, check=True)
        oracle_lib.check_invariants(s.sx, s.sy)
        S1, _ = s.moments()
        assert S1 - S1_0 == 2 * int(s.net[0])
    # heights keep the checkerboard parity h = x + y + h00 (mod 2)
    h = s.heights()
    y, x = np.mgrid[0:L, 0:L]
    assert (((h - x - y - int(s.h00[0])) % 2) == 0).all()


def test_rs_invariants_and_mass_balance(oracle_lib):
    s = oracle_lib.SlopeState(32)
    S1_0, _ = s.moments()
    s.run_rs(20, 0.8, 0.4, 11)
    oracle_lib.check_invariants(s.sx, s.sy)
    assert s.moments()[0] - S1_0 == 2 * int(s.net[0])


def test_height_path_independence(oracle_lib):
    s = oracle_lib.SlopeState(32).run_dd(10, 1.0, 0.25, 3, block=(16, 16))
    assert np.array_equal(oracle_lib.heights(s.sx, s.sy, 5), oracle_lib.heights_rowfirst(s.sx, s.sy, 5))
    # and the reconstruction inverts the slope map
    sx, sy = oracle_lib.slopes_from_heights(s.heights())
    assert np.array_equal(sx, s.sx) and np.array_equal(sy, s.sy)


def test_p_one_makes_every_attempted_minimum_flip(oracle_lib):
    """With p = 1, q = 0 a deposition never fails and nothing desorbs: the
    height field is non-decreasing site by site."""
    s = oracle_lib.SlopeState(32)
    h_prev = s.heights()
    for _ in range(5):
        s.run_dd(1, 1.0, 0.0, 9, block=(16, 16))
        h = s.heights()
        assert (h >= h_prev).all()
        h_prev = h


def test_q_zero_p_zero_is_frozen(oracle_lib):
    s = oracle_lib.SlopeState(32).run_dd(5, 0.0, 0.0, 9, block=(16, 16))
    f = oracle_lib.SlopeState(32)
    assert np.array_equal(s.sx, f.sx) and np.array_equal(s.sy, f.sy) and s.net[0] == 0


# ------------------------------------------------- conjugation symmetry (P6)

def _negated(state):
    o = state.copy()
    o.sx = (-o.sx).astype(np.int8)
    o.sy = (-o.sy).astype(np.int8)
    o.h00 = -o.h00
    o.net = -o.net
    return o


@pytest.mark.parametrize("mode", ["rs", "dd", "dd_dead"])
@pytest.mark.parametrize("p,q", [(1.0, 0.0), (0.7, 0.2), (1.0, 0.5)])
def test_conjugation_symmetry(oracle_lib, mode, p, q):
    """h -> -h swaps minima and maxima, so run(p, q, s0) = -run(q, p, -s0)
    bit for bit: site choices do not depend on the state and the same
    uniform is compared with P for a minimum and with Q for a maximum."""
    L = 32
    a = oracle_lib.SlopeState(L).run_rs(2, 0.9, 0.1, 99)   # some non-flat start
    b = _negated(a)
    for st, (pp, qq) in ((a, (p, q)), (b, (q, p))):
        if mode == "rs":
            st.run_rs(6, pp, qq, 5)
        elif mode == "dd":
            st.run_dd(6, pp, qq, 5, block=(32, 32))
        else:
            st.run_dd(6, pp, qq, 5, block=(16, 8))
    assert np.array_equal(b.sx, -a.sx) and np.array_equal(b.sy, -a.sy)
    assert b.h00[0] == -a.h00[0] and b.net[0] == -a.net[0]


# ------------------------------------------------------- schedule checks

@pytest.mark.parametrize("L,block,tile", [(16, (16, 16), (4, 4)), (32, (16, 16), (4, 4)),
                                          (64, (32, 16), (4, 4)), (16, (4, 4), (2, 2)),
                                          (16, (16, 4), (4, 4))])
def test_dd_step_attempts_never_neighbours(oracle_lib, L, block, tile):
    # check=True makes the oracle verify, for every step, that no two
    # attempted sites of the whole lattice coincide or are nearest neighbours
    oracle_lib.SlopeState(L).run_dd(4, 0.5, 0.5, 21, block=block, tile=tile, check=True)


def test_dd_invalid_shapes_rejected(oracle_lib):
    s = oracle_lib.SlopeState(32)
    for block, tile in [((12, 32), (4, 4)), ((32, 32), (16, 16)), ((32, 24), (4, 4)), ((32, 32), (3, 3)),
                        ((36, 32), (8, 8))]:
        with pytest.raises(RuntimeError):
            s.run_dd(1, 1.0, 0.0, 1, block=block, tile=tile)


def test_dd_dead_border_sites_never_change(oracle_lib):
    """Over one MCS, sites of the dead border (local x = 0 or y = 0 of the
    shifted blocks) keep their height."""
    L, B = 32, (8, 8)
    s = oracle_lib.SlopeState(L).run_dd(3, 1.0, 0.3, 4, block=B)
    t = s.t
    h0 = s.heights()
    s.run_dd(1, 1.0, 0.3, 4, block=B)
    h1 = s.heights()
    w = oracle_lib.draw(4, oracle_lib.TAG_ORIGIN, t, 0, 0)
    ox = (int(w[0]) * B[0]) >> 32
    oy = (int(w[1]) * B[1]) >> 32
    y, x = np.mgrid[0:L, 0:L]
    dead = (((x - ox) % B[0]) == 0) | (((y - oy) % B[1]) == 0)
    assert np.array_equal(h0[dead], h1[dead])
    assert (h0[~dead] != h1[~dead]).any()


# ------------------------------------------------- exact 4x4 law (P7, P8)

@pytest.fixture(scope="module")
def chain4():
    return exact_small.SmallChain(4)


def test_exact_state_count(chain4):
    # every zero-tilt surface of the 4x4 torus is reachable from flat
    assert chain4.n == exact_small.count_height_functions(4)
    assert chain4.w2[chain4.flat] == 0.25


def test_exact_first_attempt_closed_form(chain4):
    """From flat every site is an extremum; one flip by +-2 gives
    W^2 = (N/2+4)/N - ((N/2+2)/N)^2 (= the value for a -2 flip)."""
    N = 16
    w_one = Fraction(N // 2 + 4, N) - Fraction(N // 2 + 2, N) ** 2
    assert w_one == Fraction(N // 2, N) - Fraction(N // 2 - 2, N) ** 2
    for p, q in [(1.0, 0.0), (0.5, 0.5), (0.3, 0.9)]:
        T1 = sum(chain4.site_operator(s, p, q) for s in range(N)) / N
        pi = np.zeros(chain4.n)
        pi[chain4.flat] = 1
        e = (pi @ T1) @ chain4.w2
        assert e == pytest.approx(0.25 + (p + q) / 2 * float(w_one - Fraction(1, 4)), abs=1e-14)


def test_exact_symmetric_rates_uniform(chain4):
    T = chain4.rs_mcs(0.5, 0.5)
    assert np.allclose(T.sum(axis=1), 1.0)
    pi = chain4.stationary(T)
    assert np.allclose(pi, 1.0 / chain4.n, atol=1e-12)
    # any DD shape at p = q is symmetric too
    Td = chain4.dd_mcs(0.5, 0.5, (2, 2), (2, 2))
    assert np.allclose(chain4.stationary(Td), 1.0 / chain4.n, atol=1e-12)


def test_exact_conjugation(chain4):
    a = chain4.expected_w2(chain4.rs_mcs(1.0, 0.25), [1, 3])
    b = chain4.expected_w2(chain4.rs_mcs(0.25, 1.0), [1, 3])
    assert a[1] == pytest.approx(b[1], abs=1e-12) and a[3] == pytest.approx(b[3], abs=1e-12)


def test_exact_one_tile_dd_is_rs(chain4):
    """One block and one tile: uniform set x uniform site in its cell =
    uniform site, and S = N steps make one MCS -- the law of RS."""
    Trs = chain4.rs_mcs(1.0, 0.0)
    Tdd = chain4.dd_mcs(1.0, 0.0, (4, 4), (4, 4))
    assert np.allclose(Trs, Tdd, atol=1e-12)


def test_exact_checkerboard_control_is_biased(chain4):
    """1x1 cells make every step a deterministic sublattice sweep: the
    stationary width differs grossly from random-sequential."""
    prs = chain4.stationary(chain4.rs_mcs(1.0, 0.0))
    pdd = chain4.stationary(chain4.dd_mcs(1.0, 0.0, (4, 4), (2, 2)))
    assert abs(prs @ chain4.w2 - pdd @ chain4.w2) > 0.1


def _mc_w2(oracle_lib, runner, n_seeds, t):
    vals = np.empty(n_seeds)
    for i in range(n_seeds):
        st = runner(i)
        S1, S2 = st.moments() if hasattr(st, "moments") else oracle_lib.moments(st)
        vals[i] = oracle_lib.w2(S1, S2, 16)
    return vals


def _z(vals, exact):
    return (vals.mean() - exact) / (vals.std(ddof=1) / np.sqrt(len(vals)) + 1e-300)


@pytest.mark.parametrize("p,q", [(1.0, 0.0), (1.0, 0.5)])
def test_rs_oracle_matches_exact_law(oracle_lib, chain4, p, q):
    T = chain4.rs_mcs(p, q)
    t = 2
    exact = chain4.expected_w2(T, [t])[t]
    vals = _mc_w2(oracle_lib, lambda i: oracle_lib.rs_heights_run(
        oracle_lib.flat_heights(4), 0, t, p, q, 1000 + i), 3000, t)
    assert abs(_z(vals, exact)) < 4.0


DD_EXACT_CASES = [((4, 4), (4, 4)), ((4, 4), (2, 2)), ((2, 2), (2, 2)), ((4, 2), (2, 2))]


@pytest.mark.parametrize("block,tile", DD_EXACT_CASES)
def test_dd_oracle_matches_exact_law(oracle_lib, chain4, block, tile):
    p, q, t = 1.0, 0.0, 2
    T = chain4.dd_mcs(p, q, block, tile)
    pi_t = chain4.distribution(T, t)
    n = 3000
    counts = np.zeros(chain4.n)
    for i in range(n):
        st = oracle_lib.SlopeState(4).run_dd(t, p, q, 5000 + i, block=block, tile=tile)
        code = exact_small.state_from_slopes(st.sx, st.sy)
        counts[chain4.index[code]] += 1
    # compare the law of W^2 (pooled over states with equal W^2)
    keys = np.round(chain4.w2, 12)
    uniq = np.unique(keys)
    obs = np.array([counts[keys == k].sum() for k in uniq])
    exp = np.array([pi_t[keys == k].sum() for k in uniq]) * n
    big = exp >= 5
    o2 = np.append(obs[big], obs[~big].sum())
    e2 = np.append(exp[big], exp[~big].sum())
    keep = e2 > 0
    chi2 = (((o2 - e2) ** 2) / e2)[keep].sum()
    dof = keep.sum() - 1
    # chi2 upper quantile at p ~ 1e-4: dof + 4.5 sqrt(2 dof) + 10 is safely above
    assert chi2 < dof + 4.5 * np.sqrt(2 * dof) + 10, (chi2, dof)
    exact_mean = float(pi_t @ chain4.w2)
    mc_mean = float((counts @ chain4.w2) / n)
    sd = float(np.sqrt(pi_t @ (chain4.w2 - exact_mean) ** 2))
    assert abs(mc_mean - exact_mean) < 4.5 * sd / np.sqrt(n)


def test_dd_with_acceptance_matches_exact_law(oracle_lib, chain4):
    """q in (0,1) exercises the two-level acceptance uniform."""
    p, q, t = 1.0, 0.375, 3
    block, tile = (4, 4), (4, 4)
    T = chain4.dd_mcs(p, q, block, tile)
    exact = chain4.expected_w2(T, [t])[t]
    vals = _mc_w2(oracle_lib, lambda i: oracle_lib.SlopeState(4).run_dd(
        t, p, q, 9000 + i, block=block, tile=tile), 3000, t)
    assert abs(_z(vals, exact)) < 4.0


@pytest.mark.parametrize("p,q", [(1.0, 0.0), (0.6, 0.4)])
def test_block_runner_equals_full_run(oracle_lib, p, q):
    """One block on its own copy == that block's part of the whole-lattice
    MCS (blocks of one MCS do not interact)."""
    L, B, seed = 64, (32, 16), 3
    st = oracle_lib.SlopeState(L).run_dd(2, p, q, seed, block=B)
    before = st.copy()
    t = st.t
    st.run_dd(1, p, q, seed, block=B)
    origin = oracle_lib.dd_origin(seed, t, B)
    total = 0
    for by in range(L // B[1]):
        for bx in range(L // B[0]):
            rows, cols = oracle_lib.block_region(B, origin, bx, by, L)
            bsx = np.ascontiguousarray(before.sx[np.ix_(rows, cols)])
            bsy = np.ascontiguousarray(before.sy[np.ix_(rows, cols)])
            total += oracle_lib.dd_block_mcs(L, p, q, seed, B, t, bx, by, bsx, bsy)
            assert np.array_equal(bsx, st.sx[np.ix_(rows, cols)])
            assert np.array_equal(bsy, st.sy[np.ix_(rows, cols)])
    assert total == int(st.net[0] - before.net[0])


# ------------------------------------- origin moves within an MCS (tau < 1)

@pytest.mark.parametrize("block,tile,moves", [((4, 2), (2, 2), 4), ((4, 2), (2, 2), 2),
                                              ((2, 2), (2, 2), 4)])
def test_dd_moves_matches_exact_law(oracle_lib, chain4, block, tile, moves):
    """With the origin moved `moves` times per MCS, the oracle's law of W^2
    after two MCS equals the exact law of that schedule (independent uniform
    origin per residency, S/moves single-hit steps each)."""
    p, q, t = 1.0, 0.0, 2
    pi_t = chain4.distribution(chain4.dd_mcs(p, q, block, tile, moves), t)
    n = 3000
    counts = np.zeros(chain4.n)
    for i in range(n):
        st = oracle_lib.SlopeState(4).run_dd(t, p, q, 15000 + i, block=block, tile=tile,
                                             moves=moves)
        counts[chain4.index[exact_small.state_from_slopes(st.sx, st.sy)]] += 1
    keys = np.round(chain4.w2, 12)
    uniq = np.unique(keys)
    obs = np.array([counts[keys == k].sum() for k in uniq])
    exp = np.array([pi_t[keys == k].sum() for k in uniq]) * n
    big = exp >= 5
    o2 = np.append(obs[big], obs[~big].sum())
    e2 = np.append(exp[big], exp[~big].sum())
    keep = e2 > 0
    chi2 = (((o2[keep] - e2[keep]) ** 2) / e2[keep]).sum()
    dof = keep.sum() - 1
    assert chi2 < dof + 4.5 * np.sqrt(2 * dof) + 10, (chi2, dof)


def test_exact_moves_changes_the_law(chain4):
    """With dead borders the residency is part of the dynamics: one origin
    per MCS and several give clearly different laws at t = 2 (so the test
    above tells them apart).  A single periodic block with one tile is RS
    whatever the residency."""
    for block, moves in (((2, 2), 4), ((4, 2), 2)):
        a = chain4.distribution(chain4.dd_mcs(1.0, 0.0, block, (2, 2), 1), 2)
        b = chain4.distribution(chain4.dd_mcs(1.0, 0.0, block, (2, 2), moves), 2)
        assert np.abs(a - b).sum() > 0.3, block
    a = chain4.dd_mcs(1.0, 0.0, (4, 4), (4, 4), 4)
    assert np.allclose(a, chain4.rs_mcs(1.0, 0.0))


@pytest.mark.parametrize("moves", [2, 16])
def test_dd_moves_attempts_never_neighbours(oracle_lib, moves):
    oracle_lib.SlopeState(32).run_dd(3, 0.5, 0.5, 23, block=(16, 8), check=True, moves=moves)


def test_dd_moves_conjugation_and_invariants(oracle_lib):
    L = 32
    a = oracle_lib.SlopeState(L).run_rs(2, 0.9, 0.1, 99)
    b = _negated(a)
    a.run_dd(5, 1.0, 0.25, 8, block=(16, 8), moves=4)
    b.run_dd(5, 0.25, 1.0, 8, block=(16, 8), moves=4)
    assert np.array_equal(b.sx, -a.sx) and np.array_equal(b.sy, -a.sy)
    assert b.h00[0] == -a.h00[0] and b.net[0] == -a.net[0]
    oracle_lib.check_invariants(a.sx, a.sy)


def test_dd_moves_one_is_the_default_schedule(oracle_lib):
    a = oracle_lib.SlopeState(32).run_dd(4, 1.0, 0.3, 6, block=(16, 16))
    b = oracle_lib.SlopeState(32).run_dd(4, 1.0, 0.3, 6, block=(16, 16), moves=1)
    c = oracle_lib.SlopeState(32).run_dd(4, 1.0, 0.3, 6, block=(16, 16), moves=2)
    assert np.array_equal(a.sx, b.sx) and np.array_equal(a.sy, b.sy)
    assert not (np.array_equal(a.sx, c.sx) and np.array_equal(a.sy, c.sy))


@pytest.mark.parametrize("moves", [2, 8])
def test_block_runner_residencies_equal_full_run(oracle_lib, moves):
    """Residency by residency, blocks on their own copies (each residency's
    blocks from its own origin) reproduce the whole-lattice MCS."""
    L, B, seed, p, q = 64, (32, 16), 3, 1.0, 0.4
    st = oracle_lib.SlopeState(L).run_dd(1, p, q, seed, block=B, moves=moves)
    t = st.t
    cur = st.copy()
    net_before = int(cur.net[0])
    st.run_dd(1, p, q, seed, block=B, moves=moves)
    total = 0
    for res in range(moves):
        origin = oracle_lib.dd_origin(seed, t, B, res)
        nxt = cur.copy()
        for by in range(L // B[1]):
            for bx in range(L // B[0]):
                rows, cols = oracle_lib.block_region(B, origin, bx, by, L)
                bsx = np.ascontiguousarray(cur.sx[np.ix_(rows, cols)])
                bsy = np.ascontiguousarray(cur.sy[np.ix_(rows, cols)])
                total += oracle_lib.dd_block_mcs(L, p, q, seed, B, t, bx, by, bsx, bsy,
                                                 moves=moves, res=res)
                nxt.sx[np.ix_(rows, cols)] = bsx
                nxt.sy[np.ix_(rows, cols)] = bsy
        cur = nxt
    assert np.array_equal(cur.sx, st.sx) and np.array_equal(cur.sy, st.sy)
    assert total == int(st.net[0]) - net_before
