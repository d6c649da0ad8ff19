"""Pins of the exact small-lattice law and of the invariant checker against
values fixed outside the oracle (CPU only).

* ``tests/golden/exact_4x4_rs.json``: the random-sequential law on the 4 x 4
  torus (E[W^2] after t MCS, stationary W^2, stationary velocity), computed
  by an independent enumeration (Sec. 2.1 eq. ``rule``, Sec. 2.2, eq.
  ``Wdef``).
* Brute force: the zero-tilt height functions of the 4 x 4 torus, counted
  and averaged here with their own depth-first search, give the uniform
  law's mean W^2 = 92/165 exactly (the stationary law at p = q).
* The slope-consistency checker rejects surfaces that break each of its
  conditions (Sec. 2.1: slopes are +-1 and sum to zero around every
  plaquette and along every periodic row and column).
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact_small

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "exact_4x4_rs.json")


@pytest.fixture(scope="module")
def chain4():
    return exact_small.SmallChain(4)


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_rs_law_matches_golden(chain4, golden):
    tol = 1e-9   # the fixture holds 10 decimals
    for case in golden["cases"]:
        p, q = case["p"], case["q"]
        T = chain4.rs_mcs(p, q)
        times = [int(t) for t in case["E_W2"]]
        got = chain4.expected_w2(T, times)
        for t in times:
            assert got[t] == pytest.approx(case["E_W2"][str(t)], abs=tol), (p, q, t)
        pi = chain4.stationary(T)
        assert float(pi @ chain4.w2) == pytest.approx(case["stationary_W2"], abs=tol), (p, q)
        assert chain4.rs_velocity(pi, p, q) == pytest.approx(case["velocity"], abs=tol), (p, q)


def _height_functions_4x4():
    """All h on the 4 x 4 torus with h(0,0) = 0 and |h(n) - h(m)| = 1 on
    every edge, by depth-first search over the sites in row-major order."""
    L = 4
    h = [None] * (L * L)
    out = []

    def nbrs(i):
        x, y = i % L, i // L
        return [((x + 1) % L) + y * L, ((x - 1) % L) + y * L,
                x + ((y + 1) % L) * L, x + ((y - 1) % L) * L]

    def rec(i):
        if i == L * L:
            out.append(list(h))
            return
        cands = [0] if i == 0 else None
        for j in nbrs(i):
            if h[j] is not None:
                c = {h[j] - 1, h[j] + 1}
                cands = c if cands is None else (set(cands) & c)
        for v in sorted(cands):
            h[i] = v
            rec(i + 1)
        h[i] = None

    rec(0)
    return out


def test_uniform_law_mean_width_brute_force(chain4, golden):
    hs = _height_functions_4x4()
    assert len(hs) == 990 == chain4.n
    N = 16
    total = Fraction(0)
    for h in hs:
        S1, S2 = sum(h), sum(v * v for v in h)
        total += Fraction(N * S2 - S1 * S1, N * N)
    mean = total / len(hs)
    assert mean == Fraction(92, 165)
    case = next(c for c in golden["cases"] if c["p"] == c["q"])
    assert Fraction(case["stationary_W2_exact"]) == mean
    # and the exact chain's stationary law at p = q carries the same mean
    pi = chain4.stationary(chain4.rs_mcs(0.5, 0.5))
    assert float(pi @ chain4.w2) == pytest.approx(float(mean), abs=1e-13)


# ------------------------------------------------- the invariant checker

def _valid_surface(oracle_lib, L=8, n=3, seed=4):
    st = oracle_lib.SlopeState(L).run_rs(n, 1.0, 0.3, seed)
    oracle_lib.check_invariants(st.sx, st.sy)
    return st.sx.copy(), st.sy.copy()


def test_checker_accepts_valid_surfaces(oracle_lib):
    _valid_surface(oracle_lib)
    st = oracle_lib.SlopeState(16)
    oracle_lib.check_invariants(st.sx, st.sy)


def test_checker_rejects_one_flipped_slope(oracle_lib):
    sx, sy = _valid_surface(oracle_lib)
    sx[3, 5] = -sx[3, 5]
    with pytest.raises(AssertionError):
        oracle_lib.check_invariants(sx, sy)
    sx, sy = _valid_surface(oracle_lib)
    sy[6, 1] = -sy[6, 1]
    with pytest.raises(AssertionError):
        oracle_lib.check_invariants(sx, sy)


def test_checker_rejects_a_tilted_plane(oracle_lib):
    """A plane tilted along y: zero circulation everywhere, but the column
    sums of sigma_y are L (not periodic); likewise along x."""
    L = 8
    x = np.arange(L)
    sx = np.tile(np.where(x % 2 == 0, 1, -1), (L, 1)).astype(np.int8)
    sy = np.ones((L, L), np.int8)
    sx64, sy64 = sx.astype(np.int64), sy.astype(np.int64)
    curl = sx64 + np.roll(sy64, -1, axis=1) - np.roll(sx64, -1, axis=0) - sy64
    assert not curl.any()
    with pytest.raises(AssertionError, match="column sum"):
        oracle_lib.check_invariants(sx, sy)
    with pytest.raises(AssertionError, match="row sum"):
        oracle_lib.check_invariants(sy.T.copy(), sx.T.copy())


def test_checker_rejects_values_other_than_plus_minus_one(oracle_lib):
    sx, sy = _valid_surface(oracle_lib)
    sx[0, 0] = 0
    with pytest.raises(AssertionError):
        oracle_lib.check_invariants(sx, sy)
    sx, sy = _valid_surface(oracle_lib)
    sy[2, 2] = 3
    with pytest.raises(AssertionError):
        oracle_lib.check_invariants(sx, sy)


# ------------------------------------------------- the invariant counts

def test_counts_zero_on_valid_surfaces(oracle_lib):
    sx, sy = _valid_surface(oracle_lib, L=16, n=5)
    assert oracle_lib.invariant_counts(sx, sy) == (0, 0, 0)
    st = oracle_lib.SlopeState(32)
    assert oracle_lib.invariant_counts(st.sx, st.sy) == (0, 0, 0)


def test_counts_of_one_flipped_bond(oracle_lib):
    """A flipped sigma_x bond borders exactly two plaquettes (the one above
    it and the one below it), a flipped sigma_y bond the one to its left and
    the one to its right; the row or column sum moves by 2 when the bond
    lies in row 0 or column 0.  Bonds on the periodic edges included."""
    L = 16
    for (y, x) in [(3, 5), (0, 7), (L - 1, L - 1), (0, 0), (9, 15), (9, 16 % L)]:
        sx, sy = _valid_surface(oracle_lib, L=L)
        sx[y, x] = -sx[y, x]
        open_, r0, c0 = oracle_lib.invariant_counts(sx, sy)
        assert open_ == 2
        assert r0 == (2 * sx[0, x] if y == 0 else 0)
        assert c0 == 0
        sx, sy = _valid_surface(oracle_lib, L=L)
        sy[y, x] = -sy[y, x]
        open_, r0, c0 = oracle_lib.invariant_counts(sx, sy)
        assert open_ == 2
        assert r0 == 0
        assert c0 == (2 * sy[y, 0] if x == 0 else 0)


def test_counts_of_a_tilted_plane(oracle_lib):
    """A plane tilted along y closes every plaquette but sums to L along
    every column."""
    L = 8
    x = np.arange(L)
    sx = np.tile(np.where(x % 2 == 0, 1, -1), (L, 1)).astype(np.int8)
    sy = np.ones((L, L), np.int8)
    assert oracle_lib.invariant_counts(sx, sy) == (0, 0, L)
    assert oracle_lib.invariant_counts(sy.T.copy(), sx.T.copy()) == (0, L, 0)


def test_counts_agree_with_the_checker(oracle_lib):
    """Random +-1 perturbations: the counts are all zero exactly when the
    checker accepts the surface."""
    rng = np.random.default_rng(7)
    for trial in range(40):
        sx, sy = _valid_surface(oracle_lib, L=8, n=2, seed=trial + 1)
        for _ in range(int(rng.integers(0, 3))):
            a = sx if rng.integers(2) else sy
            i, j = rng.integers(8, size=2)
            a[i, j] = -a[i, j]
        zero = oracle_lib.invariant_counts(sx, sy) == (0, 0, 0)
        try:
            oracle_lib.check_invariants(sx, sy)
            ok = True
        except AssertionError:
            ok = False
        assert zero == ok
