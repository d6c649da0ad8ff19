"""Pins of the oracle's double tiling at the device layer (Sec. 3: blocks
bisected in both directions into four sets of non-interacting blocks, the
sets updated in turn in a sequence randomized every MCS; single-hit double
tiling inside each block as for dead borders): the set order is a uniform
permutation, every phase-step's attempts are pairwise non-adjacent,
surfaces stay valid, conjugation symmetry holds bit for bit, and the law of
W^2 on the 4 x 4 torus equals the exact transition matrix of the schedule."""
import itertools

import numpy as np
import pytest

from oracle import exact_small


def test_dt_order_is_a_uniform_permutation(oracle_lib):
    counts = {}
    n = 2400
    for t in range(n):
        perm = tuple(oracle_lib.dt_perm(7, t))
        assert sorted(perm) == [0, 1, 2, 3]
        counts[perm] = counts.get(perm, 0) + 1
    assert len(counts) == 24
    e = n / 24
    chi2 = sum((c - e) ** 2 / e for c in counts.values())
    assert chi2 < 60.0      # chi2(23) at p ~ 1e-4


@pytest.mark.parametrize("L,block,tile", [(32, (8, 8), (4, 4)), (64, (16, 8), (4, 4)),
                                          (16, (4, 4), (2, 2)), (8, (2, 2), (2, 2)),
                                          (64, (32, 16), (4, 4))])
def test_dt_no_conflicts_invariants_mass_balance(oracle_lib, L, block, tile):
    st = oracle_lib.SlopeState(L)
    for p, q in ((1.0, 0.0), (0.6, 0.3)):
        st.run_dt(3, p, q, 5, block, tile, check=True)
        oracle_lib.check_invariants(st.sx, st.sy)
        S1, _ = st.moments()
        assert S1 == L * L // 2 + 2 * int(st.net[0])


def test_dt_rejects_odd_block_counts(oracle_lib):
    st = oracle_lib.SlopeState(48)
    for block in ((16, 16), (48, 8), (8, 48)):      # 3 or 1 blocks along an axis
        with pytest.raises(RuntimeError):
            st.run_dt(1, 1.0, 0.0, 1, block)


def test_dt_conjugation_symmetry(oracle_lib):
    L = 32
    a = oracle_lib.SlopeState(L).run_rs(2, 0.9, 0.1, 99)
    b = a.copy()
    b.sx, b.sy = (-b.sx).astype(np.int8), (-b.sy).astype(np.int8)
    b.h00, b.net = -b.h00, -b.net
    a.run_dt(5, 1.0, 0.25, 8, (8, 16))
    b.run_dt(5, 0.25, 1.0, 8, (8, 16))
    assert np.array_equal(b.sx, -a.sx) and np.array_equal(b.sy, -a.sy)
    assert b.h00[0] == -a.h00[0] and b.net[0] == -a.net[0]


@pytest.fixture(scope="module")
def chain4():
    return exact_small.SmallChain(4)


def test_exact_dt_is_its_own_law(chain4):
    """The device layer matters: on the 4 x 4 torus with 2 x 2 blocks the
    double-tiled law after two MCS differs clearly from the dead-border one,
    and p = q keeps the uniform stationary law."""
    a = chain4.distribution(chain4.dt_mcs(1.0, 0.0, (2, 2), (2, 2)), 2)
    b = chain4.distribution(chain4.dd_mcs(1.0, 0.0, (2, 2), (2, 2)), 2)
    assert np.abs(a - b).sum() > 0.3
    pi = chain4.stationary(chain4.dt_mcs(0.5, 0.5, (2, 2), (2, 2)))
    assert np.allclose(pi, 1.0 / chain4.n, atol=1e-9)


@pytest.mark.parametrize("p,q,t", [(1.0, 0.0, 2), (1.0, 0.375, 3)])
def test_dt_oracle_matches_exact_law(oracle_lib, chain4, p, q, t):
    pi_t = chain4.distribution(chain4.dt_mcs(p, q, (2, 2), (2, 2)), t)
    n = 3000
    counts = np.zeros(chain4.n)
    for i in range(n):
        st = oracle_lib.SlopeState(4).run_dt(t, p, q, 30_000 + i, (2, 2), (2, 2))
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


def test_dt_agrees_with_random_sequential(oracle_lib):
    """L = 128, 48 seeds, p = 1: W^2 within 8 % of random-sequential dynamics
    at t = 8..64 and the growth exponent within 0.03 (the dead-border
    schedule's tolerance, reading R16)."""
    L, seeds, times = 128, 48, [8, 16, 32, 64]
    rs = np.zeros(len(times))
    dt = np.zeros(len(times))
    for s in range(seeds):
        h = oracle_lib.flat_heights(L)
        st = oracle_lib.SlopeState(L)
        t = 0
        for i, T in enumerate(times):
            h = oracle_lib.rs_heights_run(h, t, T - t, 1.0, 0.0, 60_000 + s)
            S1, S2 = oracle_lib.moments(h)
            rs[i] += oracle_lib.w2(S1, S2, L * L) / seeds
            st.run_dt(T - t, 1.0, 0.0, 61_000 + s, (32, 32))
            S1, S2 = st.moments()
            dt[i] += oracle_lib.w2(S1, S2, L * L) / seeds
            t = T
    rel = dt / rs - 1
    b_rs = np.polyfit(np.log(times), np.log(rs), 1)[0] / 2
    b_dt = np.polyfit(np.log(times), np.log(dt), 1)[0] / 2
    print("DT vs RS", np.round(rel, 3), b_dt, b_rs)
    assert np.all(np.abs(rel) < 0.08), rel
    assert abs(b_dt - b_rs) < 0.03


# Blocks of the next set updated ahead of time (Sec. 3.2; Sec. 4, the
# fraction f of full use): a set and its diagonal partner touch no common
# slope, so running them together, interleaved step by step with the
# partner's blocks first, must give the plain schedule's lattice bit for bit.
# Pairing x-neighbour sets the same way must not (the control shows the
# comparison can fail).
@pytest.mark.parametrize("L,block,tile,p,q", [(32, (8, 8), (4, 4), 1.0, 0.0),
                                              (64, (16, 8), (4, 4), 0.6, 0.3),
                                              (64, (32, 16), (4, 4), 1.0, 0.25),
                                              (16, (8, 8), (4, 4), 0.8, 0.1),
                                              (16, (4, 4), (2, 2), 1.0, 0.0),
                                              (8, (2, 2), (2, 2), 0.7, 0.2)])
def test_dt_ahead_equals_plain_schedule(oracle_lib, L, block, tile, p, q):
    n = 24
    merged = sum(any(b == a ^ 3 for a, b in zip(pm, pm[1:]))
                 for pm in (oracle_lib.dt_perm(11, t) for t in range(n)))
    assert merged >= n // 3          # the pairing occurs in about 2/3 of the MCS
    plain = oracle_lib.SlopeState(L).run_dt(n, p, q, 11, block, tile)
    ahead = oracle_lib.SlopeState(L).run_dt(n, p, q, 11, block, tile, check=True, ahead=1)
    assert np.array_equal(plain.sx, ahead.sx) and np.array_equal(plain.sy, ahead.sy)
    assert plain.h00[0] == ahead.h00[0] and plain.net[0] == ahead.net[0]
    ctrl = oracle_lib.SlopeState(L).run_dt(n, p, q, 11, block, tile, ahead=2)
    assert not (np.array_equal(plain.sx, ctrl.sx) and np.array_equal(plain.sy, ctrl.sy))
