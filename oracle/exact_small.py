"""Exact master-equation law of the octahedron model on tiny tori -- TEST
INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

All zero-tilt surfaces of the L x L torus (L = 4: a few hundred states) are
enumerated, and the one-MCS transition matrix is built

* for random-sequential dynamics: one attempt picks a uniform site and
  applies the rule of Sec. 2.1 (eq. ``rule``: minimum -> maximum with
  probability p, maximum -> minimum with probability q); one MCS is N = L^2
  attempts (Sec. 2.2);
* for the decomposed schedule of Sec. 3 / 3.1: uniform dead-border origin,
  then S = Tx*Ty single-hit steps, each with a uniform set and, in every
  tile, a uniform site of that set's cell; attempts at dead-border sites do
  nothing.  The cells of one set do not interact, so a step is the product
  of the per-cell single-site operators.

From these the exact E[W^2](t) from the flat start, the stationary law and
the stationary mean height velocity follow by linear algebra.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def _site_bits(L):
    return L * L


def state_from_slopes(sx: np.ndarray, sy: np.ndarray) -> int:
    L = sx.shape[0]
    code = 0
    for y in range(L):
        for x in range(L):
            i = y * L + x
            if sx[y, x] > 0:
                code |= 1 << i
            if sy[y, x] > 0:
                code |= 1 << (L * L + i)
    return code


def slopes_from_state(code: int, L: int):
    sx = np.empty((L, L), np.int8)
    sy = np.empty((L, L), np.int8)
    for y in range(L):
        for x in range(L):
            i = y * L + x
            sx[y, x] = 1 if (code >> i) & 1 else -1
            sy[y, x] = 1 if (code >> (L * L + i)) & 1 else -1
    return sx, sy


def _classify(code: int, L: int, x: int, y: int) -> int:
    """+1 local minimum, -1 local maximum, 0 otherwise (slope form of the rule)."""
    N = L * L
    a = (code >> (y * L + x)) & 1                       # sigma_x(x, y) > 0
    b = (code >> (N + y * L + x)) & 1                   # sigma_y(x, y) > 0
    c = (code >> (y * L + (x - 1) % L)) & 1             # sigma_x(x-1, y) > 0
    d = (code >> (N + ((y - 1) % L) * L + x)) & 1       # sigma_y(x, y-1) > 0
    if a and b and not c and not d:
        return 1
    if not a and not b and c and d:
        return -1
    return 0


def _flip(code: int, L: int, x: int, y: int) -> int:
    N = L * L
    m = (1 << (y * L + x)) | (1 << (N + y * L + x)) \
        | (1 << (y * L + (x - 1) % L)) | (1 << (N + ((y - 1) % L) * L + x))
    return code ^ m


def flat_state(L: int) -> int:
    sx = np.empty((L, L), np.int8)
    sy = np.empty((L, L), np.int8)
    for y in range(L):
        for x in range(L):
            h = (x + y) & 1
            sx[y, x] = (((x + 1) + y) & 1) - h
            sy[y, x] = ((x + (y + 1)) & 1) - h
    return state_from_slopes(sx, sy)


def reachable_states(L: int):
    """Breadth-first closure of the flat state under single-site flips."""
    start = flat_state(L)
    seen = {start: 0}
    order = [start]
    head = 0
    while head < len(order):
        s = order[head]
        head += 1
        for y in range(L):
            for x in range(L):
                if _classify(s, L, x, y):
                    n = _flip(s, L, x, y)
                    if n not in seen:
                        seen[n] = len(order)
                        order.append(n)
    return order, seen


def count_height_functions(L: int) -> int:
    """Brute-force count of height functions on the L x L torus with
    h(0,0) = 0 and |h(n) - h(m)| = 1 across every edge (each one is a
    zero-tilt slope configuration), by depth-first assignment site by site."""
    N = L * L
    h = [None] * N
    h[0] = 0
    count = 0

    def ok(i):
        y, x = divmod(i, L)
        for (xx, yy) in (((x - 1) % L, y), ((x + 1) % L, y), (x, (y - 1) % L), (x, (y + 1) % L)):
            j = yy * L + xx
            if h[j] is not None and abs(h[j] - h[i]) != 1:
                return False
        return True

    def rec(i):
        nonlocal count
        if i == N:
            count += 1
            return
        y, x = divmod(i, L)
        # a neighbour already placed fixes h up to +-1
        ref = h[y * L + x - 1] if x > 0 else h[(y - 1) * L + x]
        for v in (ref - 1, ref + 1):
            h[i] = v
            if ok(i):
                rec(i + 1)
            h[i] = None

    rec(1)
    return count


def w2_of_state(code: int, L: int) -> Fraction:
    sx, sy = slopes_from_state(code, L)
    h = np.zeros((L, L), np.int64)
    for y in range(L):
        if y > 0:
            h[y, 0] = h[y - 1, 0] + sy[y - 1, 0]
        for x in range(1, L):
            h[y, x] = h[y, x - 1] + sx[y, x - 1]
    N = L * L
    S1 = int(h.sum())
    S2 = int((h * h).sum())
    return Fraction(N * S2 - S1 * S1, N * N)


class SmallChain:
    """Exact transition matrices on the L x L torus (practical for L = 4)."""

    def __init__(self, L: int = 4):
        self.L = L
        self.N = L * L
        self.states, self.index = reachable_states(L)
        self.n = len(self.states)
        self.w2 = np.array([float(w2_of_state(s, L)) for s in self.states])
        self.w2_frac = None
        # kind[i, site] in {+1 min, -1 max, 0}; target[i, site] = flipped state index
        self.kind = np.zeros((self.n, self.N), np.int8)
        self.target = np.zeros((self.n, self.N), np.int64)
        for i, s in enumerate(self.states):
            for y in range(L):
                for x in range(L):
                    site = y * L + x
                    k = _classify(s, L, x, y)
                    self.kind[i, site] = k
                    self.target[i, site] = self.index[_flip(s, L, x, y)] if k else i
        self.flat = self.index[flat_state(L)]

    def site_operator(self, site: int, p: float, q: float) -> np.ndarray:
        """Row-stochastic matrix of one attempt at ``site``."""
        A = np.zeros((self.n, self.n))
        for i in range(self.n):
            k = self.kind[i, site]
            pr = p if k == 1 else (q if k == -1 else 0.0)
            A[i, i] += 1.0 - pr
            if pr:
                A[i, self.target[i, site]] += pr
        return A

    def rs_mcs(self, p: float, q: float) -> np.ndarray:
        T1 = sum(self.site_operator(s, p, q) for s in range(self.N)) / self.N
        return np.linalg.matrix_power(T1, self.N)

    def dd_mcs(self, p: float, q: float, block, tile, moves: int = 1) -> np.ndarray:
        """Transition matrix of one MCS of the decomposed schedule: per
        residency a uniform random origin, then S/moves single-hit steps
        (each block a uniform set, each tile a uniform site of its cell);
        the MCS is ``moves`` independent residencies (Sec. 3, 3.1)."""
        L = self.L
        Bx, By = block
        Tx, Ty = tile
        nbx, nby = L // Bx, L // By
        ntx, nty = Bx // Tx, By // Ty
        cx, cy = Tx // 2, Ty // 2
        S = Tx * Ty
        ops = {s: self.site_operator(s, p, q) for s in range(self.N)}
        I = np.eye(self.n)
        assert S % moves == 0
        total = np.zeros((self.n, self.n))
        for oy in range(By):
            for ox in range(Bx):
                # each block (work-group) draws its own set; blocks act on
                # disjoint slopes, so the lattice step is the product of the
                # per-block steps
                step = I.copy()
                for by in range(nby):
                    for bx in range(nbx):
                        bstep = np.zeros((self.n, self.n))
                        for st in range(4):
                            ssx, ssy = st & 1, st >> 1
                            M = I.copy()
                            for ty in range(nty):
                                for tx in range(ntx):
                                    cell = np.zeros((self.n, self.n))
                                    for ry in range(cy):
                                        for rx in range(cx):
                                            lx = tx * Tx + ssx * cx + rx
                                            ly = ty * Ty + ssy * cy + ry
                                            if (nbx > 1 and lx == 0) or (nby > 1 and ly == 0):
                                                cell += I
                                            else:
                                                gx = (ox + bx * Bx + lx) % L
                                                gy = (oy + by * By + ly) % L
                                                cell += ops[gy * L + gx]
                                    M = M @ (cell / (cx * cy))
                            bstep += M / 4.0
                        step = step @ bstep
                total += np.linalg.matrix_power(step, S // moves)
        return np.linalg.matrix_power(total / (Bx * By), moves)

    def dt_mcs(self, p: float, q: float, block, tile) -> np.ndarray:
        """One MCS with double tiling at the device layer: uniform origin,
        the four block sets (bx mod 2, by mod 2) in a uniformly random order,
        each block of the active set making S single-hit steps with no dead
        sites (blocks of one set share no slope, so their operators
        commute)."""
        import itertools
        L = self.L
        Bx, By = block
        Tx, Ty = tile
        nbx, nby = L // Bx, L // By
        assert nbx % 2 == 0 and nby % 2 == 0
        ntx, nty = Bx // Tx, By // Ty
        cx, cy = Tx // 2, Ty // 2
        S = Tx * Ty
        ops = {s: self.site_operator(s, p, q) for s in range(self.N)}
        I = np.eye(self.n)
        total = np.zeros((self.n, self.n))
        for oy in range(By):
            for ox in range(Bx):
                block_ops = {}
                for by in range(nby):
                    for bx in range(nbx):
                        bstep = np.zeros((self.n, self.n))
                        for st in range(4):
                            ssx, ssy = st & 1, st >> 1
                            M = I.copy()
                            for ty in range(nty):
                                for tx in range(ntx):
                                    cell = np.zeros((self.n, self.n))
                                    for ry in range(cy):
                                        for rx in range(cx):
                                            lx = tx * Tx + ssx * cx + rx
                                            ly = ty * Ty + ssy * cy + ry
                                            gx = (ox + bx * Bx + lx) % L
                                            gy = (oy + by * By + ly) % L
                                            cell += ops[gy * L + gx]
                                    M = M @ (cell / (cx * cy))
                            bstep += M / 4.0
                        block_ops[(bx, by)] = np.linalg.matrix_power(bstep, S)
                phase = {}
                for c in range(4):
                    M = I.copy()
                    for (bx, by), op in block_ops.items():
                        if (bx & 1) + 2 * (by & 1) == c:
                            M = M @ op
                    phase[c] = M
                for perm in itertools.permutations(range(4)):
                    M = I.copy()
                    for c in perm:
                        M = M @ phase[c]
                    total += M / 24.0
        return total / (Bx * By)

    def expected_w2(self, T: np.ndarray, times) -> dict:
        pi = np.zeros(self.n)
        pi[self.flat] = 1.0
        out = {}
        tmax = max(times)
        for t in range(tmax + 1):
            if t in times:
                out[t] = float(pi @ self.w2)
            pi = pi @ T
        return out

    def distribution(self, T: np.ndarray, t: int) -> np.ndarray:
        pi = np.zeros(self.n)
        pi[self.flat] = 1.0
        for _ in range(t):
            pi = pi @ T
        return pi

    @staticmethod
    def stationary(T: np.ndarray) -> np.ndarray:
        w, v = np.linalg.eig(T.T)
        k = int(np.argmin(np.abs(w - 1.0)))
        pi = np.real(v[:, k])
        return pi / pi.sum()

    def rs_velocity(self, pi: np.ndarray, p: float, q: float) -> float:
        """Stationary mean-height velocity per site per MCS under random-
        sequential updates: each of the N attempts of an MCS changes sum h by
        +2 (prob p at a minimum) or -2 (prob q at a maximum)."""
        nmin = (self.kind == 1).sum(axis=1)
        nmax = (self.kind == -1).sum(axis=1)
        return float(pi @ (2.0 * (p * nmin - q * nmax))) / self.N


class RingChain:
    """Exact law of the 1+1-d rooftop ring of L bonds with zero tilt (the
    reduction of the octahedron model to one dimension, Sec. 2.1): states
    are the bond sequences s in {-1, +1}^L with sum 0; site i touches bonds
    i-1 and i and is a minimum iff (s[i-1], s[i]) = (-1, +1)."""

    def __init__(self, L: int = 8):
        import itertools
        self.L = L
        self.states = [c for c in itertools.product((-1, 1), repeat=L) if sum(c) == 0]
        self.index = {c: i for i, c in enumerate(self.states)}
        self.n = len(self.states)
        self.w2 = np.zeros(self.n)
        for i, c in enumerate(self.states):
            h = np.concatenate([[0], np.cumsum(c[:-1])]).astype(np.int64)
            self.w2[i] = float(Fraction(int(L * (h * h).sum() - h.sum() ** 2), L * L))
        flat = tuple(1 if i % 2 == 0 else -1 for i in range(L))
        self.flat = self.index[flat]

    def site_operator(self, i: int, p: float, q: float) -> np.ndarray:
        L = self.L
        A = np.zeros((self.n, self.n))
        for a, c in enumerate(self.states):
            l, r = c[(i - 1) % L], c[i]
            pr = p if (l, r) == (-1, 1) else (q if (l, r) == (1, -1) else 0.0)
            A[a, a] += 1.0 - pr
            if pr:
                d = list(c)
                d[(i - 1) % L], d[i] = -l, -r
                A[a, self.index[tuple(d)]] += pr
        return A

    def rs_mcs(self, p: float, q: float) -> np.ndarray:
        T1 = sum(self.site_operator(i, p, q) for i in range(self.L)) / self.L
        return np.linalg.matrix_power(T1, self.L)

    def dd_mcs(self, p: float, q: float, block: int) -> np.ndarray:
        """One MCS of the decomposed ring: uniform origin, then 4 single-hit
        steps; in each step every block draws a uniform set (cell of 2
        sites in each 4-site tile) and every tile a uniform site of its
        cell; site 0 of each block is dead when there are several blocks."""
        L, B = self.L, block
        nb = L // B
        ops = {i: self.site_operator(i, p, q) for i in range(L)}
        I = np.eye(self.n)
        total = np.zeros((self.n, self.n))
        for o in range(B):
            step = I.copy()
            for b in range(nb):
                bstep = np.zeros((self.n, self.n))
                for st in range(2):
                    M = I.copy()
                    for m in range(B // 4):
                        cell = np.zeros((self.n, self.n))
                        for r in range(2):
                            lx = 4 * m + 2 * st + r
                            cell += I if (nb > 1 and lx == 0) else ops[(o + b * B + lx) % L]
                        M = M @ (cell / 2.0)
                    bstep += M / 2.0
                step = step @ bstep
            total += np.linalg.matrix_power(step, 4)
        return total / B

    def distribution(self, T: np.ndarray, t: int) -> np.ndarray:
        pi = np.zeros(self.n)
        pi[self.flat] = 1.0
        for _ in range(t):
            pi = pi @ T
        return pi
