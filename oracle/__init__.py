"""CPU oracle for the 2+1-d KPZ octahedron model -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never imports it, and
the two share no code.

The arithmetic lives in plain C (``kpz_oracle.c``, compiled with gcc); this
module adds the plain numpy definitions of the observables of Sec. 2.1:

* heights reconstructed from the slopes by summing them along a path from the
  anchor site (0, 0) (the height-reconstruction equation of Sec. 2.1, read as
  a path sum; see ``heights``),
* the moments S1 = sum h and S2 = sum h^2 as exact Python integers,
* the squared width W^2 = S2/N - (S1/N)^2 with N = L^2 (eq. ``Wdef``, the
  second term read with the 1/L^2 normalisation; the flat start then gives
  exactly 1/4).

The packed word format (16 sites per uint32, bit 2k = sigma_x > 0 and bit
2k+1 = sigma_y > 0 for site x = 16 w + k of a row) is written out here
independently of the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kpz_oracle.c")
SRC_KMC = os.path.join(HERE, "kmc_oracle.c")
LIB = os.path.join(HERE, "_build", "libkpz_oracle.so")

OR_OK, OR_EINVAL, OR_ENOMEM, OR_ECHECK = 0, -1, -2, -3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/_build``."""
    stale = not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(SRC),
                                                                    os.path.getmtime(SRC_KMC))
    if force or stale:
        os.makedirs(os.path.dirname(LIB), exist_ok=True)
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared",
                               "-fPIC", "-fopenmp", "-o", tmp, SRC, SRC_KMC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = ctypes.CDLL(LIB)
        i8p = np.ctypeslib.ndpointer(np.int8, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        c = ctypes
        L.or_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.or_philox4x32_r.argtypes = [u32p, u32p, ctypes.c_int, u32p]
        L.or_tag_rounds.argtypes = [ctypes.c_uint32]
        L.or_tag_rounds.restype = ctypes.c_int
        L.or_draw.argtypes = [c.c_uint64, c.c_uint32, c.c_uint32, c.c_uint64, c.c_uint32, u32p]
        L.or_flat.argtypes = [c.c_int, i8p, i8p]
        L.or_rs_heights_run.argtypes = [c.c_int, c.c_double, c.c_double, c.c_uint64,
                                        c.c_uint32, c.c_int, i64p]
        L.or_rs_slopes_run.argtypes = [c.c_int, c.c_double, c.c_double, c.c_uint64,
                                       c.c_uint32, c.c_int, i8p, i8p, i64p, i64p]
        L.or_dd_run.argtypes = [c.c_int, c.c_double, c.c_double, c.c_uint64,
                                c.c_int, c.c_int, c.c_int, c.c_int, c.c_int,
                                c.c_uint32, c.c_int, i8p, i8p, i64p, i64p, c.c_int]
        L.or_dd_run_par.argtypes = [c.c_int, c.c_double, c.c_double, c.c_uint64,
                                    c.c_int, c.c_int, c.c_int, c.c_int, c.c_int,
                                    c.c_uint32, c.c_int, i8p, i8p, i64p, i64p, c.c_int]
        L.or_strat_run.argtypes = [c.c_int, c.c_double, c.c_double, c.c_uint64, c.c_int,
                                   c.c_int, c.c_uint32, c.c_int, i8p, i8p, i64p, i64p]
        L.or_rs1d_run.argtypes = [c.c_int, c.c_double, c.c_double, c.c_uint64,
                                  c.c_uint32, c.c_int, i8p, i64p, i64p]
        L.or_dd_block_mcs.argtypes = [c.c_int, c.c_double, c.c_double, c.c_uint64,
                                      c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_uint32,
                                      c.c_int, c.c_int, c.c_int, i8p, i8p, i64p]
        L.or_dd_origin.argtypes = [c.c_uint64, c.c_uint32, c.c_int, c.c_int, c.c_int,
                                   c.POINTER(c.c_int), c.POINTER(c.c_int)]
        L.or_dd_origin.restype = None
        L.or_dd1d_run.argtypes = [c.c_int, c.c_double, c.c_double, c.c_uint64, c.c_int,
                                  c.c_uint32, c.c_int, i8p, i64p, i64p, c.c_int]
        L.or_dd1d_block_mcs.argtypes = [c.c_int, c.c_double, c.c_double, c.c_uint64, c.c_int,
                                        c.c_uint32, c.c_int, i8p, i64p]
        L.or_dd1d_origin.argtypes = [c.c_uint64, c.c_uint32, c.c_int]
        L.or_flat1d.argtypes = [c.c_int, i8p]
        L.or_dt_run.argtypes = [c.c_int, c.c_double, c.c_double, c.c_uint64,
                                c.c_int, c.c_int, c.c_int, c.c_int,
                                c.c_uint32, c.c_int, i8p, i8p, i64p, i64p, c.c_int, c.c_int]
        L.or_dt_perm.argtypes = [c.c_uint64, c.c_uint32, c.POINTER(c.c_int * 4)]
        for f in ("or_flat", "or_rs_heights_run", "or_rs_slopes_run", "or_dd_run", "or_dd_run_par",
                  "or_strat_run",
                  "or_rs1d_run",
                  "or_dd_block_mcs", "or_dd1d_run", "or_dd1d_block_mcs", "or_dd1d_origin",
                  "or_flat1d", "or_dt_run", "or_dt_perm"):
            getattr(L, f).restype = c.c_int
        _lib = L
    return _lib


def _check(rc: int, what: str) -> None:
    if rc != OR_OK:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


# ----------------------------------------------------------------- Philox

def philox(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def philox_rounds(ctr, key, rounds: int) -> np.ndarray:
    """Philox4x32 with the given number of rounds (philox() is rounds = 10)."""
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_r(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), int(rounds),
                          out)
    return out


def tag_rounds(tag: int) -> int:
    """Philox rounds of a draw tag: 7 for the 2+1-d lattice dynamics, 10
    for the ring and KMC."""
    return int(lib().or_tag_rounds(int(tag)))


def draw(seed: int, tag: int, t: int, idx: int, sub: int) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().or_draw(seed, tag, t, idx, sub, out)
    return out


TAG_ORIGIN, TAG_SET, TAG_SITE, TAG_ACC1, TAG_ACC2, TAG_RS, TAG_RS1D = 1, 2, 3, 4, 5, 6, 7
TAG_ORIGIN1D, TAG_SET1D, TAG_SITE1D, TAG_ACC1D, TAG_ACC1D2 = 8, 9, 10, 11, 12
TAG_DTORDER = 13


# ------------------------------------------------------------------ state

class SlopeState:
    """Unpacked slope state: sx, sy int8 arrays of shape (L, L) indexed
    [y, x]; h00 = h(0, 0); net = (#deposits - #desorptions) so far; t = next
    MCS index."""

    def __init__(self, L: int):
        self.L = L
        self.sx = np.zeros((L, L), np.int8)
        self.sy = np.zeros((L, L), np.int8)
        self.h00 = np.zeros(1, np.int64)
        self.net = np.zeros(1, np.int64)
        self.t = 0
        _check(lib().or_flat(L, self.sx, self.sy), "flat")

    def copy(self) -> "SlopeState":
        o = SlopeState.__new__(SlopeState)
        o.L, o.t = self.L, self.t
        o.sx, o.sy = self.sx.copy(), self.sy.copy()
        o.h00, o.net = self.h00.copy(), self.net.copy()
        return o

    # dynamics
    def run_dd(self, n_mcs: int, p: float, q: float, seed: int, block=(None, None),
               tile=(4, 4), check: bool = False, moves: int = 1,
               threads: int = 0) -> "SlopeState":
        """n_mcs MCS of the decomposed schedule; ``moves`` = origin moves
        per MCS (block residency 1/moves MCS).  ``threads`` > 0 runs the
        blocks of each residency in parallel (or_dd_run_par, same result;
        no neighbour check)."""
        bx = block[0] or self.L
        by = block[1] or self.L
        if threads > 0:
            assert not check, "the parallel runner has no neighbour check"
            rc = lib().or_dd_run_par(self.L, p, q, seed, bx, by, tile[0], tile[1], moves,
                                     self.t, n_mcs, self.sx, self.sy, self.h00, self.net,
                                     int(threads))
        else:
            rc = lib().or_dd_run(self.L, p, q, seed, bx, by, tile[0], tile[1], moves, self.t,
                                 n_mcs, self.sx, self.sy, self.h00, self.net, int(check))
        _check(rc, "dd_run")
        self.t += n_mcs
        return self

    def run_dt(self, n_mcs: int, p: float, q: float, seed: int, block, tile=(4, 4),
               check: bool = False, ahead: int = 0) -> "SlopeState":
        """n_mcs MCS with double tiling at the device layer too (the four
        block sets in a random order per MCS, no dead border).  ahead = 1: a
        set whose successor in the order is its diagonal partner runs
        together with it, the two interleaved step by step (Sec. 3.2,
        blocks updated ahead of time); exactly the plain result.  ahead = 2
        pairs x-neighbour sets the same way, which is not exact (a negative
        control for the tests)."""
        rc = lib().or_dt_run(self.L, p, q, seed, block[0], block[1], tile[0], tile[1], self.t,
                             n_mcs, self.sx, self.sy, self.h00, self.net, int(check),
                             int(ahead))   # 2: the x-neighbour control (not exact)
        _check(rc, "dt_run")
        self.t += n_mcs
        return self

    def run_strat(self, n_mcs: int, p: float, q: float, seed: int, tile=(4, 4)) -> "SlopeState":
        """n_mcs MCS of the stratified random-sequential control: exactly
        Tx*Ty attempts per tile per MCS in a random global order."""
        rc = lib().or_strat_run(self.L, p, q, seed, tile[0], tile[1], self.t, n_mcs, self.sx,
                                self.sy, self.h00, self.net)
        _check(rc, "strat_run")
        self.t += n_mcs
        return self

    def run_rs(self, n_mcs: int, p: float, q: float, seed: int) -> "SlopeState":
        rc = lib().or_rs_slopes_run(self.L, p, q, seed, self.t, n_mcs, self.sx, self.sy,
                                    self.h00, self.net)
        _check(rc, "rs_slopes_run")
        self.t += n_mcs
        return self

    # observables
    def heights(self) -> np.ndarray:
        return heights(self.sx, self.sy, int(self.h00[0]))

    def moments(self):
        return moments(self.heights())


def dt_perm(seed: int, t: int):
    """Order of the four block sets in MCS t (double tiling at the device layer)."""
    arr = (ctypes.c_int * 4)()
    lib().or_dt_perm(seed, t, ctypes.byref(arr))
    return list(arr)


def flat_heights(L: int) -> np.ndarray:
    y, x = np.mgrid[0:L, 0:L]
    return ((x + y) & 1).astype(np.int64)


def rs_heights_run(h: np.ndarray, t0: int, n_mcs: int, p: float, q: float, seed: int) -> np.ndarray:
    L = h.shape[0]
    h = np.ascontiguousarray(h, np.int64)
    _check(lib().or_rs_heights_run(L, p, q, seed, t0, n_mcs, h), "rs_heights_run")
    return h


def dd_origin(seed: int, t: int, block, res: int = 0) -> tuple:
    """Block origin of residency ``res`` of MCS t."""
    ox, oy = ctypes.c_int(), ctypes.c_int()
    lib().or_dd_origin(seed, t, res, block[0], block[1], ctypes.byref(ox), ctypes.byref(oy))
    return ox.value, oy.value


def dd_block_mcs(L: int, p: float, q: float, seed: int, block, t: int, bx: int, by: int,
                 bsx: np.ndarray, bsy: np.ndarray, moves: int = 1, res: int = 0) -> int:
    """Residency ``res`` of MCS t (the whole MCS when moves = 1) of block
    (bx, by) on its own slopes (arrays of shape (By, Bx), modified in
    place); returns the net number of flips."""
    net = np.zeros(1, np.int64)
    _check(lib().or_dd_block_mcs(L, p, q, seed, block[0], block[1], 4, 4, moves, t, res, bx, by,
                                 bsx, bsy, net), "dd_block_mcs")
    return int(net[0])


def block_region(block, origin, bx: int, by: int, L: int):
    """Global (rows, cols) index vectors of block (bx, by) for a given origin."""
    rows = (origin[1] + by * block[1] + np.arange(block[1])) % L
    cols = (origin[0] + bx * block[0] + np.arange(block[0])) % L
    return rows, cols


def rs1d_run(s: np.ndarray, h0: np.ndarray, net: np.ndarray, t0: int, n_mcs: int,
             p: float, q: float, seed: int) -> None:
    _check(lib().or_rs1d_run(s.shape[0], p, q, seed, t0, n_mcs, s, h0, net), "rs1d_run")


class RingState:
    """The 1+1-d rooftop ring: bonds s[i] = h(i+1) - h(i) in {-1, +1}
    (int8, length L), anchor h0 = h(0), net flips, next MCS t."""

    def __init__(self, L: int):
        self.L = L
        self.s = np.zeros(L, np.int8)
        self.h0 = np.zeros(1, np.int64)
        self.net = np.zeros(1, np.int64)
        self.t = 0
        _check(lib().or_flat1d(L, self.s), "flat1d")

    def copy(self) -> "RingState":
        o = RingState.__new__(RingState)
        o.L, o.t = self.L, self.t
        o.s, o.h0, o.net = self.s.copy(), self.h0.copy(), self.net.copy()
        return o

    def run_rs(self, n_mcs: int, p: float, q: float, seed: int) -> "RingState":
        rs1d_run(self.s, self.h0, self.net, self.t, n_mcs, p, q, seed)
        self.t += n_mcs
        return self

    def run_dd(self, n_mcs: int, p: float, q: float, seed: int, block: int,
               check: bool = False) -> "RingState":
        _check(lib().or_dd1d_run(self.L, p, q, seed, block, self.t, n_mcs, self.s, self.h0,
                                 self.net, int(check)), "dd1d_run")
        self.t += n_mcs
        return self

    def heights(self) -> np.ndarray:
        h = np.zeros(self.L, np.int64)
        h[1:] = np.cumsum(self.s[:-1].astype(np.int64))
        return h + int(self.h0[0])

    def moments(self):
        """Exact (S1, S2) = (sum h, sum h^2) as Python ints."""
        h = self.heights()
        return int(h.sum()), int(sum(int(v) * int(v) for v in h))


def pack1d(s: np.ndarray) -> np.ndarray:
    """Bond i -> bit i mod 32 of word i / 32 (1 = +1)."""
    bits = (np.asarray(s) > 0).astype(np.uint64).reshape(-1, 32)
    return (bits << np.arange(32, dtype=np.uint64)).sum(axis=1).astype(np.uint32)


def unpack1d(words: np.ndarray) -> np.ndarray:
    w = np.asarray(words, np.uint32).astype(np.uint64)
    bits = (w[:, None] >> np.arange(32, dtype=np.uint64)) & 1
    return (2 * bits.reshape(-1).astype(np.int8) - 1).astype(np.int8)


def dd1d_origin(seed: int, t: int, block: int) -> int:
    return int(lib().or_dd1d_origin(seed, t, block))


def dd1d_block_mcs(L: int, p: float, q: float, seed: int, block: int, t: int, b: int,
                   bs: np.ndarray) -> int:
    """One MCS of block b of the 1+1-d schedule on its own bonds ``bs``
    (length block, modified in place); returns the net number of flips."""
    net = np.zeros(1, np.int64)
    _check(lib().or_dd1d_block_mcs(L, p, q, seed, block, t, b, bs, net), "dd1d_block_mcs")
    return int(net[0])


# ------------------------------------------------------------ observables

def heights(sx: np.ndarray, sy: np.ndarray, h00: int = 0) -> np.ndarray:
    """h(x, y) = h00 + sum_{k<y} sigma_y(0, k) + sum_{l<x} sigma_x(l, y): the
    path from (0,0) up column 0, then along row y."""
    sx = sx.astype(np.int64)
    sy = sy.astype(np.int64)
    col0 = np.concatenate([[0], np.cumsum(sy[:-1, 0])])
    row = np.concatenate([np.zeros((sx.shape[0], 1), np.int64), np.cumsum(sx[:, :-1], axis=1)],
                         axis=1)
    return h00 + col0[:, None] + row


def heights_rowfirst(sx: np.ndarray, sy: np.ndarray, h00: int = 0) -> np.ndarray:
    """The other path: along row 0 first, then up column x."""
    sx = sx.astype(np.int64)
    sy = sy.astype(np.int64)
    row0 = np.concatenate([[0], np.cumsum(sx[0, :-1])])
    col = np.concatenate([np.zeros((1, sy.shape[1]), np.int64), np.cumsum(sy[:-1, :], axis=0)],
                         axis=0)
    return h00 + row0[None, :] + col


def slopes_from_heights(h: np.ndarray):
    sx = (np.roll(h, -1, axis=1) - h).astype(np.int8)
    sy = (np.roll(h, -1, axis=0) - h).astype(np.int8)
    return sx, sy


def moments(h: np.ndarray):
    """Exact (S1, S2) as Python integers."""
    S1 = int(h.sum(dtype=np.int64))
    S2 = sum(int(v) for v in (h.astype(np.int64) ** 2).sum(axis=1, dtype=np.int64))
    return S1, S2


def w2_exact(S1: int, S2: int, N: int) -> Fraction:
    return Fraction(N * S2 - S1 * S1, N * N)


def w2(S1: int, S2: int, N: int) -> float:
    return float(w2_exact(S1, S2, N))


# ------------------------------------------------------------ packed words

def pack(sx: np.ndarray, sy: np.ndarray) -> np.ndarray:
    """(L, L) slopes -> (L, L/16) uint32 words."""
    L = sx.shape[0]
    bx = (sx > 0).astype(np.uint64).reshape(L, L // 16, 16)
    by = (sy > 0).astype(np.uint64).reshape(L, L // 16, 16)
    k = np.arange(16, dtype=np.uint64)
    words = ((bx << (2 * k)) | (by << (2 * k + 1))).sum(axis=2)
    return words.astype(np.uint32)


def unpack(words: np.ndarray, L: int):
    w = np.asarray(words, np.uint32).reshape(L, L // 16).astype(np.uint64)
    k = np.arange(16, dtype=np.uint64)
    bx = (w[:, :, None] >> (2 * k)) & 1
    by = (w[:, :, None] >> (2 * k + 1)) & 1
    sx = (2 * bx.astype(np.int8) - 1).reshape(L, L)
    sy = (2 * by.astype(np.int8) - 1).reshape(L, L)
    return sx.astype(np.int8), sy.astype(np.int8)


# ------------------------------------------------------------- invariants

def check_invariants(sx: np.ndarray, sy: np.ndarray) -> None:
    """Raises AssertionError unless the slopes are a valid surface: values in
    {-1,+1}, zero circulation around every plaquette, zero sum along every
    periodic row (sigma_x) and column (sigma_y)."""
    assert set(np.unique(sx)) <= {-1, 1} and set(np.unique(sy)) <= {-1, 1}
    sx64 = sx.astype(np.int64)
    sy64 = sy.astype(np.int64)
    curl = sx64 + np.roll(sy64, -1, axis=1) - np.roll(sx64, -1, axis=0) - sy64
    assert not curl.any(), "plaquette circulation"
    assert not sx64.sum(axis=1).any(), "row sum of sigma_x"
    assert not sy64.sum(axis=0).any(), "column sum of sigma_y"


def invariant_counts(sx: np.ndarray, sy: np.ndarray) -> tuple:
    """(open plaquettes, sum of sigma_x along row 0, sum of sigma_y along
    column 0) of a slope field, from the definitions of Sec. 2.1: a
    plaquette is closed when the two paths from (x, y) to (x+1, y+1) have the
    same height change.  All three are zero for a valid surface (with every
    plaquette closed, every row and column carries the sums of row 0 and
    column 0)."""
    sx64 = sx.astype(np.int64)
    sy64 = sy.astype(np.int64)
    right_then_up = sx64 + np.roll(sy64, -1, axis=1)
    up_then_right = sy64 + np.roll(sx64, -1, axis=0)
    return (int(np.count_nonzero(right_then_up != up_then_right)), int(sx64[0, :].sum()),
            int(sy64[:, 0].sum()))
