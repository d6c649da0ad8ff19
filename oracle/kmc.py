"""CPU oracle for the 3-d KMC binary alloy -- TEST INFRASTRUCTURE ONLY.

Wraps ``kmc_oracle.c`` (Sec. 2.2 "Kinetic Monte Carlo": fcc sub-lattice of
a simple cubic grid, eq. ``fcc``; Metropolis exchange, eq. ``metropolis``
with Gamma = 1; Sec. 3.2 "Implementation of KMC": double tiling at both
layers, both species active).  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may use it.

State: a cubic ``uint8`` array ``occ[z, y, x]`` of shape (L, L, L); fcc
positions ((x ^ y ^ z) & 1 == 0) hold 0 (species A) or 1 (species B), the
other positions hold 0 and are never touched.  ``to_fcc``/``from_fcc``
convert to the compact layout (one byte per fcc site, x fastest, row (y, z)
holding the L/2 sites x = (y + z) % 2 + 2k).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _check, lib as _base_lib

TAG_INIT, TAG_RS, TAG_ORIGIN, TAG_ORDER, TAG_SET, TAG_STEP = 16, 17, 18, 19, 20, 21

_ready = False


def lib():
    global _ready
    L = _base_lib()
    if not _ready:
        c = ctypes
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        L.or_kmc_thresholds.argtypes = [c.c_double, u64p]
        L.or_kmc_thresholds.restype = None
        L.or_kmc_init.argtypes = [c.c_int, c.c_double, c.c_uint64, u8p]
        L.or_kmc_rs_run.argtypes = [c.c_int, c.c_double, c.c_uint64, c.c_uint32, c.c_int, u8p,
                                 c.POINTER(c.c_int64)]
        L.or_kmc_counts.argtypes = [c.c_int, u8p, c.POINTER(c.c_int64), c.POINTER(c.c_int64)]
        L.or_kmc_counts.restype = None
        L.or_kmc_attempt.argtypes = [c.c_int, c.c_double, u8p, c.c_int, c.c_int, c.c_int, c.c_int,
                                  c.c_uint32]
        L.or_kmc_order.argtypes = [c.c_uint64, c.c_uint32, i32p]
        L.or_kmc_order.restype = None
        L.or_kmc_origin.argtypes = [c.c_uint64, c.c_uint32, c.c_int, i32p]
        L.or_kmc_origin.restype = None
        L.or_kmc_dt_run.argtypes = [c.c_int, c.c_double, c.c_uint64, c.c_int, c.c_uint32, c.c_int,
                                 u8p, c.POINTER(c.c_int64), c.c_int, c.c_void_p]
        _ready = True
    return L


def thresholds(eps: float) -> np.ndarray:
    """T[d] = floor(exp(-d eps) 2^32), d = 0..12 (eq. ``metropolis`` as integers)."""
    T = np.zeros(13, np.uint64)
    lib().or_kmc_thresholds(float(eps), T)
    return T


def init(L: int, c: float, seed: int) -> np.ndarray:
    """Homogeneous random mixture: each fcc site is B with probability c."""
    occ = np.zeros((L, L, L), np.uint8)
    _check(lib().or_kmc_init(L, float(c), seed, occ), "or_kmc_init")
    return occ


def rs_run(occ: np.ndarray, eps: float, seed: int, t0: int, n_mcs: int) -> int:
    """Random-sequential dynamics in place; returns the accepted jumps."""
    mv = ctypes.c_int64(0)
    _check(lib().or_kmc_rs_run(occ.shape[0], float(eps), seed, t0, n_mcs, occ, ctypes.byref(mv)),
           "or_kmc_rs_run")
    return mv.value


def dt_run(occ: np.ndarray, eps: float, seed: int, block: int, t0: int, n_mcs: int,
           check: bool = False, counts: np.ndarray | None = None) -> int:
    """Doubly tiled dynamics in place; returns the accepted jumps.  ``counts``
    (int32, N entries, fcc order) accumulates attempts per site."""
    mv = ctypes.c_int64(0)
    ptr = None
    if counts is not None:
        assert counts.dtype == np.int32 and counts.flags.c_contiguous
        assert counts.size == occ.size // 2
        ptr = counts.ctypes.data
    _check(lib().or_kmc_dt_run(occ.shape[0], float(eps), seed, block, t0, n_mcs, occ,
                            ctypes.byref(mv), int(check), ptr), "or_kmc_dt_run")
    return mv.value


def attempt(occ: np.ndarray, eps: float, x: int, y: int, z: int, nb: int, u: int) -> int:
    rc = lib().or_kmc_attempt(occ.shape[0], float(eps), occ, x, y, z, nb, u)
    _check(min(rc, 0), "or_kmc_attempt")
    return rc


def counts(occ: np.ndarray):
    """(number of B, number of B-B nearest-neighbour bonds)."""
    nB, bonds = ctypes.c_int64(0), ctypes.c_int64(0)
    lib().or_kmc_counts(occ.shape[0], occ, ctypes.byref(nB), ctypes.byref(bonds))
    return nB.value, bonds.value


def order(seed: int, t: int) -> list:
    p = np.zeros(8, np.int32)
    lib().or_kmc_order(seed, t, p)
    return [int(v) for v in p]


def origin(seed: int, t: int, block: int) -> tuple:
    o = np.zeros(3, np.int32)
    lib().or_kmc_origin(seed, t, block, o)
    return tuple(int(v) for v in o)


def fcc_mask(L: int) -> np.ndarray:
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    return ((x ^ y ^ z) & 1) == 0


def to_fcc(occ: np.ndarray) -> np.ndarray:
    """Compact layout: one byte per fcc site, fcc order."""
    L = occ.shape[0]
    out = np.empty((L, L, L // 2), np.uint8)
    for z in range(L):
        for y in range(L):
            out[z, y] = occ[z, y, (y + z) & 1::2]
    return out.reshape(-1)


def from_fcc(comp: np.ndarray, L: int) -> np.ndarray:
    c = np.asarray(comp, np.uint8).reshape(L, L, L // 2)
    occ = np.zeros((L, L, L), np.uint8)
    for z in range(L):
        for y in range(L):
            occ[z, y, (y + z) & 1::2] = c[z, y]
    return occ
