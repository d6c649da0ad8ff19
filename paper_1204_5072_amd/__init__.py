"""MI355X-native Monte Carlo sweep of the 2+1-d KPZ octahedron model.

Thin binding over ``libkpz.so`` (the C ABI in ``include/kpz.h``): argument
marshalling only, every step of the sweep runs in the library's HIP kernels.
PyTorch provides the device memory (the packed slope words and the
workspace) and the HIP stream.

The library must have been built (``__graft_entry__.build()`` or
``python paper_1204_5072_amd/build.py``); importing the binding without it
raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Tuple

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libkpz.so")

KPZ_OK, KPZ_EINVAL, KPZ_ESIZE, KPZ_EHIP, KPZ_ESTATE, KPZ_ERANGE = 0, -1, -2, -3, -4, -5

EXPORTED = ("kpz_workspace_bytes", "kpz_block_shape", "kpz_init", "kpz_sweep", "kpz_roughness", "kpz_height_moments",
            "kpz_get_state", "kpz_set_state", "kpz_sync_words", "kpz_check_invariants", "kpz_destroy", "kpz_status_str",
            "kpz_last_error", "kpz_valu_probe", "kpz_roughness_noalloc", "kpz_dt_order",
            "kpz_batch_sizes", "kpz_batch_init", "kpz_batch_word_offset", "kpz_batch_sweep",
            "kpz_batch_roughness", "kpz_batch_run", "kpz_batch_get_t", "kpz_batch_destroy",
            "kpz_batch_last_error", "kpz_batch_sync_words",
            "kpz_pool_job_bytes", "kpz_pool_control_bytes", "kpz_pool_init", "kpz_pool_submit",
            "kpz_pool_step", "kpz_pool_poll", "kpz_pool_stats", "kpz_pool_destroy",
            "kpz_pool_last_error",
            "kpz_ring_workspace_bytes", "kpz_ring_init", "kpz_ring_sweep", "kpz_ring_roughness",
            "kpz_ring_get_state", "kpz_ring_destroy", "kpz_ring_last_error",
            "kmc_workspace_bytes", "kmc_init", "kmc_sweep", "kmc_counts", "kmc_get_state",
            "kmc_set_state", "kmc_destroy", "kmc_last_error")
BATCH_MAX_SAMPLES = 1024


class KPZError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str = ""):
        self.status = status
        msg = f"{what}: {status_str(status)} ({status})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


class kpz_params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("p", ctypes.c_double), ("q", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("block_x", ctypes.c_int32),
                ("block_y", ctypes.c_int32), ("tile_x", ctypes.c_int32),
                ("tile_y", ctypes.c_int32), ("moves", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class kpz_ring_params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int64), ("p", ctypes.c_double), ("q", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("block", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class kmc_params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int64), ("c", ctypes.c_double), ("eps", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("block", ctypes.c_int32), ("flags", ctypes.c_uint32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Loads libkpz.so; raises if it has not been built.

    torch is imported first: it loads its own HIP runtime, and libkpz.so
    then binds to that same runtime (same soname) instead of loading a
    second one from the system ROCm.  Two HIP runtimes in one process do
    not share devices, streams or allocations (the second one finds no
    device), and the device buffers and streams passed to the library come
    from torch."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        import torch  # noqa: F401  (binds the process to torch's HIP runtime)
        L = ctypes.CDLL(LIB_PATH)
        vp, c = ctypes.c_void_p, ctypes
        L.kpz_workspace_bytes.argtypes = [c.POINTER(kpz_params), c.POINTER(c.c_size_t)]
        L.kpz_block_shape.argtypes = [c.POINTER(kpz_params), c.POINTER(c.c_int32),
                                      c.POINTER(c.c_int32)]
        L.kpz_init.argtypes = [c.POINTER(vp), c.POINTER(kpz_params), vp, c.c_size_t, vp,
                               c.c_size_t, vp]
        L.kpz_sweep.argtypes = [vp, c.c_int32]
        L.kpz_valu_probe.argtypes = [vp, c.c_int32, c.c_int32, c.POINTER(c.c_int32), vp]
        L.kpz_roughness_noalloc.argtypes = [vp, c.c_int64, c.c_int64, c.POINTER(c.c_int64),
                                            c.POINTER(c.c_int64), c.POINTER(c.c_double), vp]
        L.kpz_roughness.argtypes = [vp, c.POINTER(c.c_int64), c.POINTER(c.c_int64),
                                    c.POINTER(c.c_double)]
        L.kpz_height_moments.argtypes = [vp, c.POINTER(c.c_int64), c.POINTER(c.c_double),
                                         c.POINTER(c.c_double), c.POINTER(c.c_double)]
        L.kpz_height_moments.restype = c.c_int
        L.kpz_get_state.argtypes = [vp, c.POINTER(c.c_int64), c.POINTER(c.c_int64)]
        L.kpz_dt_order.argtypes = [c.c_uint64, c.c_uint32, c.POINTER(c.c_int32 * 4)]
        L.kpz_set_state.argtypes = [vp, c.c_int64, c.c_int64]
        L.kpz_sync_words.argtypes = [vp]
        L.kpz_check_invariants.argtypes = [vp, c.POINTER(c.c_int64)]
        L.kpz_destroy.argtypes = [vp]
        L.kpz_destroy.restype = None
        L.kpz_status_str.argtypes = [c.c_int]
        L.kpz_status_str.restype = c.c_char_p
        L.kpz_last_error.argtypes = [vp]
        L.kpz_last_error.restype = c.c_char_p
        P, i64p, f64p = c.POINTER(kpz_params), c.POINTER(c.c_int64), c.POINTER(c.c_double)
        L.kpz_batch_sizes.argtypes = [P, c.c_int32, c.POINTER(c.c_size_t), c.POINTER(c.c_size_t)]
        L.kpz_batch_init.argtypes = [c.POINTER(vp), P, c.c_int32, vp, c.c_size_t, vp, c.c_size_t, vp]
        L.kpz_batch_word_offset.argtypes = [vp, c.c_int32, c.POINTER(c.c_size_t)]
        L.kpz_batch_sweep.argtypes = [vp, c.c_int32]
        L.kpz_batch_roughness.argtypes = [vp, i64p, i64p, f64p]
        L.kpz_batch_run.argtypes = [vp, c.POINTER(c.c_int32), c.c_int32, i64p, i64p, f64p]
        L.kpz_batch_get_t.argtypes = [vp, i64p]
        L.kpz_batch_sync_words.argtypes = [vp]
        L.kpz_batch_destroy.argtypes = [vp]
        L.kpz_batch_destroy.restype = None
        L.kpz_batch_last_error.argtypes = [vp]
        L.kpz_batch_last_error.restype = c.c_char_p
        szp, i32p = c.POINTER(c.c_size_t), c.POINTER(c.c_int32)
        L.kpz_pool_job_bytes.argtypes = [P, c.c_int32, c.c_int32, szp]
        L.kpz_pool_control_bytes.argtypes = [c.c_int32, szp]
        L.kpz_pool_init.argtypes = [c.POINTER(vp), vp, c.c_size_t, c.c_int32, c.c_int32, c.c_int32,
                                    c.c_int32, vp]
        L.kpz_pool_submit.argtypes = [vp, P, c.c_int64, i64p]
        L.kpz_pool_step.argtypes = [vp, c.c_int32, i32p]
        L.kpz_pool_poll.argtypes = [vp, c.c_int32, i64p, i64p, i64p, f64p, i32p, i32p]
        L.kpz_pool_stats.argtypes = [vp, i32p, szp]
        L.kpz_pool_destroy.argtypes = [vp]
        L.kpz_pool_destroy.restype = None
        L.kpz_pool_last_error.argtypes = [vp]
        L.kpz_pool_last_error.restype = c.c_char_p
        RP = c.POINTER(kpz_ring_params)
        L.kpz_ring_workspace_bytes.argtypes = [RP, szp]
        L.kpz_ring_init.argtypes = [c.POINTER(vp), RP, vp, c.c_size_t, vp, c.c_size_t, vp]
        L.kpz_ring_sweep.argtypes = [vp, c.c_int32]
        L.kpz_ring_roughness.argtypes = [vp, i64p, i64p, f64p]
        L.kpz_ring_get_state.argtypes = [vp, i64p, i64p]
        L.kpz_ring_destroy.argtypes = [vp]
        L.kpz_ring_destroy.restype = None
        L.kpz_ring_last_error.argtypes = [vp]
        L.kpz_ring_last_error.restype = c.c_char_p
        KP = c.POINTER(kmc_params)
        L.kmc_workspace_bytes.argtypes = [KP, szp]
        L.kmc_init.argtypes = [c.POINTER(vp), KP, vp, c.c_size_t, vp, c.c_size_t, vp]
        L.kmc_sweep.argtypes = [vp, c.c_int32]
        L.kmc_counts.argtypes = [vp, i64p, i64p]
        L.kmc_get_state.argtypes = [vp, i64p, i64p]
        L.kmc_set_state.argtypes = [vp, c.c_int64, c.c_int64]
        L.kmc_destroy.argtypes = [vp]
        L.kmc_destroy.restype = None
        L.kmc_last_error.argtypes = [vp]
        L.kmc_last_error.restype = c.c_char_p
        for f in ("kpz_workspace_bytes", "kpz_init", "kpz_sweep", "kpz_roughness",
                  "kpz_get_state", "kpz_set_state", "kpz_sync_words", "kpz_check_invariants",
                  "kpz_dt_order",
                  "kpz_batch_sizes",
                  "kpz_batch_init",
                  "kpz_batch_word_offset", "kpz_batch_sweep", "kpz_batch_roughness",
                  "kpz_batch_run", "kpz_batch_get_t", "kpz_batch_sync_words", "kpz_pool_job_bytes",
                  "kpz_pool_control_bytes", "kpz_pool_init", "kpz_pool_submit", "kpz_pool_step",
                  "kpz_pool_poll", "kpz_pool_stats", "kpz_ring_workspace_bytes", "kpz_ring_init",
                  "kpz_ring_sweep", "kpz_ring_roughness", "kpz_ring_get_state",
                  "kmc_workspace_bytes", "kmc_init", "kmc_sweep", "kmc_counts", "kmc_get_state",
                  "kmc_set_state"):
            getattr(L, f).restype = c.c_int
        _lib = L
    return _lib


def status_str(status: int) -> str:
    return lib().kpz_status_str(status).decode()


KPZ_FLAG_IN_PLACE = 1
KPZ_FLAG_DEVICE_DT = 2
KPZ_FLAG_DT_AHEAD = 4


def make_params(L: int, p: float = 1.0, q: float = 0.0, seed: int = 1,
                block: Optional[Tuple[int, int]] = None, tile: Tuple[int, int] = (4, 4),
                moves: int = 1, in_place: bool = False, device_dt: bool = False,
                dt_ahead: bool = False) -> kpz_params:
    """Parameters of one lattice; ``moves`` = dead-border origin moves per
    MCS (block residency 1/moves MCS); ``in_place`` = update the lattice in
    place (no second lattice buffer in the workspace); ``device_dt`` =
    double tiling instead of dead borders at the device layer;
    ``dt_ahead`` = with it, a set and its diagonal partner share a launch
    when they follow each other in the MCS's order."""
    bx, by = block if block else (0, 0)
    flags = ((KPZ_FLAG_IN_PLACE if in_place else 0) | (KPZ_FLAG_DEVICE_DT if device_dt else 0)
             | (KPZ_FLAG_DT_AHEAD if dt_ahead else 0))
    return kpz_params(L, float(p), float(q), int(seed), int(bx), int(by), int(tile[0]),
                      int(tile[1]), int(moves), flags)


def dt_order(seed: int, t: int):
    """Order of the four block sets in MCS t under device-layer double
    tiling (the library's host-side draw)."""
    arr = (ctypes.c_int32 * 4)()
    st = lib().kpz_dt_order(int(seed), int(t), ctypes.byref(arr))
    if st != KPZ_OK:
        raise KPZError(st, "kpz_dt_order", "")
    return list(arr)


def workspace_bytes(params: kpz_params) -> int:
    n = ctypes.c_size_t()
    st = lib().kpz_workspace_bytes(ctypes.byref(params), ctypes.byref(n))
    if st != KPZ_OK:
        raise KPZError(st, "kpz_workspace_bytes")
    return n.value


def block_shape(params: kpz_params) -> Tuple[int, int]:
    """The block shape (sites) these parameters run with, defaults resolved."""
    bx, by = ctypes.c_int32(), ctypes.c_int32()
    st = lib().kpz_block_shape(ctypes.byref(params), ctypes.byref(bx), ctypes.byref(by))
    if st != KPZ_OK:
        raise KPZError(st, "kpz_block_shape")
    return bx.value, by.value


@dataclass
class Moments:
    S1: int
    S2: int
    W2: float


class Sim:
    """One lattice on one GPU.  ``words`` is a torch int32 tensor of
    L*L/16 packed slope words (bit layout in include/kpz.h)."""

    def __init__(self, L: int, p: float = 1.0, q: float = 0.0, seed: int = 1,
                 block: Optional[Tuple[int, int]] = None, device="cuda", stream=None,
                 moves: int = 1, in_place: bool = False, device_dt: bool = False,
                 dt_ahead: bool = False):
        import torch
        self.params = make_params(L, p, q, seed, block, moves=moves, in_place=in_place,
                                  device_dt=device_dt, dt_ahead=dt_ahead)
        self.L = L
        ws = workspace_bytes(self.params)
        self.device = torch.device(device)
        self.words = torch.empty(L * L // 16, dtype=torch.int32, device=self.device)
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._h = ctypes.c_void_p()
        st = lib().kpz_init(ctypes.byref(self._h), ctypes.byref(self.params),
                            ctypes.c_void_p(self.words.data_ptr()), self.words.numel() * 4,
                            ctypes.c_void_p(self.workspace.data_ptr()), ws,
                            ctypes.c_void_p(self.stream.cuda_stream))
        if st != KPZ_OK:
            raise KPZError(st, "kpz_init", lib().kpz_last_error(None).decode())

    def _check(self, st: int, what: str) -> None:
        if st != KPZ_OK:
            raise KPZError(st, what, lib().kpz_last_error(self._h).decode())

    def sweep(self, n_mcs: int = 1) -> "Sim":
        self._check(lib().kpz_sweep(self._h, int(n_mcs)), "kpz_sweep")
        return self

    def roughness(self) -> Moments:
        S1, S2, W2 = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        self._check(lib().kpz_roughness(self._h, ctypes.byref(S1), ctypes.byref(S2),
                                        ctypes.byref(W2)), "kpz_roughness")
        return Moments(S1.value, S2.value, W2.value)

    def height_moments(self):
        """Exact sums M_k = sum (h - h(0,0))^k, k = 1..4 (Python ints), and
        (W2, skewness, excess kurtosis) of the height distribution."""
        sums = (ctypes.c_int64 * 8)()
        w2, sk, ku = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(lib().kpz_height_moments(self._h, sums, ctypes.byref(w2), ctypes.byref(sk),
                                             ctypes.byref(ku)), "kpz_height_moments")
        M = [(sums[2 * k + 1] << 64) + (sums[2 * k] & ((1 << 64) - 1)) for k in range(4)]
        return M, (w2.value, sk.value, ku.value)

    def check_invariants(self) -> Tuple[int, int, int]:
        """(open plaquettes, row-0 slope sum, column-0 slope sum) of the
        stored surface (kpz_check_invariants); all zero for a valid one.
        Returns the counts whatever they are; raises only on other errors."""
        counts = (ctypes.c_int64 * 3)()
        st = lib().kpz_check_invariants(self._h, counts)
        if st not in (KPZ_OK, KPZ_ESTATE):
            self._check(st, "kpz_check_invariants")
        return counts[0], counts[1], counts[2]

    def state(self) -> Tuple[int, int]:
        t, net = ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().kpz_get_state(self._h, ctypes.byref(t), ctypes.byref(net)),
                    "kpz_get_state")
        return t.value, net.value

    def set_state(self, t: int, net: int) -> None:
        self._check(lib().kpz_set_state(self._h, int(t), int(net)), "kpz_set_state")

    def sync_words(self) -> "Sim":
        """Make ``words`` hold the current state (kpz_sync_words)."""
        self._check(lib().kpz_sync_words(self._h), "kpz_sync_words")
        return self

    def words_host(self):
        """Copy of the packed words as a numpy uint32 array of shape (L, L/16)."""
        self.sync_words()
        self.stream.synchronize()
        return self.words.cpu().numpy().view("uint32").reshape(self.L, self.L // 16)

    def load_words(self, words) -> None:
        """Overwrite the lattice with host words (uint32, L*L/16)."""
        import numpy as np
        import torch
        arr = np.ascontiguousarray(np.asarray(words, dtype=np.uint32).reshape(-1)).view(np.int32)
        t, net = self.state()
        with torch.cuda.stream(self.stream):
            self.words.copy_(torch.from_numpy(arr))
        # `words` now holds the lattice (the counters are kept; set_state
        # replaces them for a checkpoint)
        self.set_state(t, net)

    def close(self) -> None:
        if self._h:
            lib().kpz_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_sizes(members) -> Tuple[int, int]:
    arr = (kpz_params * len(members))(*members)
    wb, sb = ctypes.c_size_t(), ctypes.c_size_t()
    st = lib().kpz_batch_sizes(arr, len(members), ctypes.byref(wb), ctypes.byref(sb))
    if st != KPZ_OK:
        raise KPZError(st, "kpz_batch_sizes")
    return wb.value, sb.value


class Ensemble:
    """n independent lattices on one GPU, advanced together: each MCS is one
    launch over the blocks of every member (plus the straddling-word merge).
    ``members`` is a list of kpz_params (see make_params); all must resolve
    to the same block shape."""

    def __init__(self, members, device="cuda", stream=None):
        import torch
        self.members = list(members)
        self.n = len(self.members)
        self._arr = (kpz_params * self.n)(*self.members)
        wb, sb = batch_sizes(self.members)
        self.device = torch.device(device)
        self.words = torch.empty(wb // 4, dtype=torch.int32, device=self.device)
        self.workspace = torch.empty(sb, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._h = ctypes.c_void_p()
        st = lib().kpz_batch_init(ctypes.byref(self._h), self._arr, self.n,
                                  ctypes.c_void_p(self.words.data_ptr()), wb,
                                  ctypes.c_void_p(self.workspace.data_ptr()), sb,
                                  ctypes.c_void_p(self.stream.cuda_stream))
        if st != KPZ_OK:
            raise KPZError(st, "kpz_batch_init", lib().kpz_batch_last_error(None).decode())

    def _check(self, st, what):
        if st != KPZ_OK:
            raise KPZError(st, what, lib().kpz_batch_last_error(self._h).decode())

    def sweep(self, n_mcs: int = 1) -> "Ensemble":
        self._check(lib().kpz_batch_sweep(self._h, int(n_mcs)), "kpz_batch_sweep")
        return self

    def roughness(self):
        import numpy as np
        S1 = (ctypes.c_int64 * self.n)()
        S2 = (ctypes.c_int64 * self.n)()
        W2 = (ctypes.c_double * self.n)()
        self._check(lib().kpz_batch_roughness(self._h, S1, S2, W2), "kpz_batch_roughness")
        return np.array(S1[:], dtype=object), np.array(S2[:], dtype=object), np.array(W2[:])

    def run(self, times):
        """Sweep to each of the increasing MCS counts in ``times`` and sample
        the moments there, as one captured HIP graph; returns arrays of shape
        (len(times), n)."""
        import numpy as np
        k = len(times)
        T = (ctypes.c_int32 * k)(*[int(t) for t in times])
        S1 = (ctypes.c_int64 * (k * self.n))()
        S2 = (ctypes.c_int64 * (k * self.n))()
        W2 = (ctypes.c_double * (k * self.n))()
        self._check(lib().kpz_batch_run(self._h, T, k, S1, S2, W2), "kpz_batch_run")
        shape = (k, self.n)
        return (np.array(S1[:], dtype=np.int64).reshape(shape),
                np.array(S2[:], dtype=np.int64).reshape(shape),
                np.array(W2[:]).reshape(shape))

    @property
    def t(self) -> int:
        v = ctypes.c_int64()
        self._check(lib().kpz_batch_get_t(self._h, ctypes.byref(v)), "kpz_batch_get_t")
        return v.value

    def member_words(self, r: int):
        """Copy of member r's packed words, numpy uint32 of shape (L, L/16)."""
        off = ctypes.c_size_t()
        self._check(lib().kpz_batch_word_offset(self._h, int(r), ctypes.byref(off)),
                    "kpz_batch_word_offset")
        L = self.members[r].L
        self._check(lib().kpz_batch_sync_words(self._h), "kpz_batch_sync_words")
        self.stream.synchronize()
        w = self.words[off.value: off.value + L * L // 16]
        return w.cpu().numpy().view("uint32").reshape(L, L // 16)

    def close(self) -> None:
        if self._h:
            lib().kpz_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# The job pool's block shape: None gives every job the library's default
# shape for its own L (one full wave of 64 lanes per block from L = 256 up).
POOL_BLOCK: Optional[Tuple[int, int]] = None


class Pool:
    """Continuous-batching job pool over a device arena of ``hbm_bytes``
    (the HBM budget).  submit() returns a job id, or None when the job does
    not fit right now; step() advances every resident job; poll() returns
    finished jobs' exact moments.  With ``block`` set every job runs that
    block shape (L must be a multiple of both sides); with None each job runs
    the default shape for its L."""

    def __init__(self, hbm_bytes: int, max_jobs: int = 1024, max_quantum: int = 256,
                 block: Optional[Tuple[int, int]] = POOL_BLOCK, device="cuda", stream=None):
        import torch
        self.block = tuple(block) if block else (0, 0)
        self.max_quantum = max_quantum
        self.failures = []
        self.device = torch.device(device)
        self.arena = torch.empty(int(hbm_bytes), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._h = ctypes.c_void_p()
        st = lib().kpz_pool_init(ctypes.byref(self._h), ctypes.c_void_p(self.arena.data_ptr()),
                                 self.arena.numel(), max_jobs, max_quantum, self.block[0],
                                 self.block[1], ctypes.c_void_p(self.stream.cuda_stream))
        if st != KPZ_OK:
            raise KPZError(st, "kpz_pool_init")

    def _check(self, st, what):
        if st != KPZ_OK:
            raise KPZError(st, what, lib().kpz_pool_last_error(self._h).decode())

    @staticmethod
    def control_bytes(max_jobs: int) -> int:
        """Arena bytes of the control region for ``max_jobs`` resident jobs."""
        n = ctypes.c_size_t()
        st = lib().kpz_pool_control_bytes(int(max_jobs), ctypes.byref(n))
        if st != KPZ_OK:
            raise KPZError(st, "kpz_pool_control_bytes")
        return n.value

    def job_bytes(self, params: kpz_params) -> int:
        n = ctypes.c_size_t()
        self._check(lib().kpz_pool_job_bytes(ctypes.byref(params), self.block[0], self.block[1],
                                             ctypes.byref(n)), "kpz_pool_job_bytes")
        return n.value

    def submit(self, params: kpz_params, n_mcs: int):
        jid = ctypes.c_int64()
        st = lib().kpz_pool_submit(self._h, ctypes.byref(params), int(n_mcs), ctypes.byref(jid))
        if st == KPZ_ESIZE:
            return None
        self._check(st, "kpz_pool_submit")
        return jid.value

    def step(self, quantum: int) -> int:
        n = ctypes.c_int32()
        self._check(lib().kpz_pool_step(self._h, int(quantum), ctypes.byref(n)), "kpz_pool_step")
        return n.value

    def poll(self, max_results: int = 4096):
        """Finished jobs as [(job id, Moments)], FIFO.  A job whose own
        result failed (its kpz_status is not KPZ_OK) is not in the list: it
        is appended to ``self.failures`` as (job id, status), so one bad job
        never loses the others' results."""
        ids = (ctypes.c_int64 * max_results)()
        S1 = (ctypes.c_int64 * max_results)()
        S2 = (ctypes.c_int64 * max_results)()
        W2 = (ctypes.c_double * max_results)()
        status = (ctypes.c_int32 * max_results)()
        n = ctypes.c_int32()
        self._check(lib().kpz_pool_poll(self._h, max_results, ids, S1, S2, W2, status,
                                        ctypes.byref(n)), "kpz_pool_poll")
        out = []
        for i in range(n.value):
            if status[i] == KPZ_OK:
                out.append((ids[i], Moments(S1[i], S2[i], W2[i])))
            else:
                self.failures.append((ids[i], int(status[i])))
        return out

    def stats(self):
        n, free = ctypes.c_int32(), ctypes.c_size_t()
        self._check(lib().kpz_pool_stats(self._h, ctypes.byref(n), ctypes.byref(free)),
                    "kpz_pool_stats")
        return n.value, free.value

    def close(self) -> None:
        if self._h:
            lib().kpz_pool_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ring:
    """The 1+1-d rooftop ring of L sites on one GPU (the reduction of the
    model to one dimension).  ``words`` is a torch int32 tensor of L/32
    packed bond words (bit layout in include/kpz.h)."""

    def __init__(self, L: int, p: float = 1.0, q: float = 0.0, seed: int = 1, block: int = 0,
                 device="cuda", stream=None):
        import torch
        self.params = kpz_ring_params(int(L), float(p), float(q), int(seed), int(block), 0)
        self.L = int(L)
        n = ctypes.c_size_t()
        st = lib().kpz_ring_workspace_bytes(ctypes.byref(self.params), ctypes.byref(n))
        if st != KPZ_OK:
            raise KPZError(st, "kpz_ring_workspace_bytes")
        self.device = torch.device(device)
        self.words = torch.empty(self.L // 32, dtype=torch.int32, device=self.device)
        self.workspace = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._h = ctypes.c_void_p()
        st = lib().kpz_ring_init(ctypes.byref(self._h), ctypes.byref(self.params),
                                 ctypes.c_void_p(self.words.data_ptr()), self.words.numel() * 4,
                                 ctypes.c_void_p(self.workspace.data_ptr()), n.value,
                                 ctypes.c_void_p(self.stream.cuda_stream))
        if st != KPZ_OK:
            raise KPZError(st, "kpz_ring_init", lib().kpz_last_error(None).decode())

    def _check(self, st: int, what: str) -> None:
        if st != KPZ_OK:
            raise KPZError(st, what, lib().kpz_ring_last_error(self._h).decode())

    def sweep(self, n_mcs: int = 1) -> "Ring":
        self._check(lib().kpz_ring_sweep(self._h, int(n_mcs)), "kpz_ring_sweep")
        return self

    def roughness(self) -> Moments:
        S1, S2, W2 = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        self._check(lib().kpz_ring_roughness(self._h, ctypes.byref(S1), ctypes.byref(S2),
                                             ctypes.byref(W2)), "kpz_ring_roughness")
        return Moments(S1.value, S2.value, W2.value)

    def state(self) -> Tuple[int, int]:
        t, net = ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().kpz_ring_get_state(self._h, ctypes.byref(t), ctypes.byref(net)),
                    "kpz_ring_get_state")
        return t.value, net.value

    def words_host(self):
        """Copy of the packed bonds, numpy uint32 of shape (L/32,)."""
        self.stream.synchronize()
        return self.words.cpu().numpy().view("uint32")

    def close(self) -> None:
        if self._h:
            lib().kpz_ring_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Kmc:
    """The 3-d KMC binary alloy (fcc sub-lattice of an L^3 cubic grid) on one
    GPU.  ``occ`` is a torch uint8 tensor of L^3/2 bytes, one per fcc site
    (layout in include/kmc.h); ``eps`` is the coupling of the Metropolis
    rule and ``c`` the initial B concentration."""

    def __init__(self, L: int, c: float = 0.325, eps: float = 1.5, seed: int = 1, block: int = 0,
                 device="cuda", stream=None):
        import torch
        self.params = kmc_params(int(L), float(c), float(eps), int(seed), int(block), 0)
        self.L = int(L)
        n = ctypes.c_size_t()
        st = lib().kmc_workspace_bytes(ctypes.byref(self.params), ctypes.byref(n))
        if st != KPZ_OK:
            raise KPZError(st, "kmc_workspace_bytes")
        self.device = torch.device(device)
        self.occ = torch.empty(self.L ** 3 // 2, dtype=torch.uint8, device=self.device)
        self.workspace = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._h = ctypes.c_void_p()
        st = lib().kmc_init(ctypes.byref(self._h), ctypes.byref(self.params),
                            ctypes.c_void_p(self.occ.data_ptr()), self.occ.numel(),
                            ctypes.c_void_p(self.workspace.data_ptr()), n.value,
                            ctypes.c_void_p(self.stream.cuda_stream))
        if st != KPZ_OK:
            raise KPZError(st, "kmc_init")

    def _check(self, st: int, what: str) -> None:
        if st != KPZ_OK:
            raise KPZError(st, what, lib().kmc_last_error(self._h).decode())

    def sweep(self, n_mcs: int = 1) -> "Kmc":
        self._check(lib().kmc_sweep(self._h, int(n_mcs)), "kmc_sweep")
        return self

    def counts(self) -> Tuple[int, int]:
        """(number of B, number of B-B bonds)."""
        nb, bonds = ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().kmc_counts(self._h, ctypes.byref(nb), ctypes.byref(bonds)),
                    "kmc_counts")
        return nb.value, bonds.value

    def state(self) -> Tuple[int, int]:
        """(MCS counter, accepted jumps)."""
        t, m = ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().kmc_get_state(self._h, ctypes.byref(t), ctypes.byref(m)),
                    "kmc_get_state")
        return t.value, m.value

    def occ_host(self):
        """Copy of the sites, numpy uint8 of shape (L^3/2,) in fcc order."""
        self.stream.synchronize()
        return self.occ.cpu().numpy()

    def load(self, occ_fcc, t: int = 0, moves: int = 0) -> "Kmc":
        """Replaces the state by ``occ_fcc`` (L^3/2 bytes, fcc order)."""
        import numpy as np
        import torch
        a = np.ascontiguousarray(occ_fcc, dtype=np.uint8).reshape(-1)
        if a.size != self.occ.numel():
            raise ValueError("occupation array has the wrong size")
        self.stream.synchronize()
        self.occ.copy_(torch.from_numpy(a).to(self.device))
        torch.cuda.synchronize(self.device)
        self._check(lib().kmc_set_state(self._h, int(t), int(moves)), "kmc_set_state")
        return self

    def close(self) -> None:
        if self._h:
            lib().kmc_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
