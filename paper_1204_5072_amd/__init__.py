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

EXPORTED = ("kpz_workspace_bytes", "kpz_init", "kpz_sweep", "kpz_roughness", "kpz_get_state",
            "kpz_set_state", "kpz_destroy", "kpz_status_str", "kpz_last_error")


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
                ("tile_y", ctypes.c_int32), ("flags", ctypes.c_uint32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Loads libkpz.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, c = ctypes.c_void_p, ctypes
        L.kpz_workspace_bytes.argtypes = [c.POINTER(kpz_params), c.POINTER(c.c_size_t)]
        L.kpz_init.argtypes = [c.POINTER(vp), c.POINTER(kpz_params), vp, c.c_size_t, vp,
                               c.c_size_t, vp]
        L.kpz_sweep.argtypes = [vp, c.c_int32]
        L.kpz_roughness.argtypes = [vp, c.POINTER(c.c_int64), c.POINTER(c.c_int64),
                                    c.POINTER(c.c_double)]
        L.kpz_get_state.argtypes = [vp, c.POINTER(c.c_int64), c.POINTER(c.c_int64)]
        L.kpz_set_state.argtypes = [vp, c.c_int64, c.c_int64]
        L.kpz_destroy.argtypes = [vp]
        L.kpz_destroy.restype = None
        L.kpz_status_str.argtypes = [c.c_int]
        L.kpz_status_str.restype = c.c_char_p
        L.kpz_last_error.argtypes = [vp]
        L.kpz_last_error.restype = c.c_char_p
        for f in ("kpz_workspace_bytes", "kpz_init", "kpz_sweep", "kpz_roughness",
                  "kpz_get_state", "kpz_set_state"):
            getattr(L, f).restype = c.c_int
        _lib = L
    return _lib


def status_str(status: int) -> str:
    return lib().kpz_status_str(status).decode()


def make_params(L: int, p: float = 1.0, q: float = 0.0, seed: int = 1,
                block: Optional[Tuple[int, int]] = None, tile: Tuple[int, int] = (4, 4)) -> kpz_params:
    bx, by = block if block else (0, 0)
    return kpz_params(L, float(p), float(q), int(seed), int(bx), int(by), int(tile[0]),
                      int(tile[1]), 0)


def workspace_bytes(params: kpz_params) -> int:
    n = ctypes.c_size_t()
    st = lib().kpz_workspace_bytes(ctypes.byref(params), ctypes.byref(n))
    if st != KPZ_OK:
        raise KPZError(st, "kpz_workspace_bytes")
    return n.value


@dataclass
class Moments:
    S1: int
    S2: int
    W2: float


class Sim:
    """One lattice on one GPU.  ``words`` is a torch int32 tensor of
    L*L/16 packed slope words (bit layout in include/kpz.h)."""

    def __init__(self, L: int, p: float = 1.0, q: float = 0.0, seed: int = 1,
                 block: Optional[Tuple[int, int]] = None, device="cuda", stream=None):
        import torch
        self.params = make_params(L, p, q, seed, block)
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
            raise KPZError(st, "kpz_init")

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

    def state(self) -> Tuple[int, int]:
        t, net = ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().kpz_get_state(self._h, ctypes.byref(t), ctypes.byref(net)),
                    "kpz_get_state")
        return t.value, net.value

    def set_state(self, t: int, net: int) -> None:
        self._check(lib().kpz_set_state(self._h, int(t), int(net)), "kpz_set_state")

    def words_host(self):
        """Copy of the packed words as a numpy uint32 array of shape (L, L/16)."""
        self.stream.synchronize()
        return self.words.cpu().numpy().view("uint32").reshape(self.L, self.L // 16)

    def load_words(self, words) -> None:
        """Overwrite the lattice with host words (uint32, L*L/16)."""
        import numpy as np
        import torch
        arr = np.ascontiguousarray(np.asarray(words, dtype=np.uint32).reshape(-1)).view(np.int32)
        with torch.cuda.stream(self.stream):
            self.words.copy_(torch.from_numpy(arr))

    def close(self) -> None:
        if self._h:
            lib().kpz_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
