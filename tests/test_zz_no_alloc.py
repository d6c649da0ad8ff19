"""kpz_roughness_noalloc (the entry point for callers that cannot allocate):
through the C ABI, its moments equal kpz_roughness's for the same lattice,
on two calls in a row, the second with a smaller lattice (the row-sum pass
plus finalize, then the single-work-group pass); sizes beyond the scratch
maximum are refused before any device work."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1204_5072_amd as kpz
    kpz.lib()
    return kpz


def _noalloc(kpz, words, L, net, stream):
    S1, S2, W2 = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
    st = kpz.lib().kpz_roughness_noalloc(ctypes.c_void_p(words.data_ptr()), L, net,
                                          ctypes.byref(S1), ctypes.byref(S2), ctypes.byref(W2),
                                          ctypes.c_void_p(stream.cuda_stream))
    return st, (S1.value, S2.value, W2.value)


@pytest.mark.parametrize("cases", [[(2048, (256, 128), 1.0, 0.25, 3, 4), (256, (64, 64), 1.0, 0.0, 4, 6)],
                                   [(1024, (512, 64), 0.7, 0.3, 5, 3), (64, (64, 64), 1.0, 0.0, 6, 9)]])
def test_noalloc_equals_roughness(gpu, cases):
    for L, block, p, q, seed, n in cases:
        print(f"noalloc L={L} block={block} p={p} q={q} seed={seed} n={n}", flush=True)
        sim = gpu.Sim(L, p, q, seed, block)
        sim.sweep(n)
        ref = sim.roughness()
        sim.sync_words()
        t, net = sim.state()
        st, got = _noalloc(gpu, sim.words, L, net, sim.stream)
        assert st == gpu.KPZ_OK, gpu.status_str(st)
        assert got == (ref.S1, ref.S2, ref.W2), (got, ref)
        sim.close()


def test_noalloc_refuses_oversize_and_bad_args(gpu):
    import torch
    w = torch.zeros(16, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()
    assert _noalloc(gpu, w, 131072, 0, s)[0] == gpu.KPZ_ESIZE
    assert _noalloc(gpu, w, 24, 0, s)[0] == gpu.KPZ_EINVAL
    st = gpu.lib().kpz_roughness_noalloc(None, 64, 0, None, None, None, None)
    assert st == gpu.KPZ_EINVAL


def test_noalloc_flat_start(gpu):
    """The flat start: S1 = S2 = N/2 and W^2 = 1/4 with net = 0; a wrong flip
    count is reported as an inconsistent state."""
    sim = gpu.Sim(128, 1.0, 0.0, 1, (64, 64))
    st, got = _noalloc(gpu, sim.words, 128, 0, sim.stream)
    assert st == gpu.KPZ_OK and got == (128 * 128 // 2, 128 * 128 // 2, 0.25)
    st, _ = _noalloc(gpu, sim.words, 128, 1, sim.stream)
    assert st == gpu.KPZ_ESTATE
