"""Host-only checks of the C ABI: the library loads, exports every function
include/kpz.h and include/kmc.h declare, and validates its arguments before
touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def kpz():
    import paper_1204_5072_amd as k
    if not os.path.exists(k.LIB_PATH):
        from paper_1204_5072_amd import build
        build.build()
    k.lib()
    return k


def header_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for h in sorted(os.listdir(inc)):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(inc, h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b((?:kpz|kmc)_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_exports_every_declared_function(kpz):
    names = header_functions()
    assert set(names) == set(kpz.EXPORTED)
    for n in names:
        assert hasattr(kpz.lib(), n), n


def test_status_strings(kpz):
    assert kpz.status_str(0) == "ok"
    for s in (-1, -2, -3, -4, -5):
        assert kpz.status_str(s) and kpz.status_str(s) != "unknown status"
    assert kpz.status_str(-99) == "unknown status"


@pytest.mark.parametrize("L,block", [(16, None), (64, None), (4096, None), (65536, None),
                                     (4096, (256, 64)), (48, (16, 16)), (768, (256, 128)),
                                     (65536, (512, 64)), (65536, (128, 256)), (64, (64, 4)),
                                     (65536, (1024, 32)), (4096, (1024, 16)),
                                     (320, (80, 160)), (192, (96, 192)), (384, (384, 16)),
                                     (960, (96, 240)), (48, (48, 48)), (96, (16, 12))])
def test_workspace_bytes_valid(kpz, L, block):
    n = kpz.workspace_bytes(kpz.make_params(L, 1.0, 0.0, 1, block))
    assert n >= 256 + 8 * 1024 + 16 * L


@pytest.mark.parametrize("L,shape", [
    (64, (64, 64)), (4096, (256, 128)), (65536, (256, 128)), (2048, (256, 128)),
    (128, (128, 128)), (1024 + 512, (256, 128)),
    # not multiples of 128: the valid shape dividing L with the most sites, then the widest
    (320, (80, 160)), (192, (96, 192)), (448, (112, 224)), (960, (96, 240)), (48, (48, 48)),
    (576, (96, 192)), (16, (16, 16))])
def test_default_block_shape(kpz, L, shape):
    assert kpz.block_shape(kpz.make_params(L, 1.0, 0.0, 1)) == shape



@pytest.mark.parametrize("kw", [
    dict(L=8), dict(L=24), dict(L=0), dict(L=64, p=1.5), dict(L=64, q=-0.1),
    dict(L=64, block=(48, 16)), dict(L=64, block=(8, 16)), dict(L=64, block=(128, 64)),
    dict(L=2048, block=(2048, 16)), dict(L=1024, block=(512, 256)),
    dict(L=1024, block=(256, 256)), dict(L=4096, block=(2048, 8)), dict(L=64, block=(16, 2)),
    dict(L=4096, block=(1024, 128)),
    dict(L=64, tile=(8, 8)), dict(L=96, block=(64, 32)),
    dict(L=320, block=(160, 64)), dict(L=96, block=(24, 48)), dict(L=64, block=(16, 6)),
    dict(L=1280, block=(1280, 16)), dict(L=384, block=(96, 264)),
    dict(L=64, moves=3), dict(L=64, moves=32), dict(L=64, moves=-1),
])
def test_invalid_params_rejected(kpz, kw):
    p = kpz.make_params(**kw)
    with pytest.raises(kpz.KPZError) as e:
        kpz.workspace_bytes(p)
    assert e.value.status == kpz.KPZ_EINVAL


def test_init_validates_before_device_work(kpz):
    L = kpz.lib()
    h = ctypes.c_void_p(1)
    bad = kpz.make_params(24)
    assert L.kpz_init(ctypes.byref(h), ctypes.byref(bad), ctypes.c_void_p(8), 1 << 20,
                      ctypes.c_void_p(8), 1 << 20, None) == kpz.KPZ_EINVAL
    assert h.value is None
    good = kpz.make_params(64)
    # null device pointers and short buffers are refused
    assert L.kpz_init(ctypes.byref(h), ctypes.byref(good), None, 1 << 20, ctypes.c_void_p(8),
                      1 << 20, None) == kpz.KPZ_EINVAL
    assert L.kpz_init(ctypes.byref(h), ctypes.byref(good), ctypes.c_void_p(8), 64 * 64 // 4 - 4,
                      ctypes.c_void_p(8), 1 << 20, None) == kpz.KPZ_ESIZE
    assert L.kpz_init(ctypes.byref(h), ctypes.byref(good), ctypes.c_void_p(8), 64 * 64 // 4,
                      ctypes.c_void_p(8), 100, None) == kpz.KPZ_ESIZE
    assert L.kpz_init(None, ctypes.byref(good), ctypes.c_void_p(8), 1 << 20, ctypes.c_void_p(8),
                      1 << 20, None) == kpz.KPZ_EINVAL
    assert L.kpz_sweep(None, 1) == kpz.KPZ_EINVAL
    assert L.kpz_roughness(None, None, None, None) == kpz.KPZ_EINVAL
    assert L.kpz_check_invariants(None, None) == kpz.KPZ_EINVAL
    L.kpz_destroy(None)


@pytest.mark.parametrize("moves", [0, 1, 2, 4, 8, 16])
def test_origin_moves_accepted(kpz, moves):
    assert kpz.workspace_bytes(kpz.make_params(256, 1.0, 0.0, 1, (64, 64), moves=moves)) > 0


def test_batch_members_must_share_moves(kpz):
    ms = [kpz.make_params(256, 1.0, 0.0, 1, (64, 64), moves=1),
          kpz.make_params(256, 1.0, 0.0, 2, (64, 64), moves=2)]
    with pytest.raises(kpz.KPZError):
        kpz.batch_sizes(ms)


def test_library_shares_torch_hip_runtime(kpz):
    """libkpz.so binds to the HIP runtime torch loaded: one libamdhip64 in
    the process (a second runtime would see no device)."""
    import os
    kpz.lib()
    maps = open(f"/proc/{os.getpid()}/maps").read()
    hip = {line.split()[-1] for line in maps.splitlines() if "libamdhip64" in line}
    assert len(hip) == 1, hip


@pytest.mark.parametrize("L,block,ok", [(128, 0, True), (6144, 0, True), (1 << 20, 0, True),
                                        (1 << 20, 1024, True), (1 << 32, 512, True),
                                        (1000, 0, False), (2048, 4096, False), (8192, 64, False),
                                        (384, 256, False), ((1 << 32) + 128, 0, False),
                                        (2048, 2048, False)])
def test_ring_params_validation(kpz, L, block, ok):
    p = kpz.kpz_ring_params(L, 1.0, 0.0, 1, block, 0)
    n = ctypes.c_size_t()
    st = kpz.lib().kpz_ring_workspace_bytes(ctypes.byref(p), ctypes.byref(n))
    assert (st == kpz.KPZ_OK) == ok, st
    if ok:
        assert n.value >= 256 + 8 * 1024 + 24 * (L // 8192) + 8 * (L // (64 * (block or 128)))


@pytest.mark.parametrize("L,block,ok", [(64, (16, 16), True), (256, (128, 128), True),
                                        (512, (128, 128), True), (65536, (512, 64), True),
                                        (512, (256, 256), False),
                                        (48, (16, 16), False), (64, (64, 16), False),
                                        (1024, (1024, 64), False)])
def test_device_dt_params(kpz, L, block, ok):
    p = kpz.make_params(L, 1.0, 0.0, 1, block, device_dt=True)
    if ok:
        assert kpz.workspace_bytes(p) > 0
    else:
        with pytest.raises(kpz.KPZError):
            kpz.workspace_bytes(p)


def test_device_dt_not_for_batches(kpz):
    with pytest.raises(kpz.KPZError):
        kpz.batch_sizes([kpz.make_params(64, 1.0, 0.0, 1, (16, 16), device_dt=True)])


@pytest.mark.parametrize("L,block,ok", [(16, 0, True), (16, 8, True), (32, 16, True),
                                        (512, 32, True), (2048, 0, True), (16, 16, False),
                                        (24, 8, False), (512, 64, False), (512, 4, False),
                                        (4096, 32, False), (8, 0, False)])
def test_kmc_params_validation(kpz, L, block, ok):
    p = kpz.kmc_params(L, 0.325, 1.5, 1, block, 0)
    n = ctypes.c_size_t()
    st = kpz.lib().kmc_workspace_bytes(ctypes.byref(p), ctypes.byref(n))
    assert (st == kpz.KPZ_OK) == ok, st
    if ok:
        assert n.value >= 24


@pytest.mark.parametrize("c,eps,flags", [(-0.1, 1.0, 0), (1.5, 1.0, 0), (0.3, -1.0, 0),
                                         (0.3, float("inf"), 0), (0.3, float("nan"), 0),
                                         (0.3, 1.0, 1)])
def test_kmc_bad_physics_rejected(kpz, c, eps, flags):
    p = kpz.kmc_params(64, c, eps, 1, 0, flags)
    n = ctypes.c_size_t()
    assert kpz.lib().kmc_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == kpz.KPZ_EINVAL


def test_kmc_init_checks_buffers_first(kpz):
    p = kpz.kmc_params(64, 0.3, 1.0, 1, 0, 0)
    h = ctypes.c_void_p()
    lib = kpz.lib()
    assert lib.kmc_init(ctypes.byref(h), ctypes.byref(p), None, 0, None, 0, None) == kpz.KPZ_EINVAL
    buf = ctypes.create_string_buffer(64)
    # too small: rejected before any device work
    assert lib.kmc_init(ctypes.byref(h), ctypes.byref(p), ctypes.cast(buf, ctypes.c_void_p),
                        64, ctypes.cast(buf, ctypes.c_void_p), 64, None) == kpz.KPZ_ESIZE
    assert not h.value
    assert lib.kmc_sweep(None, 1) == kpz.KPZ_EINVAL
    assert lib.kmc_counts(None, None, None) == kpz.KPZ_EINVAL


def test_dt_order_matches_oracle(oracle_lib):
    """The library's host-side order of the four block sets (it decides which
    launches take a set together with its diagonal partner) equals the
    oracle's draw for every MCS tried."""
    import paper_1204_5072_amd as kpz
    for seed in (1, 11, 2 ** 40 + 3):
        for t in range(300):
            assert kpz.dt_order(seed, t) == oracle_lib.dt_perm(seed, t)
