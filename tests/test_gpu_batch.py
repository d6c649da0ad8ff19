"""Ensemble (batched) path: every member of a multi-lattice launch
is bit-identical to the single-lattice run with the same parameters and
block shape (and so to the oracle), with uneven L, different p, q and each
member's own block shape."""
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


def _mix(kpz, Ls, qs, block, seed0=1000):
    return [kpz.make_params(L, 1.0, q, seed0 + r, block) for r, (L, q) in enumerate(zip(Ls, qs))]


@pytest.mark.parametrize("block", [(64, 64), (128, 256), (256, 128), (128, 64)])
def test_batch_members_equal_single_runs(gpu, oracle_lib, block):
    Ls = [256, 512, 256, 1024, 512, 256]
    qs = [0.0, 0.25, 0.5, 0.0, 0.5, 0.25]
    members = _mix(gpu, Ls, qs, block)
    ens = gpu.Ensemble(members)
    ens.sweep(3)
    S1, S2, W2 = ens.roughness()
    for r, m in enumerate(members):
        sim = gpu.Sim(m.L, m.p, m.q, m.seed, block)
        sim.sweep(3)
        assert np.array_equal(ens.member_words(r), sim.words_host()), r
        mr = sim.roughness()
        assert (int(S1[r]), int(S2[r]), float(W2[r])) == (mr.S1, mr.S2, mr.W2), r
    # one member against the oracle directly
    st = oracle_lib.SlopeState(256).run_dd(3, 1.0, 0.5, 1002, block=block, tile=(4, 4))
    assert np.array_equal(ens.member_words(2), oracle_lib.pack(st.sx, st.sy))


def test_batch_run_graph_equals_stepwise(gpu):
    """The captured sampling schedule gives the same moments as sweeping and
    sampling call by call."""
    Ls = [256, 512, 256, 512]
    qs = [0.0, 0.25, 0.5, 0.0]
    times = [1, 2, 3, 5, 8, 13]
    a = gpu.Ensemble(_mix(gpu, Ls, qs, (128, 256)))
    S1a, S2a, W2a = a.run(times)
    b = gpu.Ensemble(_mix(gpu, Ls, qs, (128, 256)))
    t = 0
    for k, T in enumerate(times):
        b.sweep(T - t)
        t = T
        S1, S2, W2 = b.roughness()
        assert list(S1a[k]) == [int(v) for v in S1], k
        assert list(S2a[k]) == [int(v) for v in S2], k
        assert list(W2a[k]) == list(W2), k
    assert a.t == b.t == times[-1]
    for r in range(len(Ls)):
        assert np.array_equal(a.member_words(r), b.member_words(r))


def test_batch_mixed_sizes_sweep_single_block_members(gpu):
    """Members with L equal to the block size are one periodic block."""
    members = _mix(gpu, [256, 2048, 256], [0.0, 0.0, 0.25], (256, 128))
    ens = gpu.Ensemble(members)
    ens.sweep(2)
    for r, m in enumerate(members):
        sim = gpu.Sim(m.L, m.p, m.q, m.seed, (256, 128))
        sim.sweep(2)
        assert np.array_equal(ens.member_words(r), sim.words_host()), r


def test_batch_run_every_mcs_long_schedule(gpu):
    """A one-member graph run with a sample after each of 300 MCS (more than
    one sample block) equals the single-lattice run sampled MCS by MCS, and
    a second run continues from where the first stopped."""
    p = gpu.make_params(64, 1.0, 0.25, 5, (64, 64))
    ens = gpu.Ensemble([p])
    S1a, S2a, W2a = ens.run(list(range(1, 301)))
    S1b, S2b, W2b = ens.run([305, 310])
    sim = gpu.Sim(64, 1.0, 0.25, 5, (64, 64))
    for k in range(300):
        sim.sweep(1)
        m = sim.roughness()
        assert (int(S1a[k, 0]), int(S2a[k, 0]), float(W2a[k, 0])) == (m.S1, m.S2, m.W2), k
    for k, T in enumerate([305, 310]):
        sim.sweep(T - sim.state()[0])
        m = sim.roughness()
        assert (int(S1b[k, 0]), int(S2b[k, 0]), float(W2b[k, 0])) == (m.S1, m.S2, m.W2), T
    assert np.array_equal(ens.member_words(0), sim.words_host())


def test_batch_members_with_origin_moves_equal_single_runs(gpu):
    """A batch whose members move the origin four times per MCS equals the
    single-lattice runs with the same setting."""
    members = [gpu.make_params(L, 1.0, q, 40 + r, (64, 64), moves=4)
               for r, (L, q) in enumerate([(128, 0.0), (256, 0.25), (64, 0.5)])]
    ens = gpu.Ensemble(members)
    ens.sweep(3)
    S1, S2, W2 = ens.roughness()
    for r, m in enumerate(members):
        sim = gpu.Sim(m.L, m.p, m.q, m.seed, (64, 64), moves=4)
        sim.sweep(3)
        assert np.array_equal(ens.member_words(r), sim.words_host()), r
        mm = sim.roughness()
        assert (int(S1[r]), int(S2[r]), float(W2[r])) == (mm.S1, mm.S2, mm.W2), r


def test_batch_in_place_equals_two_buffer(gpu):
    """A batch swept in place (one member flagged in place) and the same
    batch in two-buffer mode give identical lattices and moments."""
    Ls, qs = [256, 512, 256], [0.0, 0.25, 0.5]
    two = gpu.Ensemble(_mix(gpu, Ls, qs, (256, 64)))
    inp_members = _mix(gpu, Ls, qs, (256, 64))
    inp_members[1].flags = gpu.KPZ_FLAG_IN_PLACE
    inp = gpu.Ensemble(inp_members)
    for n in (1, 2, 3):
        two.sweep(n)
        inp.sweep(n)
        a, b = two.roughness(), inp.roughness()
        assert [list(x) for x in a] == [list(x) for x in b], n
    for r in range(len(Ls)):
        assert np.array_equal(two.member_words(r), inp.member_words(r)), r
    # syncing twice, and sweeping on after a sync, stay consistent
    two.sweep(1)
    inp.sweep(1)
    for r in range(len(Ls)):
        assert np.array_equal(two.member_words(r), inp.member_words(r)), r


def test_batch_members_with_own_block_shapes(gpu, oracle_lib):
    """Each member runs its own block shape (the default for its L when 0)
    in one launch; every member equals its single-lattice run, one equals
    the oracle directly."""
    shapes = [(128, 256), (512, 64), None, (64, 64), (256, 128), (32, 16), None, (48, 48)]
    Ls = [256, 1024, 512, 128, 256, 64, 320, 96]
    qs = [0.0, 0.25, 0.5, 0.0, 0.7, 0.25, 0.25, 0.0]
    members = [gpu.make_params(L, 1.0, q, 60 + r, shp)
               for r, (L, q, shp) in enumerate(zip(Ls, qs, shapes))]
    ens = gpu.Ensemble(members)
    ens.sweep(3)
    S1, S2, W2 = ens.roughness()
    for r, m in enumerate(members):
        sim = gpu.Sim(m.L, m.p, m.q, m.seed, shapes[r])
        sim.sweep(3)
        assert np.array_equal(ens.member_words(r), sim.words_host()), r
        mm = sim.roughness()
        assert (int(S1[r]), int(S2[r]), float(W2[r])) == (mm.S1, mm.S2, mm.W2), r
    st = oracle_lib.SlopeState(1024).run_dd(3, 1.0, 0.25, 61, block=(512, 64), tile=(4, 4))
    assert np.array_equal(ens.member_words(1), oracle_lib.pack(st.sx, st.sy))
