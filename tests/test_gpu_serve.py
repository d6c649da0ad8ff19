"""Job pool / serving: continuous batching with admission by HBM budget.
Each job's result is the same alone and in the mix (bit-exact moments),
whatever the quantum and whatever runs beside it."""
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


def alone(kpz, L, p, q, seed, n, block=None):
    sim = kpz.Sim(L, p, q, seed, block or kpz.POOL_BLOCK)
    sim.sweep(n)
    m = sim.roughness()
    sim.close()
    return m


JOBS = [(256, 1.0, 0.0, 11, 7), (512, 1.0, 0.3, 12, 19), (256, 1.0, 0.5, 13, 3),
        (1024, 1.0, 0.1, 14, 11), (256, 1.0, 0.25, 15, 40), (512, 1.0, 0.0, 16, 1)]


@pytest.mark.parametrize("quantum", [1, 4, 16])
def test_pool_results_equal_standalone(gpu, quantum):
    pool = gpu.Pool(256 << 20, max_jobs=16, max_quantum=16)
    ids = {}
    results = {}
    # staggered: half now, the rest after two steps
    for j in JOBS[:3]:
        ids[pool.submit(gpu.make_params(*j[:4]), j[4])] = j
    for _ in range(2):
        pool.step(quantum)
        results.update(dict(pool.poll()))
    for j in JOBS[3:]:
        ids[pool.submit(gpu.make_params(*j[:4]), j[4])] = j
    while len(results) < len(JOBS):
        pool.step(quantum)
        results.update(dict(pool.poll()))
    assert set(results) == set(ids)
    for jid, j in ids.items():
        ref = alone(gpu, *j)
        got = results[jid]
        assert (got.S1, got.S2, got.W2) == (ref.S1, ref.S2, ref.W2), j


def test_pool_admission_by_budget(gpu):
    kpz = gpu
    one = kpz.make_params(1024, 1.0, 0.0, 3)
    probe = kpz.Pool(64 << 20, max_jobs=8, max_quantum=8)
    job_bytes = probe.job_bytes(one)
    probe.close()
    ctl = kpz.Pool.control_bytes(8)
    pool = kpz.Pool(ctl + job_bytes + job_bytes // 2, max_jobs=8, max_quantum=8)
    a = pool.submit(one, 5)
    assert a is not None
    assert pool.submit(kpz.make_params(1024, 1.0, 0.0, 4), 5) is None   # does not fit now
    while pool.stats()[0]:
        pool.step(8)
    (jid, m), = pool.poll()
    assert jid == a and (m.S1, m.S2, m.W2) == tuple(vars(alone(kpz, 1024, 1.0, 0.0, 3, 5)).values())
    assert pool.submit(kpz.make_params(1024, 1.0, 0.0, 4), 5) is not None   # fits after release


def test_serve_small_poisson_run(gpu):
    from paper_1204_5072_amd import serve
    jobs = serve.poisson_jobs(n_jobs=40, rate=400.0, seed=3, log2L=(8, 10), log10_mcs=(1.0, 2.0))
    rep = serve.serve(jobs, hbm_bytes=256 << 20, quantum=8)
    assert rep.jobs == 40 and all(j.result is not None for j in jobs)
    assert 0 < rep.latency_p50_ms <= rep.latency_p99_ms
    for j in jobs[:6]:
        ref = alone(gpu, j.L, j.p, j.q, j.seed, j.n_mcs)
        assert (j.result.S1, j.result.S2, j.result.W2) == (ref.S1, ref.S2, ref.W2)
