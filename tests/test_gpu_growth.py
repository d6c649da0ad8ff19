"""Growth laws at the L = 4096 workload (flat start, 10^4 MCS, W^2 at 64
log-spaced times, 8 seeds each):

* p = 1, q = 0 (KPZ): W ~ t^beta with beta close to 0.24 in 2+1 dimensions
  (the value the cited high-precision octahedron simulations report);
* p = q = 1/2 (Edwards-Wilkinson): W^2 grows logarithmically.

Both run as one ensemble each (one captured graph of per-MCS launches).
Far below saturation: t_x ~ L^1.6 >> 10^4 at L = 4096.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def log_times(n=64, t_max=10_000):
    out = []
    for k in range(n):
        out.append(int(max((out[-1] + 1) if out else 1, round(t_max ** (k / (n - 1))))))
    return out


@pytest.fixture(scope="module")
def runs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1204_5072_amd as kpz
    times = np.array(log_times())
    out = {}
    for name, (p, q) in {"kpz": (1.0, 0.0), "ew": (0.5, 0.5)}.items():
        members = [kpz.make_params(4096, p, q, seed) for seed in range(1, 9)]
        ens = kpz.Ensemble(members)
        S1, S2, W2 = ens.run(list(times))
        out[name] = W2.mean(axis=1)
        ens.close()
    return times, out


def test_kpz_growth_exponent(runs):
    times, w2 = runs
    sel = (times >= 100) & (times <= 10_000)
    beta = np.polyfit(np.log(times[sel]), np.log(w2["kpz"][sel]), 1)[0] / 2
    print("beta_KPZ", beta, flush=True)
    assert 0.22 <= beta <= 0.26, beta


def test_ew_logarithmic_growth(runs):
    times, w2 = runs
    sel = (times >= 100) & (times <= 10_000)
    x = np.log(times[sel])
    coef = np.polyfit(x, w2["ew"][sel], 1)
    resid = w2["ew"][sel] - np.polyval(coef, x)
    print("EW W^2 = a + b ln t:", coef, "max residual", np.abs(resid).max(), flush=True)
    assert coef[0] > 0
    assert np.abs(resid).max() < 0.03 * w2["ew"][sel].max()
    beta_ew = np.polyfit(x, np.log(w2["ew"][sel]), 1)[0] / 2
    assert beta_ew < 0.12
