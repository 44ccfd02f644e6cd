"""ESS estimator pinned on AR(1) chains, whose integrated autocorrelation
time is (1 + phi) / (1 - phi) in closed form."""
import numpy as np

from paper_2511_06407_amd.analysis import ess


def ar1(phi, n, seed):
    rng = np.random.default_rng(seed)
    x = np.empty(n)
    x[0] = rng.standard_normal() / np.sqrt(1 - phi ** 2)
    e = rng.standard_normal(n)
    for t in range(1, n):
        x[t] = phi * x[t - 1] + e[t]
    return x


def test_ess_iid():
    x = np.random.default_rng(0).standard_normal(20000)
    assert abs(ess(x) / 20000 - 1.0) < 0.1


def test_ess_ar1_closed_form():
    for phi in (0.5, 0.9):
        n = 200000
        want = n * (1 - phi) / (1 + phi)
        got = ess(ar1(phi, n, 1))
        assert abs(got / want - 1.0) < 0.1, (phi, got, want)
