"""Pins of the softabs scalar functions against 50-digit mpmath.

g(lambda) = lambda coth(alpha lambda) (Sec. 2.5, coth form) evaluated through
h(x) = x coth x; T = divided differences (Sec. 2.2, Eq. d3_transform).
"""
import numpy as np
import pytest

mpmath = pytest.importorskip("mpmath")
from oracle import softabs  # noqa: E402

mpmath.mp.dps = 50


def mp_h(x):
    x = mpmath.mpf(x)
    if x == 0:
        return mpmath.mpf(1)
    return x * mpmath.coth(x)


def mp_h1(x):
    return mpmath.diff(mp_h, mpmath.mpf(x)) if x != 0 else mpmath.mpf(0)


def grid():
    pos = np.logspace(-8, 3, 400)
    return np.concatenate([pos, -pos, [0.0, 0.49999, 0.5, 0.50001, 19.999, 20.0, 20.001]])


def test_series_coefficients_are_x_coth_x():
    # coefficients of x coth x: 1, 1/3, -1/45, 2/945, -1/4725, 2/93555
    want = [1.0, 1 / 3, -1 / 45, 2 / 945, -1 / 4725, 2 / 93555]
    assert np.allclose(softabs._COEF[:6], want, rtol=1e-15, atol=0)


def test_h_against_mpmath():
    x = grid()
    got = softabs.h(x)
    want = np.array([float(mp_h(v)) for v in x])
    assert np.max(np.abs(got - want) / np.abs(want)) < 2e-15


def test_h1_against_mpmath():
    x = grid()
    got = softabs.h1(x)
    want = np.array([float(mp_h1(v)) for v in x])
    err = np.abs(got - want) / np.maximum(np.abs(want), 1e-300)
    # |h'| ~ 2x/3 near 0, so compare absolutely there
    small = np.abs(x) < 1e-6
    assert np.max(err[~small]) < 2e-14
    assert np.max(np.abs(got - want)[small]) < 1e-20


def test_h3_against_mpmath():
    x = np.concatenate([np.linspace(-19.5, 19.5, 157), [0.3, -0.3, 0.7]])
    got = softabs.h3(x)
    want = np.array([float(mpmath.diff(mp_h, mpmath.mpf(v), 3)) for v in x])
    assert np.max(np.abs(got - want)) < 1e-11


def test_g_limits():
    lam = np.array([1e-12, -1e-12, 1.0, -3.0, 0.0])
    g, gp = softabs.g_gprime(lam, 1e6)
    assert np.allclose(g[:2], 1e-6, rtol=1e-9)       # g(0) = 1/alpha
    assert g[2] == 1.0 and g[3] == 3.0 and g[4] == 1e-6
    assert gp[2] == 1.0 and gp[3] == -1.0


def test_divided_differences_against_mpmath():
    rng = np.random.default_rng(0)
    alpha = 1e6
    lam = np.concatenate([rng.uniform(-5e-5, 5e-5, 20), [1e-5, 1e-5 + 1e-13, 2e-5, -3e-5, 4.0, -4.0, 1e3]])
    T = softabs.divided_differences(lam, alpha)

    def g(l):
        return mp_h(mpmath.mpf(alpha) * mpmath.mpf(l)) / alpha

    worst = 0.0
    for j in range(lam.size):
        for l in range(lam.size):
            if j == l or lam[j] == lam[l]:
                want = mpmath.diff(lambda t: g(t), mpmath.mpf(lam[j]))
            else:
                want = (g(lam[j]) - g(lam[l])) / (mpmath.mpf(lam[j]) - mpmath.mpf(lam[l]))
            worst = max(worst, abs(T[j, l] - float(want)) / max(abs(float(want)), 1e-3))
    assert worst < 1e-12
