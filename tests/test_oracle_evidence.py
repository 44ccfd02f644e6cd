"""Pins of the thermodynamic-integration evidence estimate (appendix on
model evidence) and of the quadrature reference for Gaussian-likelihood GP
models."""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_2511_06407_amd import workloads as wl
from oracle import evidence, model


def test_paper_schedule():
    """The 101 rungs printed in Sec. 2.5: from 1 down to 0 in steps of 0.02,
    0.005, 0.002 and 0.001, changing at 0.2, 0.05 and 0.01."""
    t = evidence.paper_schedule()
    assert t.size == 101 and t[0] == 1.0 and abs(t[-1]) < 1e-15
    assert np.all(np.diff(t) < 0)
    for s, want in ((41, 0.2), (71, 0.05), (91, 0.01), (2, 0.98), (42, 0.195), (72, 0.048),
                    (92, 0.009)):
        assert math.isclose(t[s - 1], want, abs_tol=1e-14)
    steps = -np.diff(t)
    assert np.allclose(steps[:40], 0.02) and np.allclose(steps[40:70], 0.005)
    assert np.allclose(steps[70:90], 0.002) and np.allclose(steps[90:], 0.001)


def test_trapezoid_exact_for_linear_integrand():
    t = evidence.paper_schedule()
    a, b = -3.0, 2.5
    L = np.tile(a + b * t, (4, 1))
    est, var, E = evidence.ti_estimate(t, L)
    assert math.isclose(est, a + b / 2, rel_tol=1e-13)
    assert var == 0.0


def test_conjugate_gaussian_identity():
    """x ~ N(0, 1), y | x ~ N(x, s2): the power posterior at tau is Gaussian
    with precision 1 + tau/s2, so E_tau[ln p(y|x)] is in closed form and its
    integral over [0, 1] must equal ln N(y; 0, 1 + s2) (the identity the
    estimate rests on, with the orientation of the decreasing schedule)."""
    y, s2 = 1.7, 0.3
    t = evidence.paper_schedule()
    prec = 1.0 + t / s2
    m = (t * y / s2) / prec
    v = 1.0 / prec
    E = -0.5 * math.log(2 * math.pi * s2) - ((y - m) ** 2 + v) / (2 * s2)
    est, _, _ = evidence.ti_estimate(t, E[None, :])
    exact = -0.5 * math.log(2 * math.pi * (1 + s2)) - y * y / (2 * (1 + s2))
    assert abs(est - exact) < 2e-3     # trapezoid discretisation on this schedule
    # a finer uniform grid converges to the exact value
    tf = np.linspace(1.0, 0.0, 20001)
    pf = 1.0 + tf / s2
    mf = (tf * y / s2) / pf
    Ef = -0.5 * math.log(2 * math.pi * s2) - ((y - mf) ** 2 + 1.0 / pf) / (2 * s2)
    estf, _, _ = evidence.ti_estimate(tf, Ef[None, :])
    assert abs(estf - exact) < 1e-8


def test_variance_formula_monte_carlo():
    """With independent rung values of known per-rung variance the spread of
    a single chain's estimate matches the formula."""
    rng = np.random.default_rng(0)
    t = evidence.paper_schedule()
    sd = 0.5 + 3.0 * (1.0 - t)                       # per-rung standard deviations
    reps = rng.standard_normal((20000, t.size)) * sd + 10.0 * t
    ests = [evidence.ti_estimate(t, r[None, :])[0] for r in reps]
    _, var, _ = evidence.ti_estimate(t, reps[:2000])   # formula with sampled Var_s
    w = t[:-1] - t[1:]
    c = np.zeros(t.size)
    c[:-1] += 0.5 * w
    c[1:] += 0.5 * w
    exact_var = float(np.sum(c * c * sd * sd))
    assert abs(np.var(ests) / exact_var - 1.0) < 0.05
    assert abs(var / exact_var - 1.0) < 0.1
    # the appendix's printed coefficients (w_(s-1)^2 + w_s^2)/4 miss the cross
    # term: on this schedule they give about half the observed spread
    paper = 0.25 * (sd[0] ** 2 * w[0] ** 2 + sd[-1] ** 2 * w[-1] ** 2) + sum(
        0.25 * sd[s] ** 2 * (w[s - 1] ** 2 + w[s] ** 2) for s in range(1, t.size - 1))
    assert 0.4 < paper / np.var(ests) < 0.6


@pytest.mark.parametrize("P", [1, 2])
def test_gaussian_log_evidence_against_adaptive_quadrature(P):
    """The Gauss-Hermite evidence of a Gaussian-likelihood GP against scipy's
    adaptive quadrature of the same integral over eta (P = 1: one amplitude
    of a same-value kernel; P = 2: amplitude and lengthscale of an SE kernel)."""
    rng = np.random.default_rng(P)
    if P == 1:
        X = np.array([[0.0], [1.0], [1.0], [0.0]])
        terms = [(wl.BINARY_SAME, (0,))]
    else:
        X = rng.uniform(-1, 1, size=(4, 2))
        terms = [(wl.SE_ISO, (0, 1))]
    y = rng.standard_normal(4)
    spec = wl.ModelSpec(X=X, y=y, terms=terms, lik=wl.LIK_GAUSSIAN, noise_var=0.4, jitter=1e-6)
    got = evidence.gaussian_log_evidence(spec, 160 if P == 2 else 400)

    def integrand(*eta):
        C = model.gram(spec, np.array(eta)) + spec.noise_var * np.eye(4)
        _, logdet = np.linalg.slogdet(C)
        ll = -0.5 * (y @ np.linalg.solve(C, y) + logdet + 4 * math.log(2 * math.pi))
        return math.exp(ll) * np.prod([math.exp(-0.5 * e * e) / math.sqrt(2 * math.pi) for e in eta])
    if P == 1:
        val, _ = integrate.quad(integrand, -9, 9, epsabs=1e-16, epsrel=1e-12)
    else:
        val, _ = integrate.dblquad(lambda b, a: integrand(a, b), -9, 9, -9, 9,
                                   epsabs=1e-16, epsrel=1e-12)
    assert abs(got - math.log(val)) < 1e-9


def _small_gaussian_spec():
    rng = np.random.default_rng(11)
    X = rng.uniform(-1, 1, size=(4, 2))
    y = rng.standard_normal(4)
    return wl.ModelSpec(X=X, y=y, terms=[(wl.SE_ISO, (0, 1))], lik=wl.LIK_GAUSSIAN,
                        noise_var=0.3, jitter=1e-3)


def test_power_posterior_normaliser_and_rung_mean():
    """ln Z(1) of the power posterior is the evidence (a different route from
    gaussian_log_evidence: the tempered-likelihood rescaling at tau = 1);
    ln Z(0) = 0; the closed-form rung mean E(tau) is the derivative of
    ln Z(tau) (central differences); and the integral of E over [0, 1] (a
    composite Gauss-Legendre rule in tau) gives back ln Z(1)."""
    spec = _small_gaussian_spec()
    n = 60
    lz1, _ = evidence.gaussian_power_posterior(spec, 1.0, n)
    assert abs(lz1 - evidence.gaussian_log_evidence(spec, n)) < 1e-10
    lz0, _ = evidence.gaussian_power_posterior(spec, 0.0, n)
    assert abs(lz0) < 1e-12
    for tau in (0.02, 0.5, 0.9):
        h = 1e-5
        a, _ = evidence.gaussian_power_posterior(spec, tau + h, n)
        b, _ = evidence.gaussian_power_posterior(spec, tau - h, n)
        _, e = evidence.gaussian_power_posterior(spec, tau, n)
        assert abs((a - b) / (2 * h) - e) < 1e-6 * (1 + abs(e))
    # E changes fastest near tau = 0: a composite rule on geometric pieces
    x, w = np.polynomial.legendre.leggauss(16)
    edges = [0.0, 1e-4, 1e-3, 1e-2, 0.1, 1.0]
    integral = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        integral += sum(0.5 * (hi - lo) * wi * evidence.gaussian_power_posterior(
            spec, lo + 0.5 * (hi - lo) * (xi + 1), 30)[1] for xi, wi in zip(x, w))
    assert abs(integral - evidence.gaussian_power_posterior(spec, 1.0, 30)[0]) < 1e-6


def test_prior_rung_mean_by_sampling():
    """At tau = 0 the rung mean is the prior expectation of ln p(y | f),
    checked against plain Monte Carlo over eta ~ N(0, I), f ~ N(0, K(eta))."""
    spec = _small_gaussian_spec()
    _, e0 = evidence.gaussian_power_posterior(spec, 0.0, 60)
    rng = np.random.default_rng(5)
    vals = []
    for _ in range(20000):
        eta = rng.standard_normal(spec.P)
        f = np.linalg.cholesky(model.gram(spec, eta)) @ rng.standard_normal(spec.N)
        vals.append(-0.5 * spec.N * math.log(2 * math.pi * spec.noise_var)
                    - 0.5 * np.sum((spec.y - f) ** 2) / spec.noise_var)
    vals = np.array(vals)
    assert abs(vals.mean() - e0) < 4 * vals.std() / math.sqrt(vals.size)
