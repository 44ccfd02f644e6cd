"""Pins of the reference for the paper's reduced-rank basis model.

* The features and V_m against the kernel they approximate: with the 1/L
  factor restored, sum_m V_m phi_m(x) phi_m(x') / L converges to
  exp(-(x - x')^2 / sigma) (the approximation of the appendix on the
  reduced-rank representation) -- this fixes the pi^2 in V_m.
* U against scipy's densities (normal, inverse Gamma, Bernoulli).
* Gradient, Hessian and contraction by the complex step of U, of the
  gradient and of tr(W H) (exact to rounding for analytic code).
"""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2511_06407_amd import workloads as wl
from oracle import basis

H_CS = 1e-30


def small_specs():
    s1, _ = wl.basis_logistic(2, N=12, seed=1, M=4)
    rng = np.random.default_rng(3)
    X = np.column_stack([rng.standard_normal(10), rng.integers(0, 2, 10).astype(float),
                         rng.standard_normal(10)])
    s2 = wl.BasisSpec(X=X, y=rng.standard_normal(10), kinds=(wl.BASIS_GAUSS, wl.BASIS_LINEAR,
                                                               wl.BASIS_GAUSS),
                      M=3, L=4.0, bias_var=0.7, ig_alpha=(5.0, 1.0, 5.0), ig_beta=(0.5, 1.0, 0.5),
                      lik=wl.LIK_GAUSSIAN, noise_var=0.4, beta=0.6)
    return [s1, s2]


SPECS = small_specs()


def rand_q(spec, seed):
    rng = np.random.default_rng(seed)
    q = 0.5 * rng.standard_normal(spec.D)
    q[-3:] = rng.uniform(0.5, 2.0, 3)          # positive hyperparameters
    return q


def test_features_approximate_the_gaussian_kernel():
    L, M, sigma = 8.0, 160, 1.3
    x = np.linspace(-2.5, 2.5, 9)
    spec = wl.BasisSpec(X=x[:, None], y=np.zeros(x.size), kinds=(wl.BASIS_GAUSS,), M=M, L=L)
    Phi, kind, kappa = basis.features(spec)
    V = np.exp(basis.log_v(sigma, kappa))
    K = (Phi[:, :-1] * V) @ Phi[:, :-1].T / L
    want = np.exp(-(x[:, None] - x[None, :]) ** 2 / sigma)
    assert np.max(np.abs(K - want)) < 1e-10
    # the exponent printed with pi in place of pi^2 does not approximate it
    Vp = np.sqrt(math.pi * sigma) * np.exp(-math.pi * np.arange(1, M + 1) ** 2 * sigma / (16 * L * L))
    Kp = (Phi[:, :-1] * Vp) @ Phi[:, :-1].T / L
    assert np.max(np.abs(Kp - want)) > 0.1


def test_generator_matches_the_recipe():
    spec, f = wl.basis_logistic(3, N=400, seed=2)
    assert spec.D == 30 * 3 + 4 and spec.N == 400
    assert abs(np.std(f) - 1.5) < 1e-12
    assert set(np.unique(spec.y)) <= {0.0, 1.0}


@pytest.mark.parametrize("k", range(len(SPECS)))
def test_neg_log_post_against_scipy(k):
    spec = SPECS[k]
    q = rand_q(spec, 5 + k)
    Phi, kind, kappa = basis.features(spec)
    F = spec.n_features
    a, b, cg, sg, cl = q[:F], q[F], q[F + 1], q[F + 2], q[F + 3]
    f = Phi[:, :-1] @ a + b
    if spec.lik == wl.LIK_BERNOULLI_LOGIT:
        ll = stats.bernoulli.logpmf(spec.y, 1.0 / (1.0 + np.exp(-f))).sum()
    else:
        ll = stats.norm.logpdf(spec.y, f, math.sqrt(spec.noise_var)).sum()
    sd = np.sqrt(np.where(kind == 0, cg * np.sqrt(math.pi * sg) * np.exp(-kappa * sg), cl))
    lp = stats.norm.logpdf(a, 0.0, sd).sum() + stats.norm.logpdf(b, 0.0, math.sqrt(spec.bias_var))
    for th, al, be in zip((cg, sg, cl), spec.ig_alpha, spec.ig_beta):
        lp += stats.invgamma.logpdf(th, al, scale=be)
    want = -(spec.beta * ll + lp)
    assert abs(basis.neg_log_post(spec, q) - want) < 1e-12 * abs(want)
    assert abs(basis.log_likelihood(spec, q) - ll) < 1e-12 * abs(ll)


@pytest.mark.parametrize("k", range(len(SPECS)))
def test_gradient_and_hessian_complex_step(k):
    spec = SPECS[k]
    q = rand_q(spec, 7 + k)
    U, g, H = basis.derivs(spec, q)
    E = np.eye(spec.D)
    g_cs = np.array([np.imag(basis.neg_log_post(spec, q + 1j * H_CS * E[i])) / H_CS
                     for i in range(spec.D)])
    assert np.allclose(g, g_cs, rtol=1e-12, atol=1e-12)
    H_cs = np.array([np.imag(basis.derivs(spec, q + 1j * H_CS * E[i])[1]) / H_CS
                     for i in range(spec.D)])
    assert np.allclose(H, H_cs, rtol=1e-12, atol=1e-11)
    assert np.allclose(H, H.T, rtol=0, atol=1e-12)


@pytest.mark.parametrize("k", range(len(SPECS)))
def test_contraction_complex_step(k):
    spec = SPECS[k]
    q = rand_q(spec, 9 + k)
    rng = np.random.default_rng(10 + k)
    W = rng.standard_normal((spec.D, spec.D))
    W = W + W.T
    v = basis.contract(spec, q, W)
    E = np.eye(spec.D)
    v_cs = np.array([np.imag(np.sum(W * basis.derivs(spec, q + 1j * H_CS * E[i])[2])) / H_CS
                     for i in range(spec.D)])
    assert np.allclose(v, v_cs, rtol=1e-11, atol=1e-10)
