"""Pins of the reference U, grad U, H and v(W) = grad tr(W H) by the complex-step
derivative (Squire & Trapp 1998), which is exact to rounding for analytic code,
and of the kernel matrix itself by entries worked out by hand.

Models: every kernel kind (isotropic SE, SE-ARD, linear-ARD, same-value binary),
every likelihood (the mean/variance model of two latent functions included),
a tempered likelihood (beta != 1) and random points q.
Jitter 1e-2 keeps K well conditioned so the bar can be near machine precision.
"""
import dataclasses

import numpy as np
import pytest

from paper_2511_06407_amd import workloads as wl
from oracle import model

H_CS = 1e-30


def small_models():
    a, _, _ = wl.gp_logistic_2d(10, seed=1)
    b, _, _ = wl.gp_logistic_ard4(9, seed=2)
    c, _, _ = wl.propensity_mkl(12, seed=3)
    d, _, _ = wl.gaussian_gp(8, noise_var=0.3, seed=4)
    e, _, _ = wl.mean_variance(6, seed=5, delta=0.05)
    out = []
    for s, beta in ((a, 0.7), (b, 1.0), (c, 0.35), (d, 1.0), (e, 0.8)):
        out.append(dataclasses.replace(s, jitter=1e-2, beta=beta))
    return out


MODELS = small_models()


def rand_q(spec, seed):
    rng = np.random.default_rng(seed)
    q = 0.6 * rng.standard_normal(spec.D)
    return q


def cs_jacobian(fun, q):
    E = np.eye(q.size)
    return np.array([np.imag(fun(q + 1j * H_CS * E[i])) / H_CS for i in range(q.size)])


@pytest.mark.parametrize("k", range(len(MODELS)))
def test_kernel_derivatives_complex_step(k):
    spec = MODELS[k]
    eta = rand_q(spec, 10 + k)[spec.N:]
    kd = model.KernelDerivs(spec, eta)
    P = spec.P
    E = np.eye(P)
    for l in range(P):
        want = np.imag(model.gram(spec, eta + 1j * H_CS * E[l])) / H_CS
        got = kd.d((l,))
        assert np.allclose(got, want, rtol=1e-13, atol=1e-14)
        for m in range(P):
            kd_c = model.KernelDerivs(spec, eta + 1j * H_CS * E[m])
            d1 = kd_c.d((l,))
            want2 = np.zeros_like(got) if d1 is None else np.imag(d1) / H_CS
            got2 = kd.d((l, m))
            got2 = np.zeros_like(want2) if got2 is None else got2
            assert np.allclose(got2, want2, rtol=1e-13, atol=1e-14)
            for n in range(P):
                d2 = kd_c.d((l, n))
                want3 = np.zeros_like(got) if d2 is None else np.imag(d2) / H_CS
                got3 = kd.d((l, n, m))
                got3 = np.zeros_like(want3) if got3 is None else got3
                assert np.allclose(got3, want3, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("k", range(len(MODELS)))
def test_gradient_complex_step(k):
    spec = MODELS[k]
    q = rand_q(spec, k)
    g = model.gradient(spec, q)
    want = cs_jacobian(lambda z: model.neg_log_post(spec, z), q)
    assert np.linalg.norm(g - want) / np.linalg.norm(want) < 1e-13
    U, g2, _ = model.hessian(spec, q)
    assert abs(U - model.neg_log_post(spec, q)) < 1e-12 * max(1.0, abs(U))
    assert np.allclose(g2, g, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("k", range(len(MODELS)))
def test_hessian_complex_step(k):
    spec = MODELS[k]
    q = rand_q(spec, 20 + k)
    H = model.hessian(spec, q)[2]
    want = cs_jacobian(lambda z: model.gradient(spec, z), q)
    assert np.linalg.norm(H - want) / np.linalg.norm(want) < 1e-13
    assert np.array_equal(H, H.T)


@pytest.mark.parametrize("k", range(len(MODELS)))
def test_contraction_complex_step(k):
    spec = MODELS[k]
    q = rand_q(spec, 30 + k)
    rng = np.random.default_rng(40 + k)
    W = rng.standard_normal((spec.D, spec.D))
    W = W + W.T
    v = model.contract(spec, q, W)
    want = cs_jacobian(lambda z: np.sum(W * model.hessian(spec, z)[2]), q)
    assert np.linalg.norm(v - want) / np.linalg.norm(want) < 1e-12


def test_gaussian_likelihood_fixed_eta_textbook():
    """With a Gaussian likelihood the f-block of H is K^-1 + I/s2 and the
    f-gradient vanishes at the textbook posterior mean K (K + s2 I)^-1 y
    (Rasmussen & Williams, Sec. 2.2)."""
    spec = MODELS[3]
    eta = np.array([0.2, -0.3])
    K = model.gram(spec, eta)
    s2 = spec.noise_var
    mean = K @ np.linalg.solve(K + s2 * np.eye(spec.N), spec.y)
    q = np.concatenate([mean, eta])
    U, g, H = model.hessian(spec, q)
    assert np.max(np.abs(g[:spec.N])) < 1e-10
    assert np.allclose(H[:spec.N, :spec.N], np.linalg.inv(K) + np.eye(spec.N) / s2, rtol=1e-12)


# Kernel values worked out by hand on three points, one kernel kind at a time
# (Sec. 2.1, Eq. BMKL: the prior covariance is the sum of the terms).  They fix
# the conventions the complex-step pins cannot see, since those differentiate
# the same function they check: the SE amplitude enters as s^2 and the
# lengthscale as l^2 in exp(-r^2 / (2 l^2)), linear-ARD variances as e^eta,
# same-value kernels as s^2 [x_c == x'_c], and the jitter sits on the diagonal.
GRAM_X = np.array([[0.0, 0.0, 1.0, 0.0],
                   [1.0, 0.0, 2.0, 1.0],
                   [0.0, 2.0, 0.0, 1.0]])
E = np.exp


def _gram_cases():
    ln = np.log
    se_iso = ([(wl.SE_ISO, (0, 1))], [ln(2.0), ln(0.5)],     # s = 2, l = 1/2: 4 exp(-2 r^2)
              4.0 * np.array([[1, E(-2.0), E(-8.0)], [E(-2.0), 1, E(-10.0)], [E(-8.0), E(-10.0), 1]]))
    se_ard = ([(wl.SE_ARD, (0, 1, 2))], [0.0, 0.0, ln(2.0), ln(0.5 ** 0.5)],   # 2 l_d^2 = 2, 8, 1
              np.array([[1, E(-1.5), E(-1.5)], [E(-1.5), 1, E(-5.0)], [E(-1.5), E(-5.0), 1]]))
    lin = ([(wl.LINEAR_ARD, (0, 2))], [ln(3.0), ln(0.5)],   # 3 x0 x0' + x2 x2' / 2
           np.array([[0.5, 1.0, 0.0], [1.0, 5.0, 0.0], [0.0, 0.0, 0.0]]))
    same = ([(wl.BINARY_SAME, (3,))], [ln(1.5)],           # 2.25 [x3 == x3']
            2.25 * np.array([[1, 0, 0], [0, 1, 1], [0, 1, 1]]))
    cases = {"se_iso": se_iso, "se_ard": se_ard, "linear_ard": lin, "binary_same": same}
    cases["sum"] = (se_iso[0] + se_ard[0] + lin[0] + same[0],
                    se_iso[1] + se_ard[1] + lin[1] + same[1],
                    se_iso[2] + se_ard[2] + lin[2] + same[2])
    return cases


GRAM_CASES = _gram_cases()


@pytest.mark.parametrize("name", list(GRAM_CASES))
def test_gram_hand_values(name):
    terms, eta, want = GRAM_CASES[name]
    jitter = 0.125
    spec = wl.ModelSpec(X=GRAM_X, y=np.zeros(3), terms=terms, jitter=jitter)
    assert spec.P == len(eta)
    K = model.gram(spec, np.array(eta))
    assert np.allclose(K, want + jitter * np.eye(3), rtol=1e-14, atol=1e-15)


def test_mean_variance_likelihood_is_the_normal_density():
    """Sec. 2.1 Example 1: the per-record term is -ln N(y; f1, delta + exp f2),
    checked against scipy's normal log density."""
    from scipy.stats import norm
    spec, _, _ = wl.mean_variance(7, seed=3, delta=0.02)
    f = 0.8 * np.random.default_rng(1).standard_normal(spec.N)
    R = spec.n_records
    want = -norm.logpdf(spec.y[:R], loc=f[:R], scale=np.sqrt(0.02 + np.exp(f[R:])))
    assert np.allclose(model.mv_value(spec, f), want, rtol=1e-14, atol=1e-14)
    assert abs(model.lik_sum(spec, f) - want.sum()) < 1e-12 * abs(want.sum())


def test_mean_variance_prior_is_block_diagonal():
    """Each latent function has its own GP prior (Sec. 2.1): the stacked K is
    blockdiag(K1(eta_1), K2(eta_2)) + jitter, with K_j the Gram matrix of
    term j alone on the records' covariates."""
    spec, _, _ = wl.mean_variance(5, seed=2)
    eta = np.random.default_rng(0).standard_normal(spec.P)
    R = spec.n_records
    x = spec.X[:R, :2]
    (k1, c1), (k2, c2) = spec.terms
    n1 = wl.term_nparams(k1, c1)
    s1 = wl.ModelSpec(X=x, y=np.zeros(R), terms=[(k1, c1)], jitter=spec.jitter)
    s2 = wl.ModelSpec(X=x, y=np.zeros(R), terms=[(k2, c2)], jitter=spec.jitter)
    K = model.gram(spec, eta)
    assert np.array_equal(K[:R, R:], np.zeros((R, R))) and np.array_equal(K[R:, :R], np.zeros((R, R)))
    assert np.allclose(K[:R, :R], model.gram(s1, eta[:n1]), rtol=1e-15, atol=0)
    assert np.allclose(K[R:, R:], model.gram(s2, eta[n1:]), rtol=1e-15, atol=0)
