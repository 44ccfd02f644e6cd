"""Pins of the reference softabs metric (Sec. 2.2) against closed forms and
finite differences that do not use its own formulas."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import softabs


def rand_sym(D, seed, spec=None):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((D, D)))
    lam = rng.standard_normal(D) * 3 if spec is None else spec
    return (Q * lam) @ Q.T


def G_of(H, alpha):
    return softabs.metric(softabs.softabs_eig(H, alpha))


def test_diagonal_closed_form():
    d = np.array([3.0, -2.0, 1e-7, -4e-6, 0.0, 50.0])
    H = np.diag(d)
    eig = softabs.softabs_eig(H, 1e6)
    g, _ = softabs.g_gprime(d, 1e6)
    assert np.allclose(softabs.metric(eig), np.diag(g), rtol=1e-14, atol=1e-20)
    assert abs(eig["logdetG"] - np.sum(np.log(g))) < 1e-12


def test_saturated_metric_is_matrix_absolute_value():
    """For |alpha lam| >= 20 everywhere, G = |H| = (H^2)^(1/2) and
    log|G| = log|det H| (computed here by LU and the matrix square root)."""
    rng = np.random.default_rng(1)
    lam = rng.uniform(0.01, 5.0, 30) * rng.choice([-1, 1], 30)
    H = rand_sym(30, 2, lam)
    G = G_of(H, 1e6)
    absH = np.real(sla.sqrtm(H @ H))
    assert np.linalg.norm(G - absH) / np.linalg.norm(absH) < 1e-12
    sign, logabs = np.linalg.slogdet(H)
    assert abs(softabs.softabs_eig(H, 1e6)["logdetG"] - logabs) < 1e-11


@pytest.mark.parametrize("alpha,scale", [(3.0, 1.0), (1e6, 1e-5), (1e6, 1.0)])
def test_daleckii_krein_against_finite_differences(alpha, scale):
    """Psi' dG Psi = T o (Psi' dH Psi)  (Eq. d3_transform) vs central
    differences of the matrix function g(H + t E)."""
    rng = np.random.default_rng(3)
    D = 12
    lam = scale * rng.standard_normal(D)
    lam[1] = lam[0] + 1e-9 * scale            # a near-degenerate pair
    H = rand_sym(D, 4, lam)
    E = rng.standard_normal((D, D))
    E = E + E.T
    eig = softabs.softabs_eig(H, alpha)
    T = softabs.divided_differences(eig["lam"], alpha)
    Psi = eig["Psi"]
    dG = Psi @ (T * (Psi.T @ E @ Psi)) @ Psi.T
    t = 1e-4 * scale
    fd1 = (G_of(H + t * E, alpha) - G_of(H - t * E, alpha)) / (2 * t)
    fd2 = (G_of(H + t / 2 * E, alpha) - G_of(H - t / 2 * E, alpha)) / t
    fd = (4 * fd2 - fd1) / 3
    assert np.linalg.norm(dG - fd) / np.linalg.norm(fd) < 1e-7


@pytest.mark.parametrize("alpha", [2.0, 1e6])
def test_w_matrices_are_the_two_traces(alpha):
    """tr(W2 E) = d/dt log|G(H+tE)| and tr(W1 E) = -d/dt p'G(H+tE)^-1 p
    (Eq. Betancourt_formula), both checked by central differences."""
    rng = np.random.default_rng(5)
    D = 10
    lam = rng.standard_normal(D) * (1e-6 if alpha > 1e3 else 1.0)
    lam[-3:] = [2.0, -1.5, 0.7]
    H = rand_sym(D, 6, lam)
    E = rng.standard_normal((D, D))
    E = E + E.T
    p = rng.standard_normal(D)
    eig = softabs.softabs_eig(H, alpha)
    W1, W2, _, _ = softabs.w_matrices(eig, p, alpha)

    def logdet(t):
        return softabs.softabs_eig(H + t * E, alpha)["logdetG"]

    def quad(t):
        e = softabs.softabs_eig(H + t * E, alpha)
        return p @ softabs.ginv_p(e, p)

    t = 1e-3 * (1e-6 if alpha > 1e3 else 1.0)
    for fun, want_sign, W in ((logdet, 1.0, W2), (quad, -1.0, W1)):
        d1 = (fun(t) - fun(-t)) / (2 * t)
        d2 = (fun(t / 2) - fun(-t / 2)) / t
        fd = (4 * d2 - d1) / 3
        got = want_sign * np.sum(W * E)
        assert abs(got - fd) < 1e-6 * max(1.0, abs(fd))
