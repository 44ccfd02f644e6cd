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


# ---------------------------------------------------------------- g = sqrt(kappa^2 + lambda^2)
def test_sqrt_map_values_and_divided_differences_mpmath():
    """g, g' and the cancellation-free divided difference (lambda_j + lambda_l)
    / (g_j + g_l) against 50-digit evaluation of (g_j - g_l) / (lambda_j -
    lambda_l), including near-equal pairs where the direct quotient cancels."""
    import mpmath as mp
    mp.mp.dps = 50
    sq = softabs.SqrtMap(1.0)
    lam = np.array([-30.0, -1.0, -1e-3, 0.0, 2e-9, 0.7, 0.7 + 1e-12, 5.0, 1e4])
    g, gp = sq.g_gprime(lam)
    T = sq.divided_differences(lam)
    for i, a in enumerate(lam):
        ga = mp.sqrt(1 + mp.mpf(a) ** 2)
        assert abs(g[i] - float(ga)) <= 1e-15 * float(ga)
        assert abs(gp[i] - float(mp.mpf(a) / ga)) <= 1e-15
        for j, b in enumerate(lam):
            if i == j:
                want = mp.mpf(a) / ga
            else:
                gb = mp.sqrt(1 + mp.mpf(b) ** 2)
                want = (ga - gb) / (mp.mpf(a) - mp.mpf(b))
            assert abs(T[i, j] - float(want)) <= 4e-16 * max(1.0, abs(float(want))), (a, b)


def test_sqrt_map_diagonal_closed_form_and_daleckii_krein():
    """On a diagonal H the metric is diag(sqrt(1 + H_ii^2)); on a full H the
    derivative of G = g(H) along a symmetric E is Psi (T o Psi'E Psi) Psi'
    (central differences of the matrix function)."""
    sq = softabs.SqrtMap(1.0)
    d = np.array([-2.0, 0.0, 0.3, 4.0])
    eig = softabs.softabs_eig(np.diag(d), sq)
    assert np.allclose(softabs.metric(eig), np.diag(np.sqrt(1 + d * d)), rtol=1e-14, atol=1e-15)
    assert np.isclose(eig["logdetG"], np.sum(np.log(np.sqrt(1 + d * d))), rtol=1e-14)
    rng = np.random.default_rng(3)
    A = rng.standard_normal((6, 6))
    H = A + A.T
    E = rng.standard_normal((6, 6))
    E = E + E.T
    e0 = softabs.softabs_eig(H, sq)
    T = sq.divided_differences(e0["lam"])
    Psi = e0["Psi"]
    dG = Psi @ (T * (Psi.T @ E @ Psi)) @ Psi.T
    h = 1e-5
    fd = (softabs.metric(softabs.softabs_eig(H + h * E, sq))
          - softabs.metric(softabs.softabs_eig(H - h * E, sq))) / (2 * h)
    assert np.linalg.norm(dG - fd) / np.linalg.norm(fd) < 1e-8


def test_sqrt_map_hamiltonian_gradient_finite_differences():
    """dH/dq with the sqrt softabs against Richardson central differences of
    the Hamiltonian (Eq. d_Hamiltonian with the derived signs)."""
    import dataclasses
    from paper_2511_06407_amd import workloads as wl
    from oracle import hamiltonian as ham
    spec, _, _ = wl.gp_logistic_2d(6, 3)
    T = ham.GPTarget(dataclasses.replace(spec, jitter=1e-2))
    sq = softabs.SqrtMap(1.0)
    rng = np.random.default_rng(2)
    q = 0.4 * rng.standard_normal(T.D)
    p = rng.standard_normal(T.D)
    st = ham.State(T, q, sq)
    got = ham.grad_q(st, p)
    E = np.eye(T.D)

    def cd(hh):
        return np.array([(ham.hamiltonian(ham.State(T, q + hh * E[i], sq), p)
                          - ham.hamiltonian(ham.State(T, q - hh * E[i], sq), p)) / (2 * hh)
                         for i in range(T.D)])
    fd = (4 * cd(5e-4) - cd(1e-3)) / 3
    assert np.linalg.norm(got - fd) / np.linalg.norm(fd) < 1e-8
