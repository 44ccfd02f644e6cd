"""Soft-absolute metric: g(lambda) = lambda coth(alpha lambda) or
g(lambda) = sqrt(kappa^2 + lambda^2), its derivative, the divided-difference
matrix T and the cached products W1, W2.  FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper anchors
-------------
* Softabs map H = sum lam psi psi' -> G = sum g(lam) psi psi': Sec. 2.2.
* Divided differences T (Daleckii-Krein form of Psi' dG Psi): Sec. 2.2,
  Eq. (d3_transform).
* Cached W1 = Psi B T B Psi', W2 = Psi (R o T) Psi' with
  B = diag((Psi'p)_i / g_i), R = diag(1/g_i): Sec. 2.2, Eq. (Betancourt_formula).
* The coth form with kappa^-1 = alpha is the form the paper attributes to
  Hamiltorch (Sec. 2.5); it is singular-looking at 0, so it is evaluated here
  in x = alpha*lambda with h(x) = x coth x, g = h/alpha, g' = h'(x):
    |x| >= 20         : h = |x|, h' = sign x (coth 20 - 1 < 2^-53)
    |x| <  0.5        : Taylor series of x coth x (radius pi), 12 terms
    otherwise         : h = x / tanh x, h' = (sinh(2x)/2 - x) / sinh(x)^2.
* The form the paper's own runs use (Sec. 2.5): g = sqrt(kappa^2 + lambda^2),
  g' = lambda / g, and the divided difference written without cancellation,
  (g_j - g_l) / (lambda_j - lambda_l) = (lambda_j + lambda_l) / (g_j + g_l)
  (multiply by g_j + g_l and use g^2 = kappa^2 + lambda^2).  It is selected
  by passing SqrtMap(kappa) wherever `alpha` is taken.
"""
from __future__ import annotations

import math
from fractions import Fraction
from math import comb

import numpy as np

X_SAT = 20.0
X_SERIES = 0.5
N_SERIES = 12


def _bernoulli_even(n_terms):
    """B_0, B_2, ..., B_{2(n_terms-1)} as exact fractions, from the recurrence
    sum_{k=0}^{m} C(m+1, k) B_k = 0 (B_0 = 1)."""
    m_max = 2 * (n_terms - 1)
    B = [Fraction(1)]
    for m in range(1, m_max + 1):
        B.append(-sum(comb(m + 1, k) * B[k] for k in range(m)) / Fraction(m + 1))
    return [B[2 * n] for n in range(n_terms)]


# x coth x = sum_n 2^(2n) B_2n x^(2n) / (2n)!
_COEF = [float(Fraction(2) ** (2 * n) * b / math.factorial(2 * n))
         for n, b in enumerate(_bernoulli_even(N_SERIES))]


def h_series(x, deriv=0):
    """Term-wise series of x coth x (deriv = 0, 1 or 3)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    for n, c in enumerate(_COEF):
        k = 2 * n
        if deriv == 0:
            out = out + c * x ** k
        elif deriv == 1:
            if k >= 1:
                out = out + c * k * x ** (k - 1)
        elif deriv == 3:
            if k >= 3:
                out = out + c * k * (k - 1) * (k - 2) * x ** (k - 3)
        else:
            raise ValueError(deriv)
    return out


def h(x):
    x = np.asarray(x, dtype=np.float64)
    ax = np.abs(x)
    out = np.empty_like(x)
    sat = ax >= X_SAT
    ser = ax < X_SERIES
    mid = ~(sat | ser)
    out[sat] = ax[sat]
    out[ser] = h_series(x[ser], 0)
    out[mid] = x[mid] / np.tanh(x[mid])
    return out


def h1(x):
    """h'(x) = d/dx (x coth x)."""
    x = np.asarray(x, dtype=np.float64)
    ax = np.abs(x)
    out = np.empty_like(x)
    sat = ax >= X_SAT
    ser = ax < X_SERIES
    mid = ~(sat | ser)
    out[sat] = np.sign(x[sat])
    out[ser] = h_series(x[ser], 1)
    xm = x[mid]
    out[mid] = (0.5 * np.sinh(2.0 * xm) - xm) / np.sinh(xm) ** 2
    return out


def h3(x):
    """h'''(x) = 2 csch^2 x (3 coth x - 3 x coth^2 x + x)."""
    x = np.asarray(x, dtype=np.float64)
    ax = np.abs(x)
    out = np.zeros_like(x)
    ser = ax < X_SERIES
    mid = (~ser) & (ax < X_SAT)
    out[ser] = h_series(x[ser], 3)
    xm = x[mid]
    ct = 1.0 / np.tanh(xm)
    out[mid] = 2.0 / np.sinh(xm) ** 2 * (3.0 * ct - 3.0 * xm * ct * ct + xm)
    return out


class SqrtMap:
    """g(lambda) = sqrt(kappa^2 + lambda^2) (Sec. 2.5, kappa = 1 there)."""

    def __init__(self, kappa=1.0):
        self.kappa = float(kappa)

    def g_gprime(self, lam):
        lam = np.asarray(lam, dtype=np.float64)
        g = np.sqrt(self.kappa ** 2 + lam * lam)
        return g, lam / g

    def divided_differences(self, lam):
        lam = np.asarray(lam, dtype=np.float64)
        g, gp = self.g_gprime(lam)
        T = (lam[:, None] + lam[None, :]) / (g[:, None] + g[None, :])
        np.fill_diagonal(T, gp)
        return T


def g_gprime(lam, alpha):
    """g(lambda) = lambda coth(alpha lambda) and g'(lambda) (or the SqrtMap's)."""
    if isinstance(alpha, SqrtMap):
        return alpha.g_gprime(lam)
    x = alpha * np.asarray(lam, dtype=np.float64)
    return h(x) / alpha, h1(x)


def divided_differences(lam, alpha):
    if isinstance(alpha, SqrtMap):
        return alpha.divided_differences(lam)
    return _coth_divided_differences(lam, alpha)


def _coth_divided_differences(lam, alpha):
    """T_jl = (g_j - g_l)/(lam_j - lam_l), T_jj = g'(lam_j)  (Eq. d3_transform).

    Near-equal pairs (|alpha (lam_j - lam_l)| < 1e-3) use the midpoint
    expansion h'(m) + h'''(m) d^2/24; two saturated eigenvalues use the exact
    ratio (|lam_j| - |lam_l|)/(lam_j - lam_l), which is sign(lam) when the
    signs agree.
    """
    lam = np.asarray(lam, dtype=np.float64)
    x = alpha * lam
    hx = h(x)
    xj, xl = x[:, None], x[None, :]
    lj, ll = lam[:, None], lam[None, :]
    d = xj - xl
    sat = (np.abs(xj) >= X_SAT) & (np.abs(xl) >= X_SAT)
    near = (~sat) & (np.abs(d) < 1e-3)
    rest = ~(sat | near)
    T = np.zeros((lam.size, lam.size))
    with np.errstate(divide="ignore", invalid="ignore"):
        same = np.sign(xj) == np.sign(xl)
        T_sat = np.where(same, np.sign(xj) * np.ones_like(d),
                         (np.abs(lj) - np.abs(ll)) / (lj - ll))
        T_dir = (hx[:, None] - hx[None, :]) / d
    T[sat] = T_sat[sat]
    T[rest] = T_dir[rest]
    m = 0.5 * (xj + xl)[near]
    T[near] = h1(m) + h3(m) * d[near] ** 2 / 24.0
    np.fill_diagonal(T, h1(x))
    return T


def softabs_eig(H, alpha):
    """Static eigendecomposition H = Psi diag(lam) Psi' (LAPACK dsyevd via
    numpy.linalg.eigh) and the softabs spectrum g, g', log|G| = sum log g."""
    Hs = 0.5 * (H + H.T)
    lam, Psi = np.linalg.eigh(Hs)
    g, gp = g_gprime(lam, alpha)
    return {"lam": lam, "Psi": Psi, "g": g, "gp": gp, "logdetG": float(np.sum(np.log(g)))}


def metric(eig):
    """G = Psi diag(g) Psi'."""
    Psi, g = eig["Psi"], eig["g"]
    return (Psi * g) @ Psi.T


def ginv_p(eig, p):
    """G^-1 p = Psi diag(1/g) Psi' p  (= dH/dp, Eq. d_Hamiltonian)."""
    Psi, g = eig["Psi"], eig["g"]
    return Psi @ ((Psi.T @ p) / g)


def w_matrices(eig, p, alpha):
    """W1 = Psi (T o b b') Psi' with b = Psi'p / g, and W2 = Psi diag(g'/g) Psi'
    (Eq. Betancourt_formula; R o T = diag(g'/g) because R is diagonal)."""
    Psi, lam, g, gp = eig["Psi"], eig["lam"], eig["g"], eig["gp"]
    T = divided_differences(lam, alpha)
    b = (Psi.T @ p) / g
    W1 = Psi @ (T * np.outer(b, b)) @ Psi.T
    W2 = (Psi * (gp / g)) @ Psi.T
    return W1, W2, b, T
