"""Model evidence by thermodynamic integration over power posteriors, and a
quadrature reference for Gaussian-likelihood GP models.  FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper anchor: appendix "MC integration for the calculation of BME", after
Calderhead and Girolami.  The power posteriors P_tau ∝ P(X|a)^tau prior
interpolate prior (tau = 0) and posterior (tau = 1), and
    ln BME = integral_0^1 E_{P_tau}[ln P(X|a)] dtau
(the appendix writes BME on the left; the right-hand side is its logarithm).
The integral is taken by the trapezoid rule over rungs tau_1 = 1 > ... >
tau_S = 0, with E estimated by the mean of ln P(X|a) over Z chains at each
rung, and the variance of the estimate from the per-rung variances over the
chains, treating the rungs as independent.
"""
from __future__ import annotations

import math

import numpy as np

from . import model


def paper_schedule():
    """The 101 rungs of the appendix's evidence runs (Sec. 2.5):
    1 - 0.02 (s-1) for s <= 41, 0.2 - 0.005 (s-41) for 41 < s <= 71,
    0.05 - 0.002 (s-71) for 71 < s <= 91, 0.01 - 0.001 (s-91) for s > 91."""
    tau = []
    for s in range(1, 102):
        if s <= 41:
            t = 1.0 - 0.02 * (s - 1)
        elif s <= 71:
            t = 0.2 - 0.005 * (s - 41)
        elif s <= 91:
            t = 0.05 - 0.002 * (s - 71)
        else:
            t = 0.01 - 0.001 * (s - 91)
        tau.append(t)
    return np.array(tau)


def ti_estimate(tau, loglik):
    """Trapezoid estimate of ln BME and its variance.

    tau: S rungs (tau_1 = 1, tau_S = 0, decreasing); loglik: Z x S values of
    ln P(X|a) of chain z at rung s.  Returns (estimate, variance of one
    chain's estimate, per-rung means E_s).  The estimate integrates the
    per-rung means over the chains.  With the rungs independent, a chain's
    estimate sum_s c_s l_s (c_1 = w_1/2, c_s = (w_(s-1) + w_s)/2, c_S =
    w_(S-1)/2, w the rung widths) has variance sum_s c_s^2 Var_s, Var_s the
    sample variance over the chains at rung s; the appendix prints
    (w_(s-1)^2 + w_s^2)/4 for the interior coefficients, which drops the
    cross term and halves the variance on an even grid.  The variance of the
    chain mean is this divided by Z."""
    tau = np.asarray(tau, dtype=np.float64)
    L = np.asarray(loglik, dtype=np.float64)
    E = L.mean(axis=0)
    w = tau[:-1] - tau[1:]                      # positive widths of the decreasing schedule
    est = float(np.sum(0.5 * (E[1:] + E[:-1]) * w))
    Z = L.shape[0]
    var_s = L.var(axis=0, ddof=1) if Z > 1 else np.zeros(L.shape[1])
    c = np.zeros(tau.size)
    c[:-1] += 0.5 * w
    c[1:] += 0.5 * w
    return est, float(np.sum(c * c * var_s)), E


def gaussian_log_evidence(spec, n_nodes=160, half_width=9.0):
    """ln p(y) for a Gaussian-likelihood latent-GP model with eta ~ N(0, I):
    f integrates out in closed form, p(y | eta) = N(y; 0, K(eta) + s2 I), and
    the remaining integral of p(y | eta) N(eta; 0, I) over eta is taken by a
    tensor Gauss-Legendre rule on [-half_width, half_width]^P (the prior mass
    outside is below 1e-18 for the default)."""
    if spec.lik != model.LIK_GAUSSIAN:
        raise ValueError("closed form only for the Gaussian likelihood")
    P, N, y = spec.P, spec.N, spec.y
    x, w = np.polynomial.legendre.leggauss(n_nodes)
    x, w = half_width * x, half_width * w
    logs, logw = [], []
    for idx in np.ndindex(*([n_nodes] * P)):
        eta = x[list(idx)]
        C = model.gram(spec, eta) + spec.noise_var * np.eye(N)
        _, logdet = np.linalg.slogdet(C)
        logs.append(-0.5 * (y @ np.linalg.solve(C, y) + logdet + N * math.log(2.0 * math.pi))
                    - 0.5 * eta @ eta - 0.5 * P * math.log(2.0 * math.pi))
        logw.append(float(np.sum(np.log(w[list(idx)]))))
    a = np.array(logs) + np.array(logw)
    m = a.max()
    return float(m + math.log(np.sum(np.exp(a - m))))


def _eta_nodes(P, n_nodes, half_width):
    x, w = np.polynomial.legendre.leggauss(n_nodes)
    x, w = half_width * x, half_width * w
    for idx in np.ndindex(*([n_nodes] * P)):
        eta = x[list(idx)]
        yield eta, float(np.sum(np.log(w[list(idx)]))) - 0.5 * eta @ eta - 0.5 * P * math.log(2.0 * math.pi)


def gaussian_power_posterior(spec, tau, n_nodes=160, half_width=9.0):
    """For a Gaussian-likelihood latent-GP model (f ~ N(0, K(eta)), eta ~
    N(0, I), y | f ~ N(f, s2 I)), the log normaliser ln Z(tau) of the power
    posterior p(y | f)^tau p(f | eta) p(eta) and the exact rung mean
    E(tau) = E_tau[ln p(y | f)] = d ln Z / d tau.  Returns (ln Z, E).

    Given eta the tempered likelihood is Gaussian in f: p(y | f)^tau =
    (2 pi s2)^(-N tau / 2) (2 pi s2 / tau)^(N / 2) N(y; f, (s2 / tau) I), so
    Z_eta(tau) follows from N(y; 0, K + (s2 / tau) I), and f | eta has mean
    m = K (K + (s2 / tau) I)^-1 y and covariance K - K (K + (s2 / tau) I)^-1 K,
    whence E_eta(tau) = -N ln(2 pi s2) / 2 - (|y - m|^2 + tr Cov) / (2 s2).
    At tau = 0, Z_eta = 1, m = 0 and Cov = K.  eta is integrated by the
    same tensor Gauss-Legendre rule as gaussian_log_evidence, E_eta weighted
    by the posterior mass of each node."""
    if spec.lik != model.LIK_GAUSSIAN:
        raise ValueError("closed form only for the Gaussian likelihood")
    N, y, s2 = spec.N, spec.y, spec.noise_var
    c0 = -0.5 * N * math.log(2.0 * math.pi * s2)
    logz, e = [], []
    for eta, lw in _eta_nodes(spec.P, n_nodes, half_width):
        K = model.gram(spec, eta)
        if tau > 0.0:
            C = K + (s2 / tau) * np.eye(N)
            _, logdet = np.linalg.slogdet(C)
            sol = np.linalg.solve(C, y)
            lz = (tau * c0 + 0.5 * N * math.log(2.0 * math.pi * s2 / tau)
                  - 0.5 * (y @ sol + logdet + N * math.log(2.0 * math.pi)))
            m = K @ sol
            cov_tr = np.trace(K) - np.trace(K @ np.linalg.solve(C, K))
        else:
            lz, m, cov_tr = 0.0, np.zeros(N), np.trace(K)
        logz.append(lz + lw)
        e.append(c0 - 0.5 * (np.sum((y - m) ** 2) + cov_tr) / s2)
    a = np.array(logz)
    mx = a.max()
    wts = np.exp(a - mx)
    return float(mx + math.log(wts.sum())), float(np.dot(wts, e) / wts.sum())


def gaussian_rung_means(spec, tau, n_nodes=60, half_width=9.0):
    """The exact E(tau_s) of gaussian_power_posterior at every rung."""
    return np.array([gaussian_power_posterior(spec, float(t), n_nodes, half_width)[1] for t in tau])
