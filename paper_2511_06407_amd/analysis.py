"""Chain diagnostics: effective sample size by Geyer's initial monotone
sequence estimator (Geyer 1992), used for ESS/s reporting."""
import numpy as np


def autocorr(x):
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    x = x - x.mean()
    f = np.fft.rfft(x, 2 * n)
    ac = np.fft.irfft(f * np.conj(f))[:n]
    return ac / ac[0] if ac[0] > 0 else np.zeros(n)


def ess(x):
    """ESS of a scalar chain: n / (-1 + 2 sum_k Gamma_k) with Gamma_k the
    sums of adjacent autocorrelation pairs, truncated at the first
    non-positive pair and made monotone."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    if np.var(x) == 0.0:
        return 0.0          # a chain that never moved carries no information
    if n < 4:
        return float(n)
    rho = autocorr(x)
    pairs = rho[: (n // 2) * 2].reshape(-1, 2).sum(axis=1)
    s = 0.0
    prev = np.inf
    for g in pairs:
        if g <= 0:
            break
        g = min(g, prev)
        s += g
        prev = g
    tau = -1.0 + 2.0 * s
    return float(n / max(tau, 1e-12))


def ess_summary(samples, logpost):
    """min / median ESS over coordinates and ESS of the log posterior."""
    per = np.array([ess(samples[:, i]) for i in range(samples.shape[1])])
    return {"min": float(per.min()), "median": float(np.median(per)), "logpost": ess(logpost)}
