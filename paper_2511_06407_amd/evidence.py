"""Model evidence (BME) by thermodynamic integration over power posteriors,
run on the device chains (appendix "MC integration for the calculation of
BME", after Calderhead and Girolami).

Z chains each anneal through the rungs tau_1 = 1 > ... > tau_S = 0 of the
power posteriors P_tau ∝ P(X|a)^tau prior: at rung s a chain runs A moves
(Algorithm 1 with C leapfrogs each) at inverse temperature tau_s, starting
from where rung s-1 left it, and records ln P(X|a) of its final state.  The
Z chains run side by side on the worker pool.  Then
    ln BME ≈ sum_s (tau_(s-1) - tau_s) (E_(s-1) + E_s) / 2,
E_s the mean over the chains of the rung-s values, and with the rungs
treated as independent, a chain's estimate sum_s c_s l_s has variance
sum_s c_s^2 Var_s (c_s half the sum of the widths beside rung s); the
estimate from Z chains has that variance divided by Z.  (The appendix prints
(w_(s-1)^2 + w_s^2)/4 for the interior coefficients, without the cross term.)
Before the first rung each chain runs n_init moves at tau = 1 from q0.
"""
from __future__ import annotations

import time

import numpy as np


def paper_schedule():
    """The 101 rungs of the appendix's evidence runs (Sec. 2.5): steps of
    0.02 down to 0.2, 0.005 down to 0.05, 0.002 down to 0.01, 0.001 to 0."""
    t = np.concatenate([1.0 - 0.02 * np.arange(41), 0.2 - 0.005 * np.arange(1, 31),
                        0.05 - 0.002 * np.arange(1, 21), 0.01 - 0.001 * np.arange(1, 11)])
    t[-1] = 0.0
    return t


def trapezoid(tau, loglik):
    """(estimate, variance of the chain-mean estimate, per-rung means)."""
    tau = np.asarray(tau, dtype=np.float64)
    L = np.asarray(loglik, dtype=np.float64)
    E = L.mean(axis=0)
    w = tau[:-1] - tau[1:]
    est = float(np.dot(0.5 * (E[:-1] + E[1:]), w))
    Z = L.shape[0]
    c = np.concatenate([[0.0], 0.5 * w]) + np.concatenate([0.5 * w, [0.0]])
    v = L.var(axis=0, ddof=1) if Z > 1 else np.zeros(L.shape[1])
    return est, float(np.dot(c * c, v) / max(Z, 1)), E


def run_evidence(spec, n_chains=8, n_moves=5, n_leapfrog=10, n_fixed_point=6, eps=0.05,
                 alpha=1e6, n_init=20, schedule=None, seed=0, n_workers=8, log=None):
    """Thermodynamic integration on the device; returns a dict with the
    estimate, its standard error, the per-rung means and the chains' stats."""
    import torch
    from . import rmhmc

    tau = paper_schedule() if schedule is None else np.asarray(schedule, dtype=np.float64)
    models = [rmhmc.Model(spec) for _ in range(n_chains)]
    q = [torch.zeros(spec.D, dtype=torch.float64, device="cuda") for _ in range(n_chains)]
    pool = rmhmc.Pool(n_workers)
    loglik = np.zeros((n_chains, tau.size))
    accepted = np.zeros((n_chains, tau.size), dtype=np.int64)
    failures = {"all": 0, "not_pd": 0, "nonfinite": 0, "noconv": 0}
    leapfrogs = 0
    moves = 0
    t0 = time.perf_counter()

    def rung(beta, moves_per_chain, stream_base):
        nonlocal leapfrogs, moves
        jobs = []
        for z, m in enumerate(models):
            m.set_beta(beta)
            jobs.append(pool.submit(m, q[z], eps, n_leapfrog, n_fixed_point, moves_per_chain,
                                    n_burnin=0, seed=seed, stream_id=stream_base * 4096 + z, alpha=alpha))
        for z, j in enumerate(jobs):
            pool.wait(j)
            q[z] = j.samples[-1].clone()
            failures["all"] += j.stats.failures
            failures["not_pd"] += j.stats.fail_not_pd
            failures["nonfinite"] += j.stats.fail_nonfinite
            failures["noconv"] += j.stats.fail_noconv
            leapfrogs += j.stats.leapfrogs
            moves += moves_per_chain
        return jobs

    if n_init > 0:
        rung(tau[0], n_init, 0)
    for s, beta in enumerate(tau):
        jobs = rung(float(beta), n_moves, s + 1)
        for z, m in enumerate(models):
            loglik[z, s] = float(m.log_likelihood(q[z]).cpu()[0])
            accepted[z, s] = int(jobs[z].stats.accepted)
        if log and (s % 20 == 0 or s == tau.size - 1):
            log(f"rung {s + 1}/{tau.size} tau={beta:.4f} E={loglik[:, s].mean():.4f}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pool.close()
    est, var, E = trapezoid(tau, loglik)
    return {"log_evidence": est, "std_error": float(np.sqrt(var)), "tau": tau, "rung_means": E,
            "loglik": loglik, "accept_rate": float(accepted.sum() / (n_moves * accepted.size)),
            "failures": failures["all"], "failure_kinds": failures, "moves": moves,
            "leapfrogs": leapfrogs, "wall_s": wall,
            "chain_leapfrogs_per_s": leapfrogs / wall}
