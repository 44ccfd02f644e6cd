"""Tempered chains for model-evidence estimation, run concurrently.

Power posteriors P_beta ∝ P(X|f)^beta · prior (appendix on model evidence):
chain k samples at beta_k = (k/(n-1))^5 with its own model dimension.  Two
engines run the chains side by side on the GPU: "graph" admits every chain
to one ``rmhmc.Batch`` (each chain's move captured into a HIP graph and
replayed on a few streams, launch shapes tuned per chain class), "pool"
submits them to the worker pool (``rmhmc.Pool``, one eager chain per worker
thread).  Each chain's output is bitwise the same as running it alone.

The thermodynamic-integration estimate ln Z ≈ sum_s (tau_s - tau_{s-1})
(E_s + E_{s-1})/2 of E_beta[ln P(X|f)] is computed on the host from the
samples (a diagnostic, not part of the sampler).
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

from . import workloads as wl


def log_likelihood(spec, samples):
    """ln P(X|f) of each sample row (Bernoulli-logit), host-side diagnostic."""
    f = samples[:, :spec.N]
    return np.sum(spec.y * f - np.logaddexp(0.0, f), axis=1)


def trapezoid_log_evidence(betas, mean_loglik):
    order = np.argsort(betas)
    b = np.asarray(betas)[order]
    e = np.asarray(mean_loglik)[order]
    return float(np.sum(np.diff(b) * 0.5 * (e[1:] + e[:-1])))


def run_tempered(n_chains=64, n_moves=20, n_leapfrog=10, n_fixed_point=6, eps=0.01,
                 alpha=1e6, n_workers=8, seed=0, dims=None, log=None, engine="graph",
                 precision=None):
    """Run the ladder; returns per-chain results and throughput.  The timed
    region is the moves themselves (set-up, tuning and capture excluded)."""
    import torch
    from . import rmhmc

    specs, drawn_dims, betas = wl.tempered_ladder(n_chains, seed)
    if dims is not None:      # one dimension for every rung (evidence sanity run)
        base, _, _ = wl.gp_logistic_2d(dims - 2, seed)
        specs = [dataclasses.replace(base, beta=float(b)) for b in betas]
        drawn_dims = np.full(n_chains, dims)
    prec = rmhmc.FP64 if precision is None else precision
    models = [rmhmc.Model(s, prec) for s in specs]
    dev = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")  # noqa
    inputs = [dev(np.zeros(s.D)) for s in specs]
    # largest chains first: they bound the makespan
    order = np.argsort(-drawn_dims, kind="stable")
    jobs = {}
    setup_s = 0.0
    if engine == "graph":
        batch = rmhmc.Batch(n_workers)
        t0 = time.perf_counter()
        for k in order:
            jobs[k] = batch.admit(models[k], inputs[k], eps, n_leapfrog, n_fixed_point, n_moves,
                                  seed=seed, stream_id=k, alpha=alpha)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        if log:
            log(f"{n_chains} chains admitted and captured in {setup_s:.2f} s")
        t0 = time.perf_counter()
        batch.step(n_moves)
        batch.sync()
        wall = time.perf_counter() - t0
        for k in order:
            batch.retire(jobs[k])
        batch.close()
    else:
        pool = rmhmc.Pool(n_workers)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in order:
            jobs[k] = pool.submit(models[k], inputs[k], eps, n_leapfrog, n_fixed_point, n_moves,
                                  seed=seed, stream_id=k, alpha=alpha)
        for k in order:
            pool.wait(jobs[k])
            if log:
                log(f"chain {k} D={specs[k].D} done")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        pool.close()
    results = []
    total_lf = 0
    for k, s in enumerate(specs):
        j = jobs[k]
        samp = j.samples.cpu().numpy()
        ll = log_likelihood(s, samp)
        total_lf += j.stats.leapfrogs
        results.append({"k": k, "beta": float(betas[k]), "D": s.D, "accepted": j.stats.accepted,
                        "failures": j.stats.failures, "fail_noconv": j.stats.fail_noconv,
                        "leapfrogs": j.stats.leapfrogs,
                        "sweeps": j.stats.sweeps, "eig_calls": j.stats.eig_calls,
                        "mean_loglik": float(ll[len(ll) // 4:].mean()),
                        "shape": getattr(j, "shape", None)})
    return {"wall_s": wall, "setup_s": setup_s, "chain_leapfrogs": total_lf,
            "chain_leapfrogs_per_s": total_lf / wall, "n_workers": n_workers, "engine": engine,
            "chains": results, "jobs": jobs, "models": models, "inputs": inputs}
