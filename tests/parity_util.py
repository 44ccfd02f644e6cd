"""Helpers shared by the GPU parity tests: error measures and the
conditioning floor of the reference.

Errors are norm-wise: ||x - y|| / ||y|| for arrays (Frobenius for matrices),
|x - y| / max(|y|, 1) for scalars.  The floor is the disagreement of the
FP64 reference with itself when the N data points are presented in another
order (a mathematically identical problem); a GPU result is held to
max(bar, 10 x floor).
"""
import dataclasses
import json
import os
import sys

import numpy as np


def rel(x, y):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if x.ndim == 0 or x.size == 1:
        return float(abs(x.ravel()[0] - y.ravel()[0]) / max(abs(y.ravel()[0]), 1.0))
    n = np.linalg.norm(y)
    return float(np.linalg.norm(x - y) / (n if n > 0 else 1.0))


def permuted(spec, q, seed=123):
    """(spec', q', index map) with the data points in another order."""
    rng = np.random.default_rng(seed)
    if spec.n_records != spec.N:
        # two latent functions stacked record by record: permute the records
        # and keep each function's block in place
        r = rng.permutation(spec.n_records)
        p = np.concatenate([r, spec.n_records + r])
    else:
        p = rng.permutation(spec.N)
    s2 = dataclasses.replace(spec, X=spec.X[p], y=spec.y[p])
    full = np.concatenate([p, spec.N + np.arange(spec.P)])
    q2 = q[full]
    return s2, q2, full


def unpermute_vec(v2, full):
    v = np.empty_like(v2)
    v[full] = v2
    return v


def unpermute_mat(M2, full):
    M = np.empty_like(M2)
    M[np.ix_(full, full)] = M2
    return M


def record(name, **vals):
    """Print one line of measured errors (kept in the pytest log) and, when
    RMHMC_PARITY_LOG names a file, append it there as JSON."""
    items = " ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}" for k, v in vals.items())
    print(f"[parity] {name} {items}", flush=True)
    path = os.environ.get("RMHMC_PARITY_LOG")
    if path:
        clean = {k: (float(v) if isinstance(v, (float, np.floating)) else
                     int(v) if isinstance(v, (np.integer,)) else v) for k, v in vals.items()}
        with open(path, "a") as f:
            f.write(json.dumps({"case": name, **clean}) + "\n")


def progress(msg):
    """A progress line on the real stderr (long reference runs)."""
    print(f"[progress] {msg}", file=sys.__stderr__, flush=True)


def chain_floor(spec, eps, n_leapfrog, n_fixed_point, alpha, n_moves, seed, stream, ref):
    """Floor of a seeded reference chain (oracle.chain.run_seeded_chain with
    n_burnin = 0, result `ref`): the same chain with the data points in
    another order and the momentum normals permuted alike (p = G^{1/2} z is
    then the permuted momentum).  inf if the accept decisions differ."""
    from oracle import hamiltonian as oham, rng
    from oracle.chain import run_chain
    q0 = np.zeros(spec.D)
    s2, _, full = permuted(spec, q0)
    z, u = rng.chain_randoms(seed, stream, n_moves, spec.D)
    ref2 = run_chain(oham.GPTarget(s2), q0, eps, n_leapfrog, n_fixed_point, alpha, z[:, full], u)
    if not np.array_equal(ref2[2], ref[2]):
        return float("inf")
    back = np.stack([unpermute_vec(r, full) for r in ref2[0]])
    return max(rel(back, ref[0]), rel(ref2[1], ref[1]))


def _limited(args):
    """Run fn(*fargs) in a worker process with `threads` BLAS threads."""
    fn, fargs, threads = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=threads):
        return fn(*fargs)


def run_parallel(jobs, label):
    """Run [(fn, args), ...] in fresh worker processes (spawned, so nothing of
    the parent's GPU or thread state is inherited), the host cores split
    between them; prints a progress line every 20 s while they run.  fn must
    be importable (module level)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    cores = max(1, (os.cpu_count() or 2) // len(jobs))
    ctx = mp.get_context("spawn")
    with cf.ProcessPoolExecutor(len(jobs), mp_context=ctx) as ex:
        futs = [ex.submit(_limited, (fn, args, cores)) for fn, args in jobs]
        waited = 0
        while True:
            done, pending = cf.wait(futs, timeout=20)
            if not pending:
                break
            waited += 20
            progress(f"{label}: {len(pending)} reference run(s) still going after {waited} s")
        return [f.result() for f in futs]


def ref_glf(spec, q, p, eps, K, alpha, steps):
    """`steps` generalized leapfrogs of the reference from (q, p): [(q, p, H)]."""
    from oracle import hamiltonian as oham
    from oracle.integrator import glf_step
    st = oham.State(oham.GPTarget(spec), q, alpha)
    out = []
    for _ in range(steps):
        st, p = glf_step(st, p, eps, K)
        out.append((st.q.copy(), p.copy(), oham.hamiltonian(st, p)))
    return out


def ref_point(spec, q, p, alpha):
    """U, grad U, H, dH/dq, dH/dp, H(q,p) and the eigen-state of the reference."""
    from oracle import model as omodel, hamiltonian as oham
    U, g, H = omodel.hessian(spec, q)
    st = oham.State(oham.GPTarget(spec), q, alpha)
    return (U, g, H, oham.grad_q(st, p), oham.grad_p(st, p), oham.hamiltonian(st, p),
            {"Psi": st.eig["Psi"], "lam": st.eig["lam"]})


def ref_glf_basis(spec, q, p, eps, K, steps):
    """As ref_glf for the reduced-rank basis model with g = sqrt(1 + lambda^2)."""
    from oracle import basis, hamiltonian as oham, softabs
    from oracle.integrator import glf_step
    st = oham.State(basis.BasisTarget(spec), q, softabs.SqrtMap(1.0))
    out = []
    for _ in range(steps):
        st, p = glf_step(st, p, eps, K)
        out.append((st.q.copy(), p.copy(), oham.hamiltonian(st, p)))
    return out
