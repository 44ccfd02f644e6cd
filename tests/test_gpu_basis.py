"""GPU parity of the paper's reduced-rank basis model (Sec. 2.1, Eqs. BMKL,
Solin_representation and hpar_prior; Sec. 2.3's feature-ordered contraction)
with the paper's softabs g = sqrt(kappa^2 + lambda^2), kappa = 1.

Bars: 1e-10 norm-wise relative, or 10x the reference's own floor, the
reference's disagreement with itself when the data records are presented in
another order (the parameters do not depend on the record order)."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2511_06407_amd import workloads as wl  # noqa: E402
from oracle import basis as ob, hamiltonian as oham, softabs as osoft  # noqa: E402
from oracle import rng as orng  # noqa: E402
from oracle.integrator import glf_step as oglf  # noqa: E402
from oracle.chain import momentum as omomentum, run_chain, run_seeded_chain  # noqa: E402
from tests.parity_util import rel, record, progress, run_parallel, ref_glf_basis  # noqa: E402

pytestmark = pytest.mark.gpu
BAR = 1e-10
SQRT = osoft.SqrtMap(1.0)      # kappa = 1, alpha = 1 / kappa


@pytest.fixture(scope="module")
def rm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_06407_amd import rmhmc
    return rmhmc


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def specs():
    d34, _ = wl.workload("basis_logistic_d34")
    rng = np.random.default_rng(3)
    X = np.column_stack([rng.standard_normal(60), rng.integers(0, 2, 60).astype(float),
                         rng.standard_normal(60)])
    mixed = wl.BasisSpec(X=X, y=rng.standard_normal(60),
                         kinds=(wl.BASIS_GAUSS, wl.BASIS_LINEAR, wl.BASIS_GAUSS), M=7, L=5.0,
                         bias_var=0.7, ig_alpha=(5.0, 1.0, 5.0), ig_beta=(0.5, 1.0, 0.5),
                         lik=wl.LIK_GAUSSIAN, noise_var=0.4, beta=0.6)
    return {"basis_d34": d34, "basis_mixed_d19": mixed}


SPECS = specs()


def reordered(spec, seed=123):
    p = np.random.default_rng(seed).permutation(spec.N)
    return dataclasses.replace(spec, X=spec.X[p], y=spec.y[p])


def rand_q(spec, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    q = scale * rng.standard_normal(spec.D)
    q[-3:] = rng.uniform(0.6, 1.6, 3)
    return q


@pytest.mark.parametrize("name", list(SPECS))
def test_basis_hessian_and_likelihood(rm, name):
    spec = SPECS[name]
    M = rm.BasisModel(spec)
    assert (M.N, M.P, M.D) == (spec.N, 3, spec.D)
    for seed in (0, 1):
        q = rand_q(spec, seed, 0.0 if seed == 0 else 0.4)
        if seed == 0:
            q[-3:] = 1.0        # the paper's starting point: a = 0, b = 0, theta = 1
        U, g, H = M.hessian(dev(q))
        ref = ob.derivs(spec, q)
        r2 = ob.derivs(reordered(spec), q)
        fl = max(rel(r2[0], ref[0]), rel(r2[1], ref[1]), rel(r2[2], ref[2]))
        e = (rel(host(U), ref[0]), rel(host(g), ref[1]), rel(host(H), ref[2]))
        ll = float(host(M.log_likelihood(dev(q)))[0])
        e_ll = rel(ll, ob.log_likelihood(spec, q))
        record("basis_hessian", model=name, seed=seed, U=e[0], grad=e[1], H=e[2], loglik=e_ll, floor=fl)
        tol = max(BAR, 10 * fl)
        assert max(e) < tol and e_ll < tol


@pytest.mark.parametrize("name", list(SPECS))
def test_basis_metric_grad(rm, name):
    spec = SPECS[name]
    T = ob.BasisTarget(spec)
    q = rand_q(spec, 11)
    for alpha, amap, kind in ((1.0, SQRT, rm.SOFTABS_SQRT), (1e6, 1e6, rm.SOFTABS_COTH)):
        st = oham.State(T, q, amap)
        p = omomentum(st, np.random.default_rng(12).standard_normal(spec.D))
        dq, dp, ham = rm.BasisModel(spec).metric_grad(dev(q), dev(p), dev(st.eig["Psi"].T),
                                                      dev(st.eig["lam"]), alpha, softabs=kind)
        ref = (oham.grad_q(st, p), oham.grad_p(st, p), oham.hamiltonian(st, p))
        st2 = oham.State(ob.BasisTarget(reordered(spec)), q, amap)
        fl = max(rel(oham.grad_q(st2, p), ref[0]), rel(oham.grad_p(st2, p), ref[1]),
                 rel(oham.hamiltonian(st2, p), ref[2]))
        e = (rel(host(dq), ref[0]), rel(host(dp), ref[1]), rel(host(ham), ref[2]))
        record("basis_metric_grad", model=name, alpha=alpha, dHdq=e[0], dHdp=e[1], ham=e[2], floor=fl)
        assert max(e) < max(BAR, 10 * fl)


@pytest.mark.parametrize("name", list(SPECS))
def test_basis_glf(rm, name):
    spec = SPECS[name]
    q = rand_q(spec, 21, 0.2)
    eps, K = 0.003, 6
    st = oham.State(ob.BasisTarget(spec), q, SQRT)
    p = omomentum(st, np.random.default_rng(22).standard_normal(spec.D))
    S = rm.State(rm.BasisModel(spec), dev(q), dev(p), 1.0, softabs=rm.SOFTABS_SQRT)
    st2, p2 = oham.State(ob.BasisTarget(reordered(spec)), q, SQRT), p.copy()
    ref_st, ref_p = st, p
    for step in range(3):
        S.step(eps, K)
        ref_st, ref_p = oglf(ref_st, ref_p, eps, K)
        st2, p2 = oglf(st2, p2, eps, K)
        fl = max(rel(st2.q, ref_st.q), rel(p2, ref_p))
        qg, pg, hg = S.get()
        e_q, e_p = rel(host(qg), ref_st.q), rel(host(pg), ref_p)
        e_h = rel(host(hg), oham.hamiltonian(ref_st, ref_p))
        record("basis_glf", model=name, step=step, q=e_q, p=e_p, ham=e_h, floor=fl)
        tol = max(BAR, 10 * fl)
        assert e_q < tol and e_p < tol and e_h < max(tol, 1e-12)


def test_basis_chain_d34(rm):
    """Algorithm 1 on the device for the paper's d = 34 model from the
    paper's starting point: the reference's accept decisions, samples within
    10x its floor (the same chain on the reordered records)."""
    spec = SPECS["basis_d34"]
    n_moves, C_, K, eps = 5, 10, 6, 0.003
    q0 = np.zeros(spec.D)
    q0[-3:] = 1.0
    M = rm.BasisModel(spec)
    samples, logpost, acc, stats = M.chain(dev(q0), eps, C_, K, n_moves, seed=4, stream_id=2,
                                           alpha=1.0, softabs=rm.SOFTABS_SQRT)
    ref = run_seeded_chain(ob.BasisTarget(spec), q0, eps, C_, K, SQRT, n_moves, 0, 4, 2)
    z, u = orng.chain_randoms(4, 2, n_moves, spec.D)
    ref2 = run_chain(ob.BasisTarget(reordered(spec)), q0, eps, C_, K, SQRT, z, u)
    fl = max(rel(ref2[0], ref[0]), rel(ref2[1], ref[1])) if np.array_equal(ref2[2], ref[2]) else np.inf
    bar = max(BAR, 10 * fl)
    margin = np.abs(np.log(u) - (ref[4] - ref[5]))
    gs, gl, ga = host(samples), host(logpost), host(acc)
    record("basis_chain", accepted=int(ga.sum()), ref_accepted=int(ref[2].sum()), samples=rel(gs, ref[0]),
           logpost=rel(gl, ref[1]), floor=fl, bar=bar, min_margin=float(margin.min()),
           failures=stats.failures, sweeps=stats.sweeps, eig_calls=stats.eig_calls)
    assert margin.min() > 1e-8
    assert ref[2].sum() >= 3
    assert np.array_equal(ga, ref[2])
    assert rel(gs, ref[0]) < bar and rel(gl, ref[1]) < bar
    assert stats.failures == 0


@pytest.mark.timeout(900)
def test_basis_full_size_d484(rm):
    """The paper's d = 484 model (16 covariates, N = 500): Hessian, then two
    generalized leapfrogs at the paper's step size 0.001, against the
    reference and its floor (reference runs in worker processes)."""
    spec, cfg = wl.workload("basis_logistic_d484")
    q = rand_q(spec, 31, 0.05)
    M = rm.BasisModel(spec)
    U, g, H = M.hessian(dev(q))
    got_h = (float(host(U)[0]), host(g), host(H))
    st = oham.State(ob.BasisTarget(spec), q, SQRT)
    p = omomentum(st, np.random.default_rng(32).standard_normal(spec.D))
    S = rm.State(M, dev(q), dev(p), 1.0, softabs=rm.SOFTABS_SQRT)
    got = []
    for _ in range(2):
        S.step(cfg.eps, cfg.n_fixed_point)
        qg, pg, hg = S.get()
        got.append((host(qg), host(pg), float(host(hg)[0])))
    progress("basis d = 484 on the GPU done; reference runs started")
    s2 = reordered(spec)
    ref, ref2 = run_parallel([(ref_glf_basis, (spec, q, p, cfg.eps, cfg.n_fixed_point, 2)),
                              (ref_glf_basis, (s2, q, p, cfg.eps, cfg.n_fixed_point, 2))],
                             "basis d484 glf")
    r2 = ob.derivs(s2, q)
    fl_h = max(rel(r2[0], st.U), rel(r2[1], st.grad), rel(r2[2], st.H))
    e_h = max(rel(got_h[0], st.U), rel(got_h[1], st.grad), rel(got_h[2], st.H))
    record("basis_full_hessian", D=spec.D, err=e_h, floor=fl_h)
    assert e_h < max(BAR, 10 * fl_h)
    for step in range(2):
        rq, rp, rh = ref[step]
        fl = max(rel(ref2[step][0], rq), rel(ref2[step][1], rp))
        e_q, e_p, e_hm = rel(got[step][0], rq), rel(got[step][1], rp), rel(got[step][2], rh)
        tol = max(BAR, 10 * fl)
        record("basis_glf_full", D=spec.D, step=step, q=e_q, p=e_p, ham=e_hm, floor=fl, bar=tol)
        assert e_q < tol and e_p < tol and e_hm < max(tol, 1e-12)
