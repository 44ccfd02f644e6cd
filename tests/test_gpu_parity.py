"""GPU parity: every C-ABI entry point against the FP64 reference.

Bar (FP64 path): 1e-10 relative, norm-wise, or 10x the reference's own
conditioning floor where the problem is ill conditioned (jitter 1e-6
kernel matrices).  Eigenvectors are compared only through basis-invariant
quantities (G, log|G|, G^-1 p, spectra, dH/dq), never directly.
"""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2511_06407_amd import workloads as wl  # noqa: E402
from oracle import model as omodel, softabs as osoft, hamiltonian as oham, rng as orng  # noqa: E402
from oracle.integrator import glf_step as oglf  # noqa: E402
from oracle.chain import run_seeded_chain, momentum as omomentum  # noqa: E402
from tests.parity_util import (rel, permuted, unpermute_mat, unpermute_vec, record,  # noqa: E402
                               chain_floor, progress, run_parallel, ref_glf)

pytestmark = pytest.mark.gpu
BAR = 1e-10


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


def models():
    c1, _ = wl.workload("gp_logistic_d34")
    ard, _, _ = wl.gp_logistic_ard4(70, seed=1)
    mkl, _, _ = wl.propensity_mkl(90, seed=2)
    gau, _, _ = wl.gaussian_gp(40, noise_var=0.2, seed=3)
    return {
        "c1_d34": c1,
        "ard_d75_wellcond": dataclasses.replace(ard, jitter=1e-2),
        "mkl_d104_wellcond": dataclasses.replace(mkl, jitter=1e-2, beta=0.6),
        "gauss_d42": dataclasses.replace(gau, jitter=1e-3),
        "mkl_d104": mkl,
    }


MODELS = models()


def rand_q(spec, seed, scale=0.4):
    rng = np.random.default_rng(seed)
    q = scale * rng.standard_normal(spec.D)
    return q


# ---------------------------------------------------------------- GEMM
@pytest.mark.parametrize("dtype", ["f64", "f32"])
# (2050, 4100, 21): a large product, ragged in every dimension; (250, 120, 70):
# a 4 x 2 tile grid, which takes the XCD-aware tile order, ragged in m and n
@pytest.mark.parametrize("shape", [(64, 64, 64), (70, 45, 33), (1, 130, 17), (257, 3, 300), (128, 96, 1),
                                   (2050, 4100, 21), (250, 120, 70)])
@pytest.mark.parametrize("tA,tB", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_gemm(rm, dtype, shape, tA, tB):
    m, n, k = shape
    rng = np.random.default_rng(m * 7 + n * 13 + k)
    # column-major storage: a torch tensor of shape (cols, ld) holds an ld x cols matrix
    ra, ca = (k, m) if tA else (m, k)
    rb, cb = (n, k) if tB else (k, n)
    lda, ldb, ldc = ra + 3, rb + 1, m + 2
    A = rng.standard_normal((ca, lda))
    B = rng.standard_normal((cb, ldb))
    Cm = rng.standard_normal((n, ldc))
    Am = A[:, :ra].T
    Bm = B[:, :rb].T
    opA = Am.T if tA else Am
    opB = Bm.T if tB else Bm
    want = 0.7 * opA @ opB + (-0.3) * Cm[:, :m].T
    tdt = torch.float64 if dtype == "f64" else torch.float32
    At = torch.tensor(A, dtype=tdt, device="cuda")
    Bt = torch.tensor(B, dtype=tdt, device="cuda")
    Ct = torch.tensor(Cm, dtype=tdt, device="cuda")
    rm.gemm_colmajor(m, n, k, At, lda, tA, Bt, ldb, tB, Ct, ldc, alpha=0.7, beta=-0.3)
    got = host(Ct)[:, :m].T
    tol = 1e-13 if dtype == "f64" else 2e-5
    err = rel(got, want)
    record("gemm", dtype=dtype, shape=str(shape), tA=tA, tB=tB, err=err)
    assert err < tol
    # padding rows of C untouched
    assert np.array_equal(host(Ct)[:, m:], Cm[:, m:].astype(np.float32 if dtype == "f32" else np.float64))


# Split-K single products: (1088, 1088, 1088) is the eigen warm-start shape
# (17 x 17 tiles, 4 layers of 272); (130, 77, 301) is ragged in every
# dimension with a short last layer; (64, 40, 100) has k below 32 * splits and
# takes the unsplit kernel.
@pytest.mark.parametrize("shape,splits", [((1088, 1088, 1088), 4), ((130, 77, 301), 3),
                                          ((64, 40, 100), 4), ((33, 65, 500), 1)])
@pytest.mark.parametrize("tA,tB", [(0, 0), (1, 0), (0, 1)])
def test_gemm_splitk(rm, shape, splits, tA, tB):
    m, n, k = shape
    rng = np.random.default_rng(m * 5 + n * 11 + k + splits)
    ra, ca = (k, m) if tA else (m, k)
    rb, cb = (n, k) if tB else (k, n)
    lda, ldb, ldc = ra + 2, rb + 3, m + 1
    A = rng.standard_normal((ca, lda))
    B = rng.standard_normal((cb, ldb))
    Cm = rng.standard_normal((n, ldc))
    opA = A[:, :ra] if tA else A[:, :ra].T
    opB = B[:, :rb] if tB else B[:, :rb].T
    want = opA @ opB
    At = torch.tensor(A, dtype=torch.float64, device="cuda")
    Bt = torch.tensor(B, dtype=torch.float64, device="cuda")
    Ct = torch.tensor(Cm, dtype=torch.float64, device="cuda")
    work = torch.full((splits * m * n,), np.nan, dtype=torch.float64, device="cuda")
    rm.gemm_splitk_colmajor(m, n, k, At, lda, tA, Bt, ldb, tB, Ct, ldc, work, splits)
    got = host(Ct)[:, :m].T
    err = rel(got, want)
    record("gemm_splitk", shape=str(shape), splits=splits, tA=tA, tB=tB, err=err)
    assert err < 1e-13
    # padding rows of C untouched
    assert np.array_equal(host(Ct)[:, m:], Cm[:, m:])


# Tall-k products C = A' B (the trace form): (14, 56) and (14, 14) are the
# trace shapes at P = 14 (four and one 16-column tiles), (16, 17) two tiles;
# odd k leaves a last step shorter than 16 in the last chunk; (20, 30) has
# more than 16 rows and an odd leading dimension takes the tiled kernel.
@pytest.mark.parametrize("m,n,k,pad,splits", [(14, 56, 40007, 0, 64), (14, 14, 65536, 0, 512),
                                              (16, 17, 3003, 4, 7), (5, 64, 999, 0, 3),
                                              (20, 30, 5000, 0, 16), (14, 20, 4001, 1, 8)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gemm_tallk(rm, m, n, k, pad, splits, dtype):
    rng = np.random.default_rng(m * 7 + n * 13 + k + pad)
    ld = k + pad
    A = rng.standard_normal((m, ld))
    B = rng.standard_normal((n, ld))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        A, B = A.astype(np.float32).astype(np.float64), B.astype(np.float32).astype(np.float64)
    want = A[:, :k] @ B[:, :k].T
    At = torch.tensor(A, dtype=tdt, device="cuda")
    Bt = torch.tensor(B, dtype=tdt, device="cuda")
    Ct = torch.full((n, m + 2), np.nan, dtype=torch.float64, device="cuda")
    work = torch.full((splits * m * n,), np.nan, dtype=tdt, device="cuda")
    rm.gemm_tallk(m, n, k, At, ld, Bt, ld, Ct, m + 2, work, splits)
    got = host(Ct)[:, :m].T
    err = rel(got, want)
    record("gemm_tallk", m=m, n=n, k=k, pad=pad, splits=splits, dtype=dtype, err=err)
    # FP32: products rounded to FP32 and summed in FP32 within 16-long steps
    # and chunks of at most k / splits terms
    assert err < (1e-13 if dtype == "f64" else 1e-5)
    assert np.all(np.isnan(host(Ct)[:, m:]))


# ---------------------------------------------------------------- Hessian
def floor_hessian(spec, q, ref):
    s2, q2, full = permuted(spec, q)
    U2, g2, H2 = omodel.hessian(s2, q2)
    return max(rel(U2, ref[0]), rel(unpermute_vec(g2, full), ref[1]),
               rel(unpermute_mat(H2, full), ref[2]))


@pytest.mark.parametrize("name", list(MODELS))
def test_hessian_parity(rm, name):
    spec = MODELS[name]
    M = rm.Model(spec)
    for seed in (0, 1):
        q = np.zeros(spec.D) if seed == 0 else rand_q(spec, seed)
        U, g, H = M.hessian(dev(q))
        ref = omodel.hessian(spec, q)
        fl = floor_hessian(spec, q, ref)
        eU, eg, eH = rel(host(U), ref[0]), rel(host(g), ref[1]), rel(host(H), ref[2])
        record("hessian", model=name, seed=seed, U=eU, grad=eg, H=eH, floor=fl)
        tol = max(BAR, 10 * fl)
        assert eU < tol and eg < tol and eH < tol


# ---------------------------------------------------------------- softabs eig
def invariants(Q_rows, lam, g, alpha, p):
    """G, log|G|, G^-1 p from eigenvectors given as rows."""
    Psi = Q_rows.T
    G = (Psi * g) @ Psi.T
    ginvp = Psi @ ((Psi.T @ p) / g)
    return G, float(np.sum(np.log(g))), ginvp


def cluster_matrix(D, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((D, D)))
    lam = rng.standard_normal(D) * 5
    lam[: D // 3] = 1e6 + 1e-3 * rng.standard_normal(D // 3)   # tight cluster, like K^-1 at 1/jitter
    lam[D // 3] = 3e-7                                          # near-zero: the coth branch
    lam[D // 3 + 1] = -2e-6
    return (Q * lam) @ Q.T


@pytest.mark.parametrize("case", ["c1_hessian", "cluster_130", "cluster_300", "rand_64"])
def test_softabs_eig_static(rm, case):
    alpha = 1e6
    if case == "c1_hessian":
        spec = MODELS["c1_d34"]
        H = omodel.hessian(spec, rand_q(spec, 5))[2]
    elif case == "rand_64":
        rng = np.random.default_rng(9)
        H = rng.standard_normal((64, 64))
        H = H + H.T
    else:
        H = cluster_matrix(int(case.split("_")[1]), 4)
    H = 0.5 * (H + H.T)
    check_static_eig(rm, case, H, alpha)


def check_static_eig(rm, case, H, alpha, Q_warm=None, sqrt_map=False):
    """Solve H with the GPU eigensolver (cold, or warm-started from the rows
    of Q_warm) and hold the result to the bars below against the reference
    eigendecomposition; returns the sweep count.  With sqrt_map the softabs
    map is g = sqrt(kappa^2 + lambda^2), kappa = 1/alpha."""
    D = H.shape[0]
    kind = rm.SOFTABS_SQRT if sqrt_map else rm.SOFTABS_COTH
    Qt, lam, g, gp, ld, sweeps = rm.softabs_eig(dev(H), alpha, Q_warm=Q_warm, softabs=kind)
    if sqrt_map:
        alpha = osoft.SqrtMap(1.0 / alpha)
    Q = host(Qt)
    lam, g, gp, ld = host(lam), host(g), host(gp), float(host(ld)[0])
    ref = osoft.softabs_eig(H, alpha)
    p = np.random.default_rng(1).standard_normal(D)
    G, ldg, gip = invariants(Q, lam, g, alpha, p)
    Gr = osoft.metric(ref)
    e_lam = rel(np.sort(lam), ref["lam"])
    e_G = rel(G, Gr)
    e_ld = rel(ld, ref["logdetG"])
    e_gip = rel(gip, osoft.ginv_p(ref, p))
    orth = float(np.linalg.norm(Q @ Q.T - np.eye(D)))
    resid = float(np.linalg.norm(H @ Q.T - Q.T * lam) / np.linalg.norm(H))
    g_ref, gp_ref = osoft.g_gprime(lam, alpha)
    e_g = rel(g, g_ref)
    e_gp = rel(gp, gp_ref)
    # floor: the reference on a permuted copy of the same matrix
    perm = np.random.default_rng(7).permutation(D)
    ref2 = osoft.softabs_eig(H[np.ix_(perm, perm)], alpha)
    Psi2 = np.empty_like(ref2["Psi"])
    Psi2[perm] = ref2["Psi"]
    ref2 = dict(ref2, Psi=Psi2)
    fl_ld = rel(ref2["logdetG"], ref["logdetG"])
    fl_gip = rel(osoft.ginv_p(ref2, p), osoft.ginv_p(ref, p))
    fl_G = rel(osoft.metric(ref2), Gr)
    record("eig_sqrt" if sqrt_map else "eig_static", case=case, sweeps=sweeps, lam=e_lam, G=e_G, logdetG=e_ld, Ginvp=e_gip,
           orth=orth, resid=resid, g=e_g, gp=e_gp, floor_logdetG=fl_ld, floor_Ginvp=fl_gip)
    assert e_g < 1e-14 and e_gp < 1e-14
    # backward error at working accuracy: orthogonality and residual ~ sqrt(D) u
    assert orth < 1e-11 and resid < 1e-12
    assert e_lam < BAR and e_G < max(BAR, 10 * fl_G)
    # log|G| = sum_i log g(lambda_i).  Each computed eigenvalue lies within its
    # residual norm ||H psi_i - lambda_i psi_i|| of a true one, so to first
    # order |log|G|_gpu - log|G|_ref| <= sum_i |g'/g|(lambda_i) (r_i,gpu + r_i,ref).
    # Eigenvalues near 1/alpha carry |g'/g| ~ alpha and residuals ~ u ||H||.
    order = np.argsort(lam)
    r_gpu = np.linalg.norm(H @ Q.T - Q.T * lam, axis=0)[order]
    r_ref = np.linalg.norm(H @ ref["Psi"] - ref["Psi"] * ref["lam"], axis=0)
    gr, gpr = osoft.g_gprime(ref["lam"], alpha)
    bound_ld = float(np.sum(np.abs(gpr / gr) * (r_gpu + r_ref)))
    e_ld_abs = abs(ld - ref["logdetG"])
    record("eig_static_logdet", case=case, abs_err=e_ld_abs, bound=bound_ld)
    assert e_ld < BAR or e_ld_abs <= bound_ld
    # G^-1 p also depends on the eigenvectors of those eigenvalues, which no
    # backward-stable solver fixes better than ||H|| u / gap: bar against the
    # reference's own spread under a permutation of the indices
    assert e_gip < max(BAR, 10 * fl_gip)
    return sweeps, Qt


def test_full_size_softabs_eig(rm):
    """The eigensolver on the benchmarked Hessian (D = 1038: N = 1024, P = 14,
    jitter 1e-6, so K^-1 puts a cluster of eigenvalues near 1e6): a cold
    solve, then a warm start at a point one step-size away (Sec. 2.4), both
    held to the bars of the static cases; the warm start needs fewer sweeps."""
    spec, cfg = wl.workload("propensity_mkl_d1038")
    q0 = rand_q(spec, 31, 0.1)
    q1 = q0 + cfg.eps * np.random.default_rng(33).standard_normal(spec.D)
    H0 = omodel.hessian(spec, q0)[2]
    s_static, Q0 = check_static_eig(rm, "full_d1038_cold", 0.5 * (H0 + H0.T), cfg.alpha)
    H1 = omodel.hessian(spec, q1)[2]
    s_dyn, _ = check_static_eig(rm, "full_d1038_warm", 0.5 * (H1 + H1.T), cfg.alpha, Q_warm=Q0)
    record("full_eig_sweeps", static=s_static, dynamic=s_dyn)
    assert s_dyn < s_static


def test_softabs_eig_dynamic(rm):
    """Warm start from the eigenvectors at a nearby point (Sec. 2.4): same
    invariants, fewer sweeps than the static solve."""
    spec = MODELS["ard_d75_wellcond"]
    q0 = rand_q(spec, 3)
    q1 = q0 + 0.01 * np.random.default_rng(4).standard_normal(spec.D)
    H0 = omodel.hessian(spec, q0)[2]
    H1 = omodel.hessian(spec, q1)[2]
    alpha = 1e6
    Q0, _, _, _, _, s_static0 = rm.softabs_eig(dev(H0), alpha)
    _, _, _, _, _, s_static1 = rm.softabs_eig(dev(H1), alpha)
    Qt, lam, g, gp, ld, s_dyn = rm.softabs_eig(dev(H1), alpha, Q_warm=Q0)
    Q, lam, g = host(Qt), host(lam), host(g)
    ref = osoft.softabs_eig(H1, alpha)
    p = np.random.default_rng(1).standard_normal(spec.D)
    G, ldg, gip = invariants(Q, lam, g, alpha, p)
    e_G = rel(G, osoft.metric(ref))
    e_ld = rel(float(host(ld)[0]), ref["logdetG"])
    record("eig_dynamic", static_sweeps=s_static1, dynamic_sweeps=s_dyn, G=e_G, logdetG=e_ld)
    assert e_G < BAR and e_ld < BAR
    assert s_dyn < s_static1


# ---------------------------------------------------------------- metric grad
@pytest.mark.parametrize("name", ["c1_d34", "ard_d75_wellcond", "mkl_d104_wellcond", "gauss_d42"])
def test_metric_grad_parity(rm, name):
    spec = MODELS[name]
    T = oham.GPTarget(spec)
    q = rand_q(spec, 11, 0.3)
    for alpha in (1e6, 2.0):
        st = oham.State(T, q, alpha)
        p = omomentum(st, np.random.default_rng(12).standard_normal(spec.D))
        Qt = dev(st.eig["Psi"].T)          # rows = eigenvectors = column-major Psi
        dq, dp, ham = rm.Model(spec).metric_grad(dev(q), dev(p), Qt, dev(st.eig["lam"]), alpha)
        ref_dq = oham.grad_q(st, p)
        ref_dp = oham.grad_p(st, p)
        ref_h = oham.hamiltonian(st, p)
        # floor: the reference on the same problem with the data reordered
        s2, q2, full = permuted(spec, q)
        st2 = oham.State(oham.GPTarget(s2), q2, alpha)
        fl = max(rel(unpermute_vec(oham.grad_q(st2, p[full]), full), ref_dq),
                 rel(unpermute_vec(oham.grad_p(st2, p[full]), full), ref_dp),
                 rel(oham.hamiltonian(st2, p[full]), ref_h))
        e_dq, e_dp, e_h = rel(host(dq), ref_dq), rel(host(dp), ref_dp), rel(host(ham), ref_h)
        record("metric_grad", model=name, alpha=alpha, dHdq=e_dq, dHdp=e_dp, ham=e_h, floor=fl)
        tol = max(BAR, 10 * fl)
        assert e_dq < tol and e_dp < tol and e_h < tol


def test_full_size_hessian_and_metric_grad(rm):
    """The benchmarked workload itself (D = 1038: N = 1024, P = 14, jitter
    1e-6): U, grad U and H, then dH/dq, dH/dp and the Hamiltonian for the
    reference eigen-state, against the reference and its own floor (the
    reference with the data points reordered)."""
    spec, cfg = wl.workload("propensity_mkl_d1038")
    q = rand_q(spec, 31, 0.1)
    M = rm.Model(spec)
    U, g, H = M.hessian(dev(q))
    ref = omodel.hessian(spec, q)
    fl_h = floor_hessian(spec, q, ref)
    eU, eg, eH = rel(host(U), ref[0]), rel(host(g), ref[1]), rel(host(H), ref[2])
    record("full_hessian", D=spec.D, U=eU, grad=eg, H=eH, floor=fl_h)
    tol = max(BAR, 10 * fl_h)
    assert eU < tol and eg < tol and eH < tol
    st = oham.State(oham.GPTarget(spec), q, cfg.alpha)
    p = omomentum(st, np.random.default_rng(32).standard_normal(spec.D))
    dq, dp, ham = M.metric_grad(dev(q), dev(p), dev(st.eig["Psi"].T), dev(st.eig["lam"]), cfg.alpha)
    ref_dq, ref_dp, ref_h = oham.grad_q(st, p), oham.grad_p(st, p), oham.hamiltonian(st, p)
    s2, q2, full = permuted(spec, q)
    st2 = oham.State(oham.GPTarget(s2), q2, cfg.alpha)
    fl = max(rel(unpermute_vec(oham.grad_q(st2, p[full]), full), ref_dq),
             rel(unpermute_vec(oham.grad_p(st2, p[full]), full), ref_dp),
             rel(oham.hamiltonian(st2, p[full]), ref_h))
    e_dq, e_dp, e_h = rel(host(dq), ref_dq), rel(host(dp), ref_dp), rel(host(ham), ref_h)
    record("full_metric_grad", D=spec.D, dHdq=e_dq, dHdp=e_dp, ham=e_h, floor=fl)
    tol = max(BAR, 10 * fl)
    assert e_dq < tol and e_dp < tol and e_h < tol


def test_metric_grad_two_parameter_se_n1000(rm):
    """GP-logistic with an isotropic SE kernel (P = 2) at N = 1000, the
    largest size of the serving mix: three second-derivative pairs against
    two weights, so the tall-K contraction of the pairs writes more split
    partials (splits x 3 x 2) than the P x P and P x n_Y trace products
    (splits x 2 x 2).  dH/dq, dH/dp and H against the reference."""
    spec, _, _ = wl.gp_logistic_2d(1000, seed=7)
    q = rand_q(spec, 41, 0.1)
    alpha = 1e6
    st = oham.State(oham.GPTarget(spec), q, alpha)
    p = omomentum(st, np.random.default_rng(42).standard_normal(spec.D))
    M = rm.Model(spec)
    dq, dp, ham = M.metric_grad(dev(q), dev(p), dev(st.eig["Psi"].T), dev(st.eig["lam"]), alpha)
    ref_dq, ref_dp, ref_h = oham.grad_q(st, p), oham.grad_p(st, p), oham.hamiltonian(st, p)
    s2, q2, full = permuted(spec, q)
    st2 = oham.State(oham.GPTarget(s2), q2, alpha)
    fl = max(rel(unpermute_vec(oham.grad_q(st2, p[full]), full), ref_dq),
             rel(unpermute_vec(oham.grad_p(st2, p[full]), full), ref_dp),
             rel(oham.hamiltonian(st2, p[full]), ref_h))
    e_dq, e_dp, e_h = rel(host(dq), ref_dq), rel(host(dp), ref_dp), rel(host(ham), ref_h)
    record("metric_grad", model="gp_logistic_n1000", alpha=alpha, dHdq=e_dq, dHdp=e_dp, ham=e_h,
           floor=fl)
    tol = max(BAR, 10 * fl)
    assert e_dq < tol and e_dp < tol and e_h < tol


# ---------------------------------------------------------------- leapfrog
@pytest.mark.parametrize("name,eps", [("c1_d34", 0.01), ("mkl_d104_wellcond", 0.003),
                                      ("ard_d75_wellcond", 0.01)])
def test_glf_step_parity(rm, name, eps):
    spec = MODELS[name]
    T = oham.GPTarget(spec)
    q = rand_q(spec, 21, 0.2)
    alpha, K = 1e6, 6
    st = oham.State(T, q, alpha)
    p = omomentum(st, np.random.default_rng(22).standard_normal(spec.D))
    S = rm.State(rm.Model(spec), dev(q), dev(p), alpha)
    ref_st, ref_p = st, p
    s2, q2, full = permuted(spec, q)
    st2, p2 = oham.State(oham.GPTarget(s2), q2, alpha), p[full]
    for step in range(2):
        S.step(eps, K)
        ref_st, ref_p = oglf(ref_st, ref_p, eps, K)
        st2, p2 = oglf(st2, p2, eps, K)
        fl = max(rel(unpermute_vec(st2.q, full), ref_st.q), rel(unpermute_vec(p2, full), ref_p))
        qg, pg, hg = S.get()
        e_q, e_p = rel(host(qg), ref_st.q), rel(host(pg), ref_p)
        e_h = rel(host(hg), oham.hamiltonian(ref_st, ref_p))
        record("glf_step", model=name, step=step, q=e_q, p=e_p, ham=e_h, floor=fl)
        tol = max(BAR, 10 * fl)
        assert e_q < tol and e_p < tol and e_h < max(tol, 1e-12)


@pytest.mark.timeout(1500)
def test_glf_step_parity_full_size(rm):
    """Two generalized leapfrogs of the benchmarked workload itself (D = 1038:
    N = 1024, P = 14, jitter 1e-6) at its step size, against the reference
    and its permutation floor (the two reference runs go to two processes)."""
    spec, cfg = wl.workload("propensity_mkl_d1038")
    q = rand_q(spec, 41, 0.05)
    alpha, K, eps = cfg.alpha, cfg.n_fixed_point, cfg.eps
    st = oham.State(oham.GPTarget(spec), q, alpha)
    p = omomentum(st, np.random.default_rng(42).standard_normal(spec.D))
    S = rm.State(rm.Model(spec), dev(q), dev(p), alpha)
    got = []
    for _ in range(2):
        S.step(eps, K)
        qg, pg, hg = S.get()
        got.append((host(qg), host(pg), float(host(hg)[0])))
    progress("full-size leapfrogs on the GPU done; reference runs started")
    s2, q2, full = permuted(spec, q)
    ref, ref2 = run_parallel([(ref_glf, (spec, q, p, eps, K, alpha, 2)),
                              (ref_glf, (s2, q2, p[full], eps, K, alpha, 2))], "full-size glf")
    for step in range(2):
        rq, rp, rh = ref[step]
        q2s, p2s, _ = ref2[step]
        fl = max(rel(unpermute_vec(q2s, full), rq), rel(unpermute_vec(p2s, full), rp))
        e_q, e_p, e_h = rel(got[step][0], rq), rel(got[step][1], rp), rel(got[step][2], rh)
        tol = max(BAR, 10 * fl)
        record("glf_step_full", D=spec.D, step=step, q=e_q, p=e_p, ham=e_h, floor=fl, bar=tol)
        assert e_q < tol and e_p < tol and e_h < max(tol, 1e-12)


# ---------------------------------------------------------------- chain
def test_chain_randoms_match_reference(rm):
    """The device Philox4x64-10 stream: uniforms bit for bit, normals to the
    last place (the two sides' log/sqrt/sin/cos)."""
    for seed, stream, move, D in ((0, 0, 0, 34), (7, 3, 5, 1038), (2 ** 63 + 5, 2 ** 40, 123, 9)):
        z, u = rm.chain_randoms(D, seed, stream, move)
        zr = orng.momentum_normals(seed, stream, move, D)
        ur = orng.mh_uniform(seed, stream, move)
        ez = float(np.max(np.abs(host(z) - zr)))
        record("chain_randoms", seed=seed, stream=stream, move=move, D=D, z_maxabs=ez)
        assert float(host(u)[0]) == ur
        assert ez < 1e-14


def test_chain_parity_c1(rm):
    """Algorithm 1 on the device against the reference, same (seed, stream):
    identical accept decisions, samples within 10 x the reference's own
    permutation floor; burn-in moves are not returned."""
    spec, cfg = wl.workload("gp_logistic_d34")
    T = oham.GPTarget(spec)
    n_moves, n_burnin, C_, K = 5, 1, 3, cfg.n_fixed_point
    q0 = np.zeros(spec.D)
    M = rm.Model(spec)
    samples, logpost, acc, stats = M.chain(dev(q0), cfg.eps, C_, K, n_moves, n_burnin=n_burnin,
                                           seed=11, stream_id=2, alpha=cfg.alpha)
    ref = run_seeded_chain(T, q0, cfg.eps, C_, K, cfg.alpha, n_moves, n_burnin, 11, 2)
    ref_all = run_seeded_chain(T, q0, cfg.eps, C_, K, cfg.alpha, n_moves, 0, 11, 2)
    fl = chain_floor(spec, cfg.eps, C_, K, cfg.alpha, n_moves, 11, 2, ref_all)
    bar = max(BAR, 10 * fl)
    gs, gl, ga = host(samples), host(logpost), host(acc)
    # decisions within 1e-8 of the threshold may legitimately flip
    margin = np.abs(np.log([orng.mh_uniform(11, 2, m) for m in range(n_moves)])
                    - (ref_all[4] - ref_all[5]))
    record("chain_c1", accepted=int(ga.sum()), ref_accepted=int(ref[2].sum()),
           samples=rel(gs, ref[0]), logpost=rel(gl, ref[1]), floor=fl, bar=bar,
           min_margin=float(margin.min()), sweeps=stats.sweeps, eig_calls=stats.eig_calls,
           res_p=stats.max_res_p, res_q=stats.max_res_q)
    assert margin.min() > 1e-8
    assert gs.shape == (n_moves - n_burnin, spec.D)
    assert ref[2].sum() >= 2            # the reference accepts at this step size
    assert np.array_equal(ga, ref[2])
    assert rel(gs, ref[0]) < bar and rel(gl, ref[1]) < bar
    assert stats.leapfrogs == n_moves * C_
    assert stats.accepted == int(ref[2].sum()) and stats.accepted_all == int(ref_all[2].sum())
    assert stats.failures == 0
    assert stats.max_res_p < 1e-6 and stats.max_res_q < 1e-6


def test_chain_failures_are_rejections(rm):
    """A first point the eigensolver cannot finish (one sweep allowed) is an
    error; a step size far beyond stability (eps = 5) makes every trajectory
    leave the domain, as in the reference: each move is a counted failure and
    a rejection, and q stays at q0."""
    spec, cfg = wl.workload("gp_logistic_d34")
    q0 = np.zeros(spec.D)
    M = rm.Model(spec)
    with pytest.raises(rm.RmhmcError):
        M.chain(dev(q0), cfg.eps, 2, 3, 2, max_sweeps=1)
    with np.errstate(all="ignore"):
        ref = run_seeded_chain(oham.GPTarget(spec), q0, 5.0, 2, 3, cfg.alpha, 3, 0, 3, 0)
    assert not ref[2].any() and not np.isfinite(ref[5]).any()
    samples, logpost, acc, stats = M.chain(dev(q0), 5.0, 2, 3, 3, seed=3)
    record("chain_fail", failures=stats.failures, not_pd=stats.fail_not_pd,
           nonfinite=stats.fail_nonfinite, noconv=stats.fail_noconv, accepted=stats.accepted)
    assert stats.failures == 3 and stats.accepted == 0
    assert stats.failures <= stats.fail_not_pd + stats.fail_nonfinite + stats.fail_noconv
    assert not host(acc).any()
    assert np.array_equal(host(samples), np.zeros((3, spec.D)))


# ---------------------------------------------------------------- g = sqrt(kappa^2 + lambda^2)
SQRT = osoft.SqrtMap(1.0)   # kappa = 1 (alpha = 1), the paper's own softabs


@pytest.mark.parametrize("case", ["c1_hessian", "cluster_130"])
def test_softabs_eig_sqrt_map(rm, case):
    """The eigensolver with the sqrt map, held to the bars of the coth cases
    (G^-1 p against the reference's own spread under a permutation)."""
    if case == "c1_hessian":
        spec = MODELS["c1_d34"]
        H = omodel.hessian(spec, rand_q(spec, 5))[2]
    else:
        H = cluster_matrix(130, 4)
    check_static_eig(rm, case, 0.5 * (H + H.T), 1.0, sqrt_map=True)


@pytest.mark.parametrize("name", ["c1_d34", "mkl_d104_wellcond", "mkl_d104"])
def test_metric_grad_and_glf_sqrt_map(rm, name):
    spec = MODELS[name]
    T = oham.GPTarget(spec)
    q = rand_q(spec, 13, 0.3)
    st = oham.State(T, q, SQRT)
    p = omomentum(st, np.random.default_rng(14).standard_normal(spec.D))
    M = rm.Model(spec)
    dq, dp, ham = M.metric_grad(dev(q), dev(p), dev(st.eig["Psi"].T), dev(st.eig["lam"]), 1.0,
                                softabs=rm.SOFTABS_SQRT)
    ref = (oham.grad_q(st, p), oham.grad_p(st, p), oham.hamiltonian(st, p))
    s2, q2, full = permuted(spec, q)
    st2 = oham.State(oham.GPTarget(s2), q2, SQRT)
    fl = max(rel(unpermute_vec(oham.grad_q(st2, p[full]), full), ref[0]),
             rel(unpermute_vec(oham.grad_p(st2, p[full]), full), ref[1]),
             rel(oham.hamiltonian(st2, p[full]), ref[2]))
    e_dq, e_dp, e_h = rel(host(dq), ref[0]), rel(host(dp), ref[1]), rel(host(ham), ref[2])
    tol = max(BAR, 10 * fl)
    record("metric_grad_sqrt", model=name, dHdq=e_dq, dHdp=e_dp, ham=e_h, floor=fl, bar=tol)
    assert e_dq < tol and e_dp < tol and e_h < tol
    # one generalized leapfrog with the same map
    eps = 0.01
    S = rm.State(M, dev(q), dev(p), 1.0, softabs=rm.SOFTABS_SQRT)
    S.step(eps, 6)
    qg, pg, _ = S.get()
    rst, rp = oglf(st, p, eps, 6)
    st2n, p2n = oglf(st2, p[full], eps, 6)
    fl = max(rel(unpermute_vec(st2n.q, full), rst.q), rel(unpermute_vec(p2n, full), rp))
    tol = max(BAR, 10 * fl)
    e_q, e_p = rel(host(qg), rst.q), rel(host(pg), rp)
    record("glf_sqrt", model=name, q=e_q, p=e_p, floor=fl, bar=tol)
    assert e_q < tol and e_p < tol


def test_chain_sqrt_map_c1(rm):
    """The seeded device chain with the paper's softabs map against the
    reference chain: identical decisions, samples within the floor bar."""
    spec, cfg = wl.workload("gp_logistic_d34")
    T = oham.GPTarget(spec)
    n_moves, C_, K, eps = 4, 3, 6, 0.02
    q0 = np.zeros(spec.D)
    s, l, a, stats = rm.Model(spec).chain(dev(q0), eps, C_, K, n_moves, seed=21, stream_id=1,
                                          alpha=1.0, softabs=rm.SOFTABS_SQRT)
    ref = run_seeded_chain(T, q0, eps, C_, K, SQRT, n_moves, 0, 21, 1)
    fl = chain_floor(spec, eps, C_, K, SQRT, n_moves, 21, 1, ref)
    bar = max(BAR, 10 * fl)
    gs, ga = host(s), host(a)
    record("chain_sqrt", accepted=int(ga.sum()), ref_accepted=int(ref[2].sum()),
           samples=rel(gs, ref[0]), floor=fl, bar=bar, failures=stats.failures)
    assert np.array_equal(ga, ref[2]) and ref[2].sum() >= 2
    assert rel(gs, ref[0]) < bar
