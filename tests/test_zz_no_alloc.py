"""GPU: the eigensolver entry point that allocates nothing (its workspace is
the library's static device array) against the allocating one, through the
C ABI, on two calls in a row, the second with a smaller matrix: identical
sweeps and eigenvalues, and G, log|G|, G^-1 p within the FP64 bar."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2511_06407_amd import workloads as wl  # noqa: E402
from oracle import model as omodel  # noqa: E402
from tests.parity_util import rel, record  # noqa: E402

pytestmark = pytest.mark.gpu


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


def invariants(Qt, lam, g, p):
    Psi = host(Qt).T
    g = host(g)
    return (Psi * g) @ Psi.T, float(np.sum(np.log(g))), Psi @ ((Psi.T @ p) / g)


def test_noalloc_matches_allocating_entry_point(rm):
    spec, _ = wl.workload("propensity_mkl_d1038")
    q = 0.1 * np.random.default_rng(31).standard_normal(spec.D)
    H_big = omodel.hessian(spec, q)[2]
    small, _, _ = wl.gp_logistic_2d(200, seed=4)
    H_small = omodel.hessian(small, 0.3 * np.random.default_rng(5).standard_normal(small.D))[2]
    for name, H in (("d1038", H_big), ("d202", H_small)):   # second call: smaller input
        H = 0.5 * (H + H.T)
        D = H.shape[0]
        p = np.random.default_rng(D).standard_normal(D)
        a = rm.softabs_eig(dev(H), 1e6)
        b = rm.softabs_eig(dev(H), 1e6, noalloc=True)
        Ga, lda, gpa = invariants(a[0], a[1], a[2], p)
        Gb, ldb, gpb = invariants(b[0], b[1], b[2], p)
        e_G, e_ld, e_gp = rel(Gb, Ga), rel(ldb, lda), rel(gpb, gpa)
        same_lam = np.array_equal(host(a[1]), host(b[1]))
        record("noalloc_eig", matrix=name, D=D, sweeps_alloc=a[5], sweeps_noalloc=b[5], G=e_G,
               logdetG=e_ld, Ginvp=e_gp, identical_eigenvalues=int(same_lam))
        assert a[5] == b[5]
        assert e_G < 1e-10 and e_ld < 1e-10 and e_gp < 1e-10
        # warm start on the no-allocation path, from the allocating cold solve
        c = rm.softabs_eig(dev(H), 1e6, Q_warm=a[0])
        d = rm.softabs_eig(dev(H), 1e6, Q_warm=a[0], noalloc=True)
        Gc, ldc, gpc = invariants(c[0], c[1], c[2], p)
        Gd, ldd, gpd = invariants(d[0], d[1], d[2], p)
        assert c[5] == d[5]
        assert rel(Gd, Gc) < 1e-10 and rel(ldd, ldc) < 1e-10 and rel(gpd, gpc) < 1e-10


def test_noalloc_rejects_oversized_input(rm):
    H = dev(np.eye(1100))
    with pytest.raises(rm.RmhmcError) as ei:
        rm.softabs_eig(H, 1e6, noalloc=True)
    assert ei.value.status == rm.E_ARG
