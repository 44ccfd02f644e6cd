"""ctypes binding of librmhmc.so (C ABI in include/rmhmc.h).

Argument marshalling only: every step of the sampler runs in the HIP
library.  Device arrays are torch CUDA tensors (float64, contiguous); streams
are torch.cuda streams.  Importing this module loads the library and raises
if it has not been built (``python -m paper_2511_06407_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import workloads as wl

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librmhmc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2511_06407_amd.build`")
# torch ships its own HIP runtime under the same soname (libamdhip64.so.7)
# as the one the library links against; whichever is loaded first serves the
# whole process.  Loading torch first makes its runtime the shared one, so
# its tensors and streams are valid in the library (loaded the other way
# round, torch finds no GPU).
import torch  # noqa: E402,F401
_lib = C.CDLL(LIB_PATH)

MAX_TERM_COLS = 8
OK, E_ARG, E_NOT_PD, E_EIG_NOCONV, E_NONFINITE, E_NOMEM, E_HIP = 0, -1, -2, -3, -4, -5, -6
FP64, MIXED = 0, 1
SOFTABS_COTH, SOFTABS_SQRT = 0, 1

EXPORTED = ["rmhmc_model_create", "rmhmc_model_dims", "rmhmc_model_destroy", "rmhmc_hessian",
            "rmhmc_softabs_eig", "rmhmc_metric_grad", "rmhmc_state_create", "rmhmc_state_get",
            "rmhmc_state_set_momentum", "rmhmc_state_destroy", "rmhmc_glf_step", "rmhmc_chain",
            "rmhmc_gemm_f64", "rmhmc_gemm_f32", "rmhmc_gemm_f64_splitk", "rmhmc_last_error",
            "rmhmc_state_draw_momentum",
            "rmhmc_timing_enable", "rmhmc_timing_read", "rmhmc_pool_create", "rmhmc_pool_submit",
            "rmhmc_pool_poll", "rmhmc_pool_destroy", "rmhmc_state_stats", "rmhmc_model_bytes",
            "rmhmc_softabs_eig_reserve", "rmhmc_chain_randoms", "rmhmc_softabs_eig_noalloc",
            "rmhmc_batch_create", "rmhmc_batch_admit", "rmhmc_batch_step", "rmhmc_batch_sync",
            "rmhmc_batch_retire", "rmhmc_batch_destroy", "rmhmc_model_set_beta",
            "rmhmc_log_likelihood", "rmhmc_basis_model_create", "rmhmc_gemm_tallk_f64",
            "rmhmc_gemm_tallk_f32"]

TIMER_KINDS = {"gemm_f64": 0, "gemm_f32": 1, "jacobi_round": 2, "jacobi_round_static": 3, "kd_wsum": 4,
               "kd_matvec": 5, "potrf_diag": 6}


class KernelTerm(C.Structure):
    _fields_ = [("kind", C.c_int), ("ncols", C.c_int), ("cols", C.c_int * MAX_TERM_COLS),
                ("fn", C.c_int)]


class ModelDesc(C.Structure):
    _fields_ = [("N", C.c_int), ("dx", C.c_int), ("X", C.POINTER(C.c_double)),
                ("y", C.POINTER(C.c_double)), ("lik", C.c_int), ("noise_var", C.c_double),
                ("nterms", C.c_int), ("terms", C.POINTER(KernelTerm)), ("jitter", C.c_double),
                ("beta", C.c_double), ("n_fns", C.c_int), ("fn_col", C.c_int),
                ("delta", C.c_double)]


class BasisDesc(C.Structure):
    _fields_ = [("N", C.c_int), ("dx", C.c_int), ("X", C.POINTER(C.c_double)),
                ("y", C.POINTER(C.c_double)), ("lik", C.c_int), ("noise_var", C.c_double),
                ("kinds", C.POINTER(C.c_int)), ("M", C.c_int), ("L", C.c_double),
                ("bias_var", C.c_double), ("ig_alpha", C.c_double * 3), ("ig_beta", C.c_double * 3),
                ("beta", C.c_double)]


class ChainCfg(C.Structure):
    _fields_ = [("eps", C.c_double), ("alpha", C.c_double), ("zeta", C.c_double),
                ("n_leapfrog", C.c_int), ("n_moves", C.c_int), ("n_burnin", C.c_int),
                ("n_fixed_point", C.c_int), ("max_sweeps", C.c_int), ("reorth_every", C.c_int),
                ("seed", C.c_ulonglong), ("stream_id", C.c_ulonglong), ("precision", C.c_int),
                ("softabs", C.c_int)]


class ChainStats(C.Structure):
    _fields_ = [("accepted", C.c_int), ("accepted_all", C.c_int), ("failures", C.c_int),
                ("fail_not_pd", C.c_int), ("fail_nonfinite", C.c_int), ("fail_noconv", C.c_int),
                ("leapfrogs", C.c_longlong), ("eig_calls", C.c_longlong),
                ("sweeps", C.c_longlong), ("eig_fallbacks", C.c_int),
                ("max_res_p", C.c_double), ("max_res_q", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = C.c_void_p
_i, _d = C.c_int, C.c_double
_sig = {
    "rmhmc_model_create": [C.POINTER(ModelDesc), _i, C.POINTER(_vp)],
    "rmhmc_model_dims": [_vp, C.POINTER(_i), C.POINTER(_i), C.POINTER(_i)],
    "rmhmc_model_bytes": [_vp, C.POINTER(C.c_longlong)],
    "rmhmc_model_set_beta": [_vp, _d],
    "rmhmc_log_likelihood": [_vp, _vp, _vp, _vp],
    "rmhmc_softabs_eig_reserve": [_i],
    "rmhmc_chain_randoms": [_i, C.c_ulonglong, C.c_ulonglong, C.c_ulonglong, _vp, _vp, _vp],
    "rmhmc_model_destroy": [_vp],
    "rmhmc_hessian": [_vp, _vp, _vp, _vp, _vp, _i, _vp],
    "rmhmc_softabs_eig": [_i, _vp, _i, _d, _i, _d, _i, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(_i),
                          _vp],
    "rmhmc_softabs_eig_noalloc": [_i, _vp, _i, _d, _i, _d, _i, _vp, _vp, _vp, _vp, _vp, _vp,
                                  C.POINTER(_i), _vp],
    "rmhmc_metric_grad": [_vp, _vp, _vp, _vp, _vp, _d, _i, _vp, _vp, _vp, _vp],
    "rmhmc_state_create": [_vp, _vp, _vp, _d, _i, _vp, C.POINTER(_vp)],
    "rmhmc_state_get": [_vp, _vp, _vp, _vp, _vp],
    "rmhmc_state_set_momentum": [_vp, _vp, _vp],
    "rmhmc_state_destroy": [_vp],
    "rmhmc_state_draw_momentum": [_vp, _vp, _vp],
    "rmhmc_state_stats": [_vp, C.POINTER(ChainStats)],
    "rmhmc_timing_enable": [C.c_uint],
    "rmhmc_pool_create": [_i, C.POINTER(_vp)],
    "rmhmc_pool_submit": [_vp, _vp, C.POINTER(ChainCfg), _vp, _vp, _vp, _vp,
                          C.POINTER(C.c_longlong)],
    "rmhmc_pool_poll": [_vp, C.c_longlong, _i, C.POINTER(_i), C.POINTER(ChainStats),
                        C.POINTER(_d)],
    "rmhmc_pool_destroy": [_vp],
    "rmhmc_batch_create": [_i, C.POINTER(_vp)],
    "rmhmc_batch_admit": [_vp, _vp, C.POINTER(ChainCfg), _vp, _vp, _vp, _vp, C.POINTER(_i)],
    "rmhmc_batch_step": [_vp, _i],
    "rmhmc_batch_sync": [_vp],
    "rmhmc_batch_retire": [_vp, _i, C.POINTER(_i), C.POINTER(ChainStats), C.POINTER(_i),
                           C.POINTER(_i)],
    "rmhmc_batch_destroy": [_vp],
    "rmhmc_timing_read": [_i, C.POINTER(C.c_longlong), C.POINTER(_d), C.POINTER(_d), C.POINTER(_d)],
    "rmhmc_glf_step": [_vp, _vp, _d, _i, _vp],
    "rmhmc_chain": [_vp, C.POINTER(ChainCfg), _vp, _vp, _vp, _vp, C.POINTER(ChainStats), _vp],
    "rmhmc_gemm_f64": [_i, _i, _i, _d, _vp, _i, _i, _vp, _i, _i, _d, _vp, _i, _vp],
    "rmhmc_gemm_f64_splitk": [_i, _i, _i, _vp, _i, _i, _vp, _i, _i, _vp, _i, _vp, _i, _vp],
    "rmhmc_gemm_f32": [_i, _i, _i, C.c_float, _vp, _i, _i, _vp, _i, _i, C.c_float, _vp, _i, _vp],
    "rmhmc_gemm_tallk_f64": [_i, _i, C.c_long, _vp, C.c_long, _vp, C.c_long, _vp, _i, _vp, _i, _vp],
    "rmhmc_gemm_tallk_f32": [_i, _i, C.c_long, _vp, C.c_long, _vp, C.c_long, _vp, _i, _vp, _i, _vp],
}
for _name, _args in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
_lib.rmhmc_last_error.restype = C.c_char_p
_lib.rmhmc_last_error.argtypes = []


class RmhmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"rmhmc status {status}: {msg}")
        self.status = status


def _check(status):
    if status != OK:
        raise RmhmcError(status, _lib.rmhmc_last_error().decode())


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t, dtype=None):
    if t is None:
        return None
    torch = _torch()
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    return C.c_void_p(t.data_ptr())


def _f64(t):
    return _ptr(t, _torch().float64)


def gemm_colmajor(m, n, k, A, lda, tA, B, ldb, tB, Cm, ldc, alpha=1.0, beta=0.0, stream=None):
    torch = _torch()
    if A.dtype == torch.float64:
        _check(_lib.rmhmc_gemm_f64(m, n, k, alpha, _f64(A), lda, int(tA), _f64(B), ldb, int(tB),
                                   beta, _f64(Cm), ldc, _stream(stream)))
    else:
        f32 = torch.float32
        _check(_lib.rmhmc_gemm_f32(m, n, k, alpha, _ptr(A, f32), lda, int(tA), _ptr(B, f32), ldb,
                                   int(tB), beta, _ptr(Cm, f32), ldc, _stream(stream)))


def gemm_splitk_colmajor(m, n, k, A, lda, tA, B, ldb, tB, Cm, ldc, work, splits, stream=None):
    """C = op(A) op(B) in FP64 with the k range split over `splits` layers."""
    _check(_lib.rmhmc_gemm_f64_splitk(m, n, k, _f64(A), lda, int(tA), _f64(B), ldb, int(tB),
                                      _f64(Cm), ldc, _f64(work), splits, _stream(stream)))


def gemm_tallk(m, n, k, A, lda, B, ldb, Cm, ldc, work, splits, stream=None):
    """C (FP64) = A' B over a long k: A, B hold m and n columns of length k
    (FP64 or FP32 operands, `work` of the operand type)."""
    torch = _torch()
    if A.dtype == torch.float64:
        _check(_lib.rmhmc_gemm_tallk_f64(m, n, k, _f64(A), lda, _f64(B), ldb, _f64(Cm), ldc,
                                         _f64(work), splits, _stream(stream)))
    else:
        f32 = torch.float32
        _check(_lib.rmhmc_gemm_tallk_f32(m, n, k, _ptr(A, f32), lda, _ptr(B, f32), ldb, _f64(Cm),
                                         ldc, _ptr(work, f32), splits, _stream(stream)))


class Model:
    """A latent-GP model resident on the device (rmhmc_model)."""

    def __init__(self, spec: wl.ModelSpec, precision=FP64):
        terms = (KernelTerm * len(spec.terms))()
        for t, (kind, cols) in enumerate(spec.terms):
            terms[t].kind = kind
            terms[t].ncols = len(cols)
            terms[t].fn = spec.term_fns[t] if spec.term_fns else -1
            for c, col in enumerate(cols):
                terms[t].cols[c] = col
        X = np.ascontiguousarray(spec.X, dtype=np.float64)
        y = np.ascontiguousarray(spec.y, dtype=np.float64)
        self._keep = (X, y, terms)
        desc = ModelDesc(spec.N, spec.dx, X.ctypes.data_as(C.POINTER(C.c_double)),
                         y.ctypes.data_as(C.POINTER(C.c_double)), spec.lik, spec.noise_var,
                         len(spec.terms), terms, spec.jitter, spec.beta,
                         2 if spec.lik == wl.LIK_GAUSSIAN_MV else 1, spec.fn_col, spec.delta)
        h = C.c_void_p()
        _check(_lib.rmhmc_model_create(C.byref(desc), precision, C.byref(h)))
        self._h = h
        N, P, D = C.c_int(), C.c_int(), C.c_int()
        _check(_lib.rmhmc_model_dims(h, C.byref(N), C.byref(P), C.byref(D)))
        self.N, self.P, self.D = N.value, P.value, D.value
        self.spec = spec
        self.precision = precision

    def close(self):
        if getattr(self, "_h", None):
            _lib.rmhmc_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def hessian(self, q, stream=None):
        torch = _torch()
        U = torch.empty(1, dtype=torch.float64, device=q.device)
        g = torch.empty(self.D, dtype=torch.float64, device=q.device)
        H = torch.empty((self.D, self.D), dtype=torch.float64, device=q.device)
        _check(_lib.rmhmc_hessian(self._h, _f64(q), _f64(U), _f64(g), _f64(H), self.D, _stream(stream)))
        # H is symmetric, so the row-major view equals the column-major matrix
        return U, g, H

    def metric_grad(self, q, p, Q, lam, alpha, stream=None, softabs=SOFTABS_COTH):
        """Q: device tensor whose column-major layout holds the eigenvectors,
        i.e. Q_t[j, i] = Q(i, j) (pass Q.T.contiguous() of a row-major matrix)."""
        torch = _torch()
        dq = torch.empty(self.D, dtype=torch.float64, device=q.device)
        dp = torch.empty(self.D, dtype=torch.float64, device=q.device)
        ham = torch.empty(1, dtype=torch.float64, device=q.device)
        _check(_lib.rmhmc_metric_grad(self._h, _f64(q), _f64(p), _f64(Q), _f64(lam), alpha,
                                      softabs, _f64(dq), _f64(dp), _f64(ham), _stream(stream)))
        return dq, dp, ham

    def set_beta(self, beta):
        """Inverse temperature of the power posterior for later calls."""
        _check(_lib.rmhmc_model_set_beta(self._h, float(beta)))

    def log_likelihood(self, q, stream=None):
        """ln P(X | f) at q, as a device scalar."""
        torch = _torch()
        ll = torch.empty(1, dtype=torch.float64, device=q.device)
        _check(_lib.rmhmc_log_likelihood(self._h, _f64(q), _f64(ll), _stream(stream)))
        return ll

    @property
    def device_bytes(self):
        b = C.c_longlong()
        _check(_lib.rmhmc_model_bytes(self._h, C.byref(b)))
        return b.value

    def chain(self, q0, eps, n_leapfrog, n_fixed_point, n_moves, n_burnin=0, seed=0,
              stream_id=0, alpha=1e6, zeta=0.0, max_sweeps=0, reorth_every=0, stream=None,
              softabs=SOFTABS_COTH):
        """Algorithm 1 on the device; returns (samples, logpost, accepted, stats)
        for the moves n_burnin .. n_moves-1."""
        torch = _torch()
        kept = n_moves - n_burnin
        samples = torch.empty((max(kept, 1), self.D), dtype=torch.float64, device=q0.device)
        logpost = torch.empty(max(kept, 1), dtype=torch.float64, device=q0.device)
        acc = torch.empty(max(kept, 1), dtype=torch.int32, device=q0.device)
        cfg = chain_cfg(self, eps, n_leapfrog, n_fixed_point, n_moves, n_burnin, seed, stream_id,
                        alpha, zeta, max_sweeps, reorth_every, softabs)
        stats = ChainStats()
        _check(_lib.rmhmc_chain(self._h, C.byref(cfg), _f64(q0), _f64(samples), _f64(logpost),
                                _ptr(acc, torch.int32), C.byref(stats), _stream(stream)))
        return samples[:kept], logpost[:kept], acc[:kept], stats


class BasisModel(Model):
    """The paper's reduced-rank basis model resident on the device
    (rmhmc_basis_model_create); every Model method applies."""

    def __init__(self, spec: wl.BasisSpec):
        X = np.ascontiguousarray(spec.X, dtype=np.float64)
        y = np.ascontiguousarray(spec.y, dtype=np.float64)
        kinds = (C.c_int * spec.dx)(*spec.kinds)
        self._keep = (X, y, kinds)
        desc = BasisDesc(spec.N, spec.dx, X.ctypes.data_as(C.POINTER(C.c_double)),
                         y.ctypes.data_as(C.POINTER(C.c_double)), spec.lik, spec.noise_var,
                         kinds, spec.M, spec.L, spec.bias_var, (C.c_double * 3)(*spec.ig_alpha),
                         (C.c_double * 3)(*spec.ig_beta), spec.beta)
        h = C.c_void_p()
        _check(_lib.rmhmc_basis_model_create(C.byref(desc), C.byref(h)))
        self._h = h
        N, P, D = C.c_int(), C.c_int(), C.c_int()
        _check(_lib.rmhmc_model_dims(h, C.byref(N), C.byref(P), C.byref(D)))
        self.N, self.P, self.D = N.value, P.value, D.value
        self.spec = spec
        self.precision = FP64


def chain_cfg(model, eps, n_leapfrog, n_fixed_point, n_moves, n_burnin=0, seed=0, stream_id=0,
              alpha=1e6, zeta=0.0, max_sweeps=0, reorth_every=0, softabs=SOFTABS_COTH):
    return ChainCfg(eps, alpha, zeta, n_leapfrog, n_moves, n_burnin, n_fixed_point, max_sweeps,
                    reorth_every, seed, stream_id, model.precision, softabs)


def chain_randoms(D, seed, stream_id, move, stream=None):
    """(z, u) of one move of the chain (seed, stream_id), drawn on the device."""
    torch = _torch()
    z = torch.empty(D, dtype=torch.float64, device="cuda")
    u = torch.empty(1, dtype=torch.float64, device="cuda")
    _check(_lib.rmhmc_chain_randoms(D, seed, stream_id, move, _f64(z), _f64(u), _stream(stream)))
    return z, u


def softabs_eig_reserve(D):
    _check(_lib.rmhmc_softabs_eig_reserve(D))


def softabs_eig(H, alpha, Q_warm=None, zeta=0.0, max_sweeps=0, stream=None, noalloc=False,
                softabs=SOFTABS_COTH):
    """H: symmetric D x D device tensor.  Returns (Q_colmajor, lam, g, gp, logdetG, sweeps);
    Q_colmajor[j] is the j-th eigenvector.  noalloc: the entry point whose
    workspace is the library's static device array (D <= 1088)."""
    torch = _torch()
    D = H.shape[0]
    Q = torch.empty((D, D), dtype=torch.float64, device=H.device)
    lam = torch.empty(D, dtype=torch.float64, device=H.device)
    g = torch.empty(D, dtype=torch.float64, device=H.device)
    gp = torch.empty(D, dtype=torch.float64, device=H.device)
    ld = torch.empty(1, dtype=torch.float64, device=H.device)
    sw = C.c_int()
    fn = _lib.rmhmc_softabs_eig_noalloc if noalloc else _lib.rmhmc_softabs_eig
    _check(fn(D, _f64(H), D, alpha, softabs, zeta, max_sweeps, _f64(Q_warm), _f64(Q), _f64(lam),
              _f64(g), _f64(gp), _f64(ld), C.byref(sw), _stream(stream)))
    return Q, lam, g, gp, ld, sw.value


class State:
    """Device-resident integrator state (rmhmc_state)."""

    def __init__(self, model: Model, q0, p0, alpha=1e6, stream=None, softabs=SOFTABS_COTH):
        h = C.c_void_p()
        _check(_lib.rmhmc_state_create(model._h, _f64(q0), _f64(p0), alpha, softabs,
                                       _stream(stream), C.byref(h)))
        self._h, self.model = h, model

    def step(self, eps, n_fixed_point, stream=None):
        _check(_lib.rmhmc_glf_step(self.model._h, self._h, eps, n_fixed_point, _stream(stream)))

    def get(self, stream=None):
        torch = _torch()
        D = self.model.D
        q = torch.empty(D, dtype=torch.float64, device="cuda")
        p = torch.empty(D, dtype=torch.float64, device="cuda")
        ham = torch.empty(1, dtype=torch.float64, device="cuda")
        _check(_lib.rmhmc_state_get(self._h, _f64(q), _f64(p), _f64(ham), _stream(stream)))
        return q, p, ham

    def draw_momentum(self, z, stream=None):
        """p = Q diag(sqrt g) z at the current point (p ~ N(0, G(q)))."""
        _check(_lib.rmhmc_state_draw_momentum(self._h, _f64(z), _stream(stream)))

    def stats(self):
        st = ChainStats()
        _check(_lib.rmhmc_state_stats(self._h, C.byref(st)))
        return st

    def set_momentum(self, p, stream=None):
        _check(_lib.rmhmc_state_set_momentum(self._h, _f64(p), _stream(stream)))

    def close(self):
        if getattr(self, "_h", None):
            _lib.rmhmc_state_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def timing_enable(kinds=("gemm_f64",)):
    """Time the given kernel families (names of TIMER_KINDS); () switches off."""
    mask = 0
    for k in kinds:
        mask |= 1 << (TIMER_KINDS[k] if isinstance(k, str) else int(k))
    _check(_lib.rmhmc_timing_enable(mask))


def timing_read(kind):
    """(launches, kernel ms, algorithmic flops, algorithmic bytes) for a kernel family."""
    n, ms, fl, by = C.c_longlong(), C.c_double(), C.c_double(), C.c_double()
    _check(_lib.rmhmc_timing_read(TIMER_KINDS[kind] if isinstance(kind, str) else kind,
                                  C.byref(n), C.byref(ms), C.byref(fl), C.byref(by)))
    return n.value, ms.value, fl.value, by.value


class ChainJob:
    """Device buffers of one submitted chain (kept alive until collected)."""

    def __init__(self, model, q0, cfg):
        torch = _torch()
        kept = max(cfg.n_moves - cfg.n_burnin, 1)
        self.model, self.q0, self.cfg = model, q0, cfg
        self.samples = torch.empty((kept, model.D), dtype=torch.float64, device=q0.device)
        self.logpost = torch.empty(kept, dtype=torch.float64, device=q0.device)
        self.accepted = torch.empty(kept, dtype=torch.int32, device=q0.device)
        self.ticket = None
        self.stats = None
        self.times_ms = None


class Pool:
    """Worker pool running chains concurrently (rmhmc_pool)."""

    def __init__(self, n_workers=4):
        h = C.c_void_p()
        _check(_lib.rmhmc_pool_create(n_workers, C.byref(h)))
        self._h = h
        self.n_workers = n_workers

    def submit(self, model, q0, eps, n_leapfrog, n_fixed_point, n_moves, n_burnin=0, seed=0,
               stream_id=0, alpha=1e6, zeta=0.0, max_sweeps=0, reorth_every=0,
               softabs=SOFTABS_COTH):
        torch = _torch()
        job = ChainJob(model, q0, chain_cfg(model, eps, n_leapfrog, n_fixed_point, n_moves,
                                            n_burnin, seed, stream_id, alpha, zeta, max_sweeps,
                                            reorth_every, softabs))
        t = C.c_longlong()
        _check(_lib.rmhmc_pool_submit(self._h, model._h, C.byref(job.cfg), _f64(q0),
                                      _f64(job.samples), _f64(job.logpost),
                                      _ptr(job.accepted, torch.int32), C.byref(t)))
        job.ticket = t.value
        return job

    def poll(self, job, wait=False):
        """True when the job has finished (raises if it failed)."""
        done = C.c_int()
        stats = ChainStats()
        times = (C.c_double * 3)()
        _check(_lib.rmhmc_pool_poll(self._h, job.ticket, int(wait), C.byref(done),
                                    C.byref(stats), times))
        if done.value == 0:
            return False
        if done.value < 0:
            raise RmhmcError(done.value, _lib.rmhmc_last_error().decode())
        job.stats = stats
        job.times_ms = tuple(times)
        return True

    def wait(self, job):
        return self.poll(job, wait=True)

    def close(self):
        if getattr(self, "_h", None):
            _lib.rmhmc_pool_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Chains whose moves are captured into HIP graphs and replayed side by
    side on a few streams (rmhmc_batch)."""

    def __init__(self, n_streams=8):
        h = C.c_void_p()
        _check(_lib.rmhmc_batch_create(n_streams, C.byref(h)))
        self._h = h
        self.jobs = {}

    def admit(self, model, q0, eps, n_leapfrog, n_fixed_point, n_moves, n_burnin=0, seed=0,
              stream_id=0, alpha=1e6, zeta=0.0, max_sweeps=0, reorth_every=0,
              softabs=SOFTABS_COTH):
        torch = _torch()
        job = ChainJob(model, q0, chain_cfg(model, eps, n_leapfrog, n_fixed_point, n_moves,
                                            n_burnin, seed, stream_id, alpha, zeta, max_sweeps,
                                            reorth_every, softabs))
        slot = C.c_int()
        _check(_lib.rmhmc_batch_admit(self._h, model._h, C.byref(job.cfg), _f64(q0),
                                      _f64(job.samples), _f64(job.logpost),
                                      _ptr(job.accepted, torch.int32), C.byref(slot)))
        job.ticket = slot.value
        self.jobs[slot.value] = job
        return job

    def step(self, n_moves):
        _check(_lib.rmhmc_batch_step(self._h, n_moves))

    def sync(self):
        _check(_lib.rmhmc_batch_sync(self._h))

    def retire(self, job):
        done, budget, layers = C.c_int(), C.c_int(), C.c_int()
        st = ChainStats()
        _check(_lib.rmhmc_batch_retire(self._h, job.ticket, C.byref(done), C.byref(st),
                                       C.byref(budget), C.byref(layers)))
        job.stats = st
        job.moves_done = done.value
        job.shape = {"sweep_budget": budget.value, "gsplit": layers.value}
        self.jobs.pop(job.ticket, None)
        return job

    def close(self):
        if getattr(self, "_h", None):
            _lib.rmhmc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
