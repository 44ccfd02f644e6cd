"""Latent-GP negative log posterior U(q), its gradient, Hessian H(q) and the
third-derivative contraction v(W) = grad_q tr(W H(q)).  FP64 reference.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper anchors
-------------
* Per-sample likelihood exp(-U_i(f(X_i))): Sec. 2.1, Eq. (data_likelihood).
  Its third derivatives are diagonal in the sample index, which is what the
  structured contraction of Sec. 2.3 exploits; with the latent values f as
  coordinates the feature matrix of Sec. 2.3 is the identity, so the
  likelihood part of tr(W dH/dq) reduces to diag(W_ff) * U_i'''.
* Multiple-kernel GP prior (sum of kernels): Sec. 2.1, Eq. (BMKL).
* Power posterior (only the likelihood is raised to the power beta):
  Appendix "MC integration for the calculation of BME".

Every function here is written so that it also runs on complex inputs
without conjugation or absolute values (solve/inv/slogdet only), which lets
the tests pin gradients and Hessians with the complex-step derivative.

Notation (also in the module docstring of ``paper_2511_06407_amd.workloads``):
q = (f, eta); K = K(eta) incl. jitter; alpha = K^-1 f; K_l = dK/d eta_l;
A_l = K^-1 K_l; l_i(f_i) per-sample negative log likelihood.
"""
from __future__ import annotations

import math

import numpy as np

from paper_2511_06407_amd.workloads import (SE_ISO, SE_ARD, LINEAR_ARD, BINARY_SAME,
                                            LIK_BERNOULLI_LOGIT, LIK_GAUSSIAN, LIK_GAUSSIAN_MV,
                                            term_nparams)

LOG2PI = math.log(2.0 * math.pi)


# --------------------------------------------------------------------------
# Kernel matrix and its hyperparameter derivatives
# --------------------------------------------------------------------------

def _term_layout(spec):
    """[(kind, cols, first_param_index, nparams)] in parameter order."""
    out, i = [], 0
    for kind, cols in spec.terms:
        n = term_nparams(kind, cols)
        out.append((kind, cols, i, n))
        i += n
    return out


def _term_mask(spec, t):
    """1 where term t acts: between two points of its latent function (Sec.
    2.1: each f_j has its own GP prior), everywhere for untagged terms."""
    if not spec.term_fns or spec.term_fns[t] < 0:
        return 1.0
    on = spec.X[:, spec.fn_col] == spec.term_fns[t]
    return (on[:, None] & on[None, :]).astype(np.float64)


def _se_pieces(spec, eta, cols, i0, kind):
    """log K of one squared-exponential term and its eta-derivatives.

    log K = 2 eta_s - 1/2 sum_g R_g exp(-2 eta_g), with R_g the squared
    distance over the columns sharing lengthscale g.  Returns (Kterm, c1, c2,
    c3) where c1[j] = d logK / d eta_(i0+j) as arrays, c2 and c3 hold only the
    non-zero diagonal entries (d^2/d eta_g^2 = -2 u_g, d^3 = 4 u_g).
    """
    X = spec.X
    groups = [list(cols)] if kind == SE_ISO else [[c] for c in cols]
    u = []
    for g, gcols in enumerate(groups):
        R = 0.0
        for c in gcols:
            R = R + (X[:, c, None] - X[None, :, c]) ** 2
        u.append(R * np.exp(-2.0 * eta[i0 + 1 + g]))
    logk = 2.0 * eta[i0] - 0.5 * sum(u)
    Kt = np.exp(logk)
    c1 = [2.0 * np.ones_like(Kt)] + u
    c2 = {1 + g: -2.0 * u[g] for g in range(len(groups))}
    c3 = {1 + g: 4.0 * u[g] for g in range(len(groups))}
    return Kt, c1, c2, c3


def gram(spec, eta):
    """K(eta) = sum of kernel terms + jitter I (Sec. 2.1, Eq. BMKL); a term
    tagged with a latent function acts only within that function's block."""
    N = spec.N
    K = spec.jitter * np.eye(N, dtype=np.result_type(eta, np.float64))
    for t, (kind, cols, i0, n) in enumerate(_term_layout(spec)):
        if kind in (SE_ISO, SE_ARD):
            Kt = _se_pieces(spec, eta, cols, i0, kind)[0]
        elif kind == LINEAR_ARD:
            Kt = 0.0
            for j, c in enumerate(cols):
                Kt = Kt + np.exp(eta[i0 + j]) * np.outer(spec.X[:, c], spec.X[:, c])
        elif kind == BINARY_SAME:
            c = cols[0]
            Kt = np.exp(2.0 * eta[i0]) * (spec.X[:, c, None] == spec.X[None, :, c])
        K = K + _term_mask(spec, t) * Kt
    return K


class KernelDerivs:
    """Hyperparameter derivatives of K, evaluated on demand.

    ``d(idx)`` returns the matrix d^k K / d eta_idx[0] ... d eta_idx[k-1]
    (k = 1, 2 or 3) or ``None`` when it is identically zero (parameters of
    different kernel terms never interact).  Squared-exponential terms use the
    chain rule for exp(log K): with c = derivatives of log K,
      K_l   = K c_l
      K_lm  = K (c_l c_m + c_lm)
      K_lmn = K (c_l c_m c_n + c_lm c_n + c_ln c_m + c_mn c_l + c_lmn).
    Linear-ARD terms have every derivative equal to the term itself (one
    parameter each); same-value binary terms scale by 2 per derivative.
    """

    def __init__(self, spec, eta):
        self.spec, self.eta = spec, eta
        self.owner = {}
        self.cache = {}
        for t, (kind, cols, i0, n) in enumerate(_term_layout(spec)):
            for j in range(n):
                self.owner[i0 + j] = (t, kind, cols, i0, j)

    def _se(self, t, kind, cols, i0):
        if t not in self.cache:
            self.cache[t] = _se_pieces(self.spec, self.eta, cols, i0, kind)
        return self.cache[t]

    def d(self, idx):
        idx = tuple(idx)
        terms = {self.owner[i][0] for i in idx}
        if len(terms) != 1:
            return None
        out = self._d(idx)
        return None if out is None else _term_mask(self.spec, self.owner[idx[0]][0]) * out

    def _d(self, idx):
        t, kind, cols, i0, _ = self.owner[idx[0]]
        loc = [i - i0 for i in idx]
        if kind in (SE_ISO, SE_ARD):
            Kt, c1, c2, c3 = self._se(t, kind, cols, i0)

            def C2(a, b):
                return c2[a] if (a == b and a in c2) else 0.0
            if len(loc) == 1:
                (a,) = loc
                return Kt * c1[a]
            if len(loc) == 2:
                a, b = loc
                return Kt * (c1[a] * c1[b] + C2(a, b))
            a, b, c = loc
            c3v = c3[a] if (a == b == c and a in c3) else 0.0
            return Kt * (c1[a] * c1[b] * c1[c] + C2(a, b) * c1[c] + C2(a, c) * c1[b]
                         + C2(b, c) * c1[a] + c3v)
        if kind == LINEAR_ARD:
            if len(set(loc)) != 1:
                return None
            c = cols[loc[0]]
            return np.exp(self.eta[idx[0]]) * np.outer(self.spec.X[:, c], self.spec.X[:, c])
        if kind == BINARY_SAME:
            c = cols[0]
            Kt = np.exp(2.0 * self.eta[idx[0]]) * (self.spec.X[:, c, None] == self.spec.X[None, :, c])
            return (2.0 ** len(loc)) * Kt
        raise ValueError(kind)


# --------------------------------------------------------------------------
# Likelihood pieces (Sec. 2.1, Eq. data_likelihood; logistic form Sec. 2.5)
# --------------------------------------------------------------------------

def lik_terms(spec, f):
    """(l_i, l_i', l_i'', l_i''') of the per-sample negative log likelihood."""
    y = spec.y
    if spec.lik == LIK_BERNOULLI_LOGIT:
        # l(f) = log(1 + e^f) - y f   (y in {0,1}; same as log(1+e^{-y' f}), y' = +-1)
        if np.iscomplexobj(f):
            l0 = np.log1p(np.exp(f)) - y * f
        else:
            l0 = np.logaddexp(0.0, f) - y * f
        s = 1.0 / (1.0 + np.exp(-f))
        return l0, s - y, s * (1.0 - s), s * (1.0 - s) * (1.0 - 2.0 * s)
    if spec.lik == LIK_GAUSSIAN:
        v = spec.noise_var
        r = f - y
        return (0.5 * r * r / v + 0.5 * math.log(2.0 * math.pi * v), r / v,
                np.full_like(f, 1.0 / v), np.zeros_like(f))
    raise ValueError(spec.lik)


def mv_value(spec, f):
    """Per-record negative log likelihood of the mean/variance model (Sec.
    2.1, Eq. mvmodel): y_i ~ N(f1_i, delta + exp f2_i), with f = (f1, f2)."""
    R = spec.N // 2
    a, b, y = f[:R], f[R:], spec.y[:R]
    v = spec.delta + np.exp(b)
    return 0.5 * (y - a) ** 2 / v + 0.5 * np.log(2.0 * np.pi * v)


def mv_partials(spec, f):
    """Partial derivatives of mv_value in (a, b) = (f1_i, f2_i), up to third
    order, from l = r^2 / (2v) + ln(2 pi v) / 2 with r = a - y, v = delta + e,
    e = exp(b), dv/db = e:
      l_a = r/v, l_aa = 1/v, l_aaa = 0, l_ab = -r e / v^2, l_aab = -e / v^2,
      l_b = (e/v - r^2 e / v^2) / 2, l_abb = -r e (v - 2e) / v^3,
      l_bb = (delta e / v^2 - r^2 e (v - 2e) / v^3) / 2,
      l_bbb = (delta e (v - 2e) / v^3 - r^2 (e/v^2 - 6 e^2/v^3 + 6 e^3/v^4)) / 2."""
    R = spec.N // 2
    a, b, y = f[:R], f[R:], spec.y[:R]
    e = np.exp(b)
    v = spec.delta + e
    r = a - y
    dl = spec.delta
    return {
        "a": r / v, "b": 0.5 * (e / v - r * r * e / v ** 2),
        "aa": 1.0 / v, "ab": -r * e / v ** 2,
        "bb": 0.5 * (dl * e / v ** 2 - r * r * e * (v - 2.0 * e) / v ** 3),
        "aaa": np.zeros_like(v), "aab": -e / v ** 2,
        "abb": -r * e * (v - 2.0 * e) / v ** 3,
        "bbb": 0.5 * (dl * e * (v - 2.0 * e) / v ** 3
                      - r * r * (e / v ** 2 - 6.0 * e * e / v ** 3 + 6.0 * e ** 3 / v ** 4)),
    }


def lik_parts(spec, f):
    """The likelihood in the latent coordinates: (sum_i l_i, gradient,
    Hessian, v3) with v3(W)_k = sum_mn W_mn d^3 L / df_k df_m df_n.  The
    single-function likelihoods are diagonal in the points; the mean/variance
    model couples the two functions' values at each record (a 2 x 2 block per
    record: Sec. 2.3's per-sample structure with J = 2)."""
    if spec.lik != LIK_GAUSSIAN_MV:
        l0, l1, l2, l3 = lik_terms(spec, f)
        return np.sum(l0), l1, np.diag(l2), lambda W: np.diag(W) * l3
    R = spec.N // 2
    d = mv_partials(spec, f)
    g = np.concatenate([d["a"], d["b"]])
    H = np.zeros((spec.N, spec.N), dtype=np.result_type(f, np.float64))
    i = np.arange(R)
    H[i, i] = d["aa"]
    H[R + i, R + i] = d["bb"]
    H[i, R + i] = d["ab"]
    H[R + i, i] = d["ab"]

    def v3(W):
        w11, w22 = np.diag(W)[:R], np.diag(W)[R:]
        w12 = 0.5 * (W[i, R + i] + W[R + i, i])
        return np.concatenate([w11 * d["aaa"] + 2.0 * w12 * d["aab"] + w22 * d["abb"],
                               w11 * d["aab"] + 2.0 * w12 * d["abb"] + w22 * d["bbb"]])
    return np.sum(mv_value(spec, f)), g, H, v3


def lik_sum(spec, f):
    """-ln P(X | f): the sum of the per-record negative log likelihoods."""
    if spec.lik == LIK_GAUSSIAN_MV:
        return np.sum(mv_value(spec, f))
    return np.sum(lik_terms(spec, f)[0])


# --------------------------------------------------------------------------
# U, grad U, H
# --------------------------------------------------------------------------

def neg_log_post(spec, q):
    """U(q) = -ln P(q): beta*sum l_i + 1/2 f'K^-1 f + 1/2 ln|K| + 1/2 eta'eta + consts.

    Written from the definitions only (no derivative formulas), so that the
    complex-step derivative of this function pins ``gradient``.
    """
    N, P = spec.N, spec.P
    f, eta = q[:N], q[N:]
    K = gram(spec, eta)
    a = np.linalg.solve(K, f)
    sign, logabs = np.linalg.slogdet(K)
    logdet = logabs + np.log(sign) if np.iscomplexobj(K) else logabs
    return (spec.beta * lik_sum(spec, f) + 0.5 * f @ a + 0.5 * logdet + 0.5 * eta @ eta
            + 0.5 * (N + P) * LOG2PI)


def gradient(spec, q):
    """grad U: f-part beta l' + K^-1 f; eta_l part -1/2 a'K_l a + 1/2 tr(K^-1 K_l) + eta_l."""
    N, P = spec.N, spec.P
    f, eta = q[:N], q[N:]
    K = gram(spec, eta)
    Kinv = np.linalg.inv(K)
    a = Kinv @ f
    kd = KernelDerivs(spec, eta)
    g = np.empty(N + P, dtype=np.result_type(q, np.float64))
    g[:N] = spec.beta * lik_parts(spec, f)[1] + a
    for l in range(P):
        Kl = kd.d((l,))
        g[N + l] = -0.5 * a @ (Kl @ a) + 0.5 * np.sum(Kinv * Kl) + eta[l]
    return g


def hessian(spec, q):
    """U, grad U and the Hessian H of U at q.

    H_ff = beta L'' + K^-1   (L'' = diag(l'') for one latent function)
    H_fl = -A_l alpha
    H_lm = a'K_l A_m a - 1/2 a'K_lm a + 1/2 tr(K^-1 K_lm) - 1/2 tr(A_l A_m) + delta_lm
    """
    N, P = spec.N, spec.P
    f, eta = q[:N], q[N:]
    K = gram(spec, eta)
    Kinv = np.linalg.inv(K)
    a = Kinv @ f
    kd = KernelDerivs(spec, eta)
    Kl = [kd.d((l,)) for l in range(P)]
    A = [Kinv @ Kl[l] for l in range(P)]
    lsum, l1, Hl, _ = lik_parts(spec, f)
    dt = np.result_type(q, np.float64)
    H = np.zeros((N + P, N + P), dtype=dt)
    H[:N, :N] = 0.5 * (Kinv + Kinv.T) + spec.beta * Hl
    for l in range(P):
        col = -(A[l] @ a)
        H[:N, N + l] = col
        H[N + l, :N] = col
    for l in range(P):
        kla = Kl[l] @ a
        for m in range(l, P):                   # H_lm = H_ml: fill both
            Klm = kd.d((l, m))
            v = kla @ (A[m] @ a) - 0.5 * np.sum(A[l] * A[m].T) + (1.0 if l == m else 0.0)
            if Klm is not None:
                v = v - 0.5 * a @ (Klm @ a) + 0.5 * np.sum(Kinv * Klm)
            H[N + l, N + m] = v
            H[N + m, N + l] = v
    sign, logabs = np.linalg.slogdet(K)
    logdet = logabs + np.log(sign) if np.iscomplexobj(K) else logabs
    U = (spec.beta * lsum + 0.5 * f @ a + 0.5 * logdet + 0.5 * eta @ eta
         + 0.5 * (N + P) * LOG2PI)
    grad = np.empty(N + P, dtype=dt)
    grad[:N] = spec.beta * l1 + a
    for l in range(P):
        grad[N + l] = -0.5 * a @ (Kl[l] @ a) + 0.5 * np.sum(Kinv * Kl[l]) + eta[l]
    return U, grad, H


# --------------------------------------------------------------------------
# Third-derivative contraction (Sec. 2.3)
# --------------------------------------------------------------------------

def contract(spec, q, W):
    """v(W)_i = tr(W dH/dq_i) for a fixed symmetric W, without forming dH/dq.

    Sec. 2.3 orders the computation of tr(W_s dH/dq) by model structure so the
    D^3 derivative tensor is never built.  In the latent parameterisation the
    likelihood block is diagonal (f-part term 1 below); the hyperparameter
    blocks (omitted in the paper's display) are written out here in full.
    With w_l = W[f, eta_l], u_l = K^-1 w_l, a_m = A_m alpha, k_l = K_l alpha:

    v_f = beta v3(W_ff) - 2 sum_l A_l u_l   (v3 = diag(W_ff) l''' for one function)
          + K^-1 [ 2 sum_lm W_lm K_l a_m - sum_lm W_lm K_lm alpha ]
    v_n = -tr(K^-1 W_ff K^-1 K_n) + 2 sum_l [u_l'K_n a_l + u_l'K_l a_n - u_l'K_ln alpha]
          + sum_lm W_lm dH_lm/d eta_n
    """
    N, P = spec.N, spec.P
    f, eta = q[:N], q[N:]
    W = 0.5 * (W + W.T)
    Wff, w, Wee = W[:N, :N], W[:N, N:], W[N:, N:]
    K = gram(spec, eta)
    Kinv = np.linalg.inv(K)
    a = Kinv @ f
    kd = KernelDerivs(spec, eta)
    K1 = [kd.d((l,)) for l in range(P)]
    K2 = [[kd.d((l, m)) for m in range(P)] for l in range(P)]
    A = [Kinv @ K1[l] for l in range(P)]
    B = [A[l] @ Kinv for l in range(P)]            # K^-1 K_l K^-1
    am = [A[m] @ a for m in range(P)]
    kl = [K1[l] @ a for l in range(P)]
    zero = np.zeros(N)
    k2a = [[(K2[l][m] @ a) if K2[l][m] is not None else zero for m in range(P)] for l in range(P)]
    ik2a = [[Kinv @ k2a[l][m] for m in range(P)] for l in range(P)]
    Aam = [[A[l] @ am[m] for m in range(P)] for l in range(P)]
    u = [Kinv @ w[:, l] for l in range(P)]
    v3 = lik_parts(spec, f)[3]

    v = np.zeros(N + P)
    # f-part
    vf = spec.beta * v3(Wff)
    for l in range(P):
        vf = vf - 2.0 * (A[l] @ u[l])
    z = np.zeros(N)
    for l in range(P):
        for m in range(P):
            z = z + Wee[l, m] * (2.0 * (K1[l] @ am[m]) - k2a[l][m])
    v[:N] = vf + Kinv @ z

    # eta-part
    S = Kinv @ Wff @ Kinv
    CW = np.zeros((N, N))
    for l in range(P):
        Bl = np.zeros((N, N))
        for m in range(P):
            Bl = Bl + Wee[l, m] * A[m]
        CW = CW + A[l] @ Bl                          # sum_lm W_lm A_l A_m
    # BK[n][l][m] = tr(K^-1 K_n K^-1 K_lm) = sum(B_n * K_lm)
    BK = [[[np.sum(B[n] * K2[l][m]) if K2[l][m] is not None else 0.0 for m in range(P)]
           for l in range(P)] for n in range(P)]
    for n in range(P):
        vn = -np.sum(S * K1[n])
        for l in range(P):
            vn += 2.0 * (u[l] @ (K1[n] @ am[l]) + u[l] @ (K1[l] @ am[n]) - u[l] @ k2a[l][n])
        acc = np.sum(A[n].T * CW)                    # sum_lm W_lm tr(A_n A_l A_m)
        for l in range(P):
            for m in range(P):
                wlm = Wee[l, m]
                if wlm == 0.0:
                    continue
                d = (-kl[n] @ Aam[l][m] + k2a[l][n] @ am[m] - kl[l] @ Aam[n][m]
                     + kl[l] @ ik2a[m][n] - kl[l] @ Aam[m][n] + kl[n] @ ik2a[l][m])
                K3 = kd.d((l, m, n))
                if K3 is not None:
                    d += -0.5 * a @ (K3 @ a) + 0.5 * np.sum(Kinv * K3)
                d += -0.5 * (BK[n][l][m] + BK[m][l][n] + BK[l][m][n])
                acc += wlm * d
        v[N + n] = vn + acc
    return v
