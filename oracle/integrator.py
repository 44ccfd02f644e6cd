"""Generalized (implicit) leapfrog.  FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper anchor: Sec. 2.2, Eq. (leapfrog):
    p(t+e/2) = p(t) - e/2 dH/dq(q(t), p(t+e/2))                      [implicit in p]
    q(t+e)   = q(t) + e/2 {dH/dp(q(t), p(t+e/2)) + dH/dp(q(t+e), p(t+e/2))}  [implicit in q]
    p(t+e)   = p(t+e/2) - e/2 dH/dq(q(t+e), p(t+e/2))                 [explicit]
The paper does not say how the two implicit equations are solved.  Here each
is solved by K plain fixed-point iterations started from p(t) and q(t), with
no early exit.  The q-iteration therefore evaluates the metric at K-1 new
points plus the end point, K eigendecompositions per leapfrog in all.

The fixed-point map is a contraction only for a small enough step: with the
softabs metric its Lipschitz constant grows with eps |G^-1 dG G^-1 p|, so a
step that is too long makes the iteration diverge instead of converging.  The
residuals ||p_(k+1) - p_k|| and ||q_(k+1) - q_k|| of every iteration can be
collected (argument `log`) to tell an unconverged or diverging solve from a
converged one.
"""
from __future__ import annotations

import numpy as np

from .hamiltonian import State, grad_q, grad_p


def glf_step(st, p, eps, n_fixed_point, log=None):
    """One generalized leapfrog from (st.q, p).  Returns (state at q', p').

    log: optional dict; its lists "res_p" and "res_q" receive the residual
    norm of every fixed-point iteration of this step."""
    if n_fixed_point < 1:
        raise ValueError("n_fixed_point must be >= 1")
    q = st.q
    res_p, res_q = [], []
    # implicit momentum half step at fixed q
    ph = np.array(p, dtype=np.float64)
    for _ in range(n_fixed_point):
        nxt = p - 0.5 * eps * grad_q(st, ph)
        res_p.append(float(np.linalg.norm(nxt - ph)))
        ph = nxt
    # implicit position step
    v0 = grad_p(st, ph)
    stk = st
    qk = q
    for k in range(n_fixed_point):
        if k > 0:
            stk = State(st.target, qk, st.alpha)
        nxt = q + 0.5 * eps * (v0 + grad_p(stk, ph))
        res_q.append(float(np.linalg.norm(nxt - qk)))
        qk = nxt
    if log is not None:
        log.setdefault("res_p", []).append(res_p)
        log.setdefault("res_q", []).append(res_q)
    st_new = State(st.target, qk, st.alpha)
    # explicit momentum half step
    p_new = ph - 0.5 * eps * grad_q(st_new, ph)
    return st_new, p_new


def trajectory(st, p, eps, n_leapfrog, n_fixed_point):
    for _ in range(n_leapfrog):
        st, p = glf_step(st, p, eps, n_fixed_point)
    return st, p
