"""Riemannian Hamiltonian and its derivatives for the softabs metric.  FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper anchors
-------------
* H(q,p) = -ln P(q) + 1/2 ln((2 pi)^d |G(q)|) + 1/2 p' G(q)^-1 p:
  Sec. 2.2, Eq. (Hamiltonian).
* dH/dp = G^-1 p and dH/dq: Sec. 2.2, Eq. (d_Hamiltonian).  The printed
  equation carries the two metric terms with swapped signs; differentiating
  Eq. (Hamiltonian) gives
      dH/dq_i = -d ln P/dq_i + 1/2 tr(G^-1 dG/dq_i) - 1/2 p'G^-1 (dG/dq_i) G^-1 p,
  which is what is implemented (the tests pin it with finite differences of H).
* Both trace terms come from the cached W1, W2 (Eq. Betancourt_formula) and the
  structured contraction of Sec. 2.3 (``model.contract``).
"""
from __future__ import annotations

import math

import numpy as np

from . import model, softabs

LOG2PI = math.log(2.0 * math.pi)


class GPTarget:
    """The latent-GP posterior as a sampling target."""

    def __init__(self, spec):
        self.spec = spec
        self.D = spec.D

    def derivs(self, q):
        return model.hessian(self.spec, q)

    def contract(self, q, W):
        return model.contract(self.spec, q, W)


class State:
    """Everything that depends on q only: U, grad U, H and its softabs eigen-state.
    v(W2) is q-only as well and is cached on first use."""

    def __init__(self, target, q, alpha):
        self.target, self.q, self.alpha = target, np.array(q, dtype=np.float64), alpha
        self.U, self.grad, self.H = target.derivs(self.q)
        if not (np.isfinite(self.U) and np.all(np.isfinite(self.H))):
            raise FloatingPointError("non-finite U or H")
        self.eig = softabs.softabs_eig(self.H, alpha)
        self._vW2 = None

    def v_w2(self):
        if self._vW2 is None:
            eig = self.eig
            W2 = (eig["Psi"] * (eig["gp"] / eig["g"])) @ eig["Psi"].T
            self._vW2 = self.target.contract(self.q, W2)
        return self._vW2


def hamiltonian(st, p):
    """H = U + 1/2 sum ln g + 1/2 sum (psi_j'p)^2 / g_j + D/2 ln 2 pi."""
    eig = st.eig
    c = eig["Psi"].T @ p
    return (st.U + 0.5 * eig["logdetG"] + 0.5 * np.sum(c * c / eig["g"])
            + 0.5 * p.size * LOG2PI)


def grad_p(st, p):
    return softabs.ginv_p(st.eig, p)


def grad_q(st, p):
    """dH/dq = grad U + 1/2 v(W2) - 1/2 v(W1(p))."""
    W1, _, _, _ = softabs.w_matrices(st.eig, p, st.alpha)
    return st.grad + 0.5 * st.v_w2() - 0.5 * st.target.contract(st.q, W1)
