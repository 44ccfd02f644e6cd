"""RMHMC chain (Algorithm 1) with the softabs metric.  FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper anchor: Algorithm 1 ((RM)HMC).  Per move: draw p ~ N(0, G(q)), run C
generalized leapfrogs, then a Metropolis-Hastings test.  The printed test
restores the old q exactly when r < exp(H_old - H_new), i.e. on the event
that should *accept*; the standard rule is used here: accept iff
log r < H_old - H_new, otherwise restore q (and its eigen-state).
The momentum draw p = G^{1/2} z = Psi diag(sqrt g) Psi' z (z ~ N(0, I))
realises N(0, G) with the symmetric square root, which depends on G alone
(an eigenvector-based draw Psi diag(sqrt g) z would depend on the signs and
in-cluster rotation of the computed eigenvectors).
The normals z and uniforms r are inputs, drawn by the shared seeded input
generator, so the GPU chain and this reference consume identical randomness.
A failure inside a trajectory (non-finite value, non-positive-definite K)
counts as a rejection.
"""
from __future__ import annotations

import numpy as np

from .hamiltonian import State, hamiltonian
from .integrator import glf_step


def momentum(st, z):
    """p = G^{1/2} z with the symmetric square root Psi diag(sqrt g) Psi'."""
    eig = st.eig
    return eig["Psi"] @ (np.sqrt(eig["g"]) * (eig["Psi"].T @ z))


def run_chain(target, q0, eps, n_leapfrog, n_fixed_point, alpha, z, u):
    """Returns samples (n_moves x D), log posterior per move, accept flags,
    and H_old/H_new per move."""
    n_moves = z.shape[0]
    st = State(target, q0, alpha)
    D = st.q.size
    samples = np.empty((n_moves, D))
    logpost = np.empty(n_moves)
    accepted = np.zeros(n_moves, dtype=np.int32)
    h_old = np.empty(n_moves)
    h_new = np.empty(n_moves)
    for ell in range(n_moves):
        p = momentum(st, z[ell])
        h0 = hamiltonian(st, p)
        ok = True
        try:
            stn, pn = st, p
            for _ in range(n_leapfrog):
                stn, pn = glf_step(stn, pn, eps, n_fixed_point)
            h1 = hamiltonian(stn, pn)
            ok = bool(np.isfinite(h1) and np.all(np.isfinite(stn.q)))
        except (FloatingPointError, np.linalg.LinAlgError):
            ok, h1 = False, np.inf
        h_old[ell], h_new[ell] = h0, h1
        if ok and np.log(u[ell]) < h0 - h1:
            st = stn
            accepted[ell] = 1
        samples[ell] = st.q
        logpost[ell] = -st.U
    return samples, logpost, accepted, h_old, h_new
