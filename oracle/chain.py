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
The normals z and uniforms r of ``run_chain`` are inputs; ``run_seeded_chain``
derives them from (seed, stream_id) with the counter-based generator of
``oracle.rng``, as the device chain does, so both consume identical
randomness.  Algorithm 1 runs A moves and returns the positions after moves
A0 .. A-1 (its burn-in A0).  A failure inside a trajectory (non-finite
value, non-positive-definite K) counts as a rejection.
"""
from __future__ import annotations

import numpy as np

from . import rng
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


def run_seeded_chain(target, q0, eps, n_leapfrog, n_fixed_point, alpha, n_moves, n_burnin,
                     seed, stream_id):
    """Algorithm 1 with A = n_moves moves, of which the first A0 = n_burnin are
    burn-in, and the randomness of (seed, stream_id).  Returns the kept
    samples, log posteriors and accept flags (moves A0 .. A-1) and, for all A
    moves, the accept flags and H_old / H_new."""
    if not 0 <= n_burnin < n_moves:
        raise ValueError("need 0 <= n_burnin < n_moves")
    z, u = rng.chain_randoms(seed, stream_id, n_moves, target.D)
    samples, logpost, accepted, h_old, h_new = run_chain(target, q0, eps, n_leapfrog,
                                                         n_fixed_point, alpha, z, u)
    k = slice(n_burnin, n_moves)
    return samples[k], logpost[k], accepted[k], accepted, h_old, h_new
