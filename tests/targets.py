"""Small analytic sampling targets for integrator and chain pins.

Each target provides derivs(q) -> (U, grad U, Hessian) and contract(q, W) ->
[tr(W dH/dq_i)]_i in closed form, so the reference integrator can be checked
on problems whose answers are known without the GP model.
"""
import numpy as np


class Quadratic:
    """U = 1/2 (q-mu)' A (q-mu): constant Hessian, so dG/dq = 0."""

    def __init__(self, A, mu=None):
        self.A = np.asarray(A, dtype=np.float64)
        self.D = self.A.shape[0]
        self.mu = np.zeros(self.D) if mu is None else np.asarray(mu, dtype=np.float64)

    def derivs(self, q):
        r = q - self.mu
        return 0.5 * r @ self.A @ r, self.A @ r, self.A.copy()

    def contract(self, q, W):
        return np.zeros(self.D)


class Quartic:
    """Separable U = sum(c4 q^4/4 + c2 q^2/2): H = diag(3 c4 q^2 + c2),
    dH/dq_i has the single entry 6 c4 q_i at (i, i), so v(W)_i = 6 c4 q_i W_ii.
    With c2 < 0 the Hessian is indefinite near the origin."""

    def __init__(self, D, c4=1.0, c2=1.0):
        self.D, self.c4, self.c2 = D, c4, c2

    def derivs(self, q):
        U = np.sum(self.c4 * q ** 4 / 4 + self.c2 * q ** 2 / 2)
        return U, self.c4 * q ** 3 + self.c2 * q, np.diag(3 * self.c4 * q ** 2 + self.c2)

    def contract(self, q, W):
        return 6 * self.c4 * q * np.diag(W)
