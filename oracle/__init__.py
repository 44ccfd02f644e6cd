"""Plain FP64 CPU reference ("oracle") for softabs RMHMC on latent-GP models.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never imports, links or calls it, and it
never imports the product path: the two share nothing except the seeded input
generators in ``paper_2511_06407_amd.workloads``.

Every routine follows a passage of Hayakawa & Asai, "Fast Riemannian-manifold
Hamiltonian Monte Carlo for hierarchical Gaussian-process models" (arXiv
2511.06407), cited by section and equation label, and is written for clarity,
not speed: NumPy/LAPACK primitives (matmul, solve, eigh) are the only
building blocks.
"""
from . import model, softabs, hamiltonian, integrator, chain  # noqa: F401
