"""MI355X-native softabs Riemannian-manifold HMC for hierarchical GP models.

The compute path lives in the HIP library ``librmhmc.so`` (sources under
``csrc/``); ``rmhmc`` is its thin ctypes binding.  Importing this package does
not load the library: ``from paper_2511_06407_amd import rmhmc`` does, and
fails loudly if it has not been built.
"""
__all__ = ["workloads", "rmhmc", "analysis"]
