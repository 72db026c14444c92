"""MI355X-native Hamilton-Jacobi reachability safe-set solver (libhjr).

The compute path is the C-ABI library ``libhjr.so`` (HIP kernels for gfx950)
wrapped by :mod:`paper_2101_05916_amd.hjr`.  Importing the package does not
load the library; importing ``hjr`` and calling it does, and fails loudly if
the library has not been built.
"""
__all__ = ["hjr", "workloads"]
