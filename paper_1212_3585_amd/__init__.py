"""MI355X-native one-step ADER-WENO hot path (HIP kernels behind a C ABI).

Importing the package loads nothing; ``paper_1212_3585_amd.ader`` loads the
shared library and fails loudly when it has not been built.
"""
__all__ = ["ader", "workloads"]
