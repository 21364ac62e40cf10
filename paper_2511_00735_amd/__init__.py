"""MI355X-native HPS-as-multigrid Helmholtz solver.

Importing the package is cheap: the HIP library (``_lib/libhps.so``) is loaded
only when ``paper_2511_00735_amd.hps`` is imported, and that import fails
loudly when the library is missing.  ``workloads`` holds the seeded problem
generators and is importable without a GPU.
"""
__all__ = ["workloads"]
