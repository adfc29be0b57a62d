"""MI355X-native (gfx950, FP64) well-balanced fifth-order finite-difference HWENO solver for the
shallow water equations (Zhao & Zhang, arXiv 2208.01260).

The numerical work runs in the HIP kernels of ``libswe_hweno.so`` behind the C ABI of
``include/swe_hweno.h``; ``Solver`` (in ``solver``) is a thin torch-tensor front end and
``inputs`` builds the seeded synthetic workloads. Submodules are imported lazily so that the
input generators are usable without a GPU.
"""

__all__ = ["inputs", "solver", "build"]
