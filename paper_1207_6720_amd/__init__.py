"""MI355X-native FMG-FAS with segmental refinement for the 1D model problem.

The solver is the HIP library ``libfmgsr.so`` (C ABI in ``include/fmgsr.h``);
``fmgsr`` is its Python binding and ``workloads`` generates seeded inputs.
"""
__all__ = ["fmgsr", "workloads"]
