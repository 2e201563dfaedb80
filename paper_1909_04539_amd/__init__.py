"""Shared-LHS batched tridiagonal / pentadiagonal solvers for MI355X (gfx950).

The solver itself is the C-ABI library ``libsbs.so`` built from ``csrc/``;
``paper_1909_04539_amd.sbs`` is its thin ctypes binding and
``paper_1909_04539_amd.workloads`` holds the seeded input generators.
Nothing is imported eagerly so that the generators can be used without
loading the GPU library.
"""
__all__ = ["sbs", "workloads"]
