"""Windowed regularized LBM-LES solver and discrete adjoint for MI355X.

The solver runs in the HIP library liblbmadj.so (C ABI in include/lbm.h);
this package holds its Python binding (`binding`, `solver`), the autograd
entry point (`autograd.WindowedJ`) and the seeded input generators
(`workloads`, importable without a GPU or the library).
"""

import importlib

__all__ = ["Solver", "WindowedJ", "windowed_objective"]


def __getattr__(name):
    if name == "Solver":
        return importlib.import_module(".solver", __name__).Solver
    if name in ("WindowedJ", "windowed_objective"):
        return getattr(importlib.import_module(".autograd", __name__), name)
    raise AttributeError(name)
