"""Pipelined BiCGStab with residual replacement on one MI355X (gfx950).

The solver library is ``libpbcgs.so`` (HIP, C ABI in ``include/pbcgs.h``);
this package adds a ctypes/PyTorch binding (``solver``) and the seeded
workload inputs (``inputs``).  Importing the package loads nothing; the
binding loads the library on first use and fails if it is not built.
"""

__all__ = ["solver", "inputs"]


def __getattr__(name):
    if name in ("solver", "inputs", "_lib", "build"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    from . import solver
    if hasattr(solver, name):
        return getattr(solver, name)
    raise AttributeError(name)
