"""camg: classical AMG-preconditioned CG for sparse SPD systems on AMD MI355X.

The solver itself is the HIP library libcamg.so (C-ABI in include/camg.h);
``camg`` is its ctypes binding and ``problems`` builds seeded synthetic test
matrices.
"""
from . import problems  # noqa: F401

__all__ = ["problems", "camg"]
