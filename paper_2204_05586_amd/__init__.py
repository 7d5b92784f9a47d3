"""MI355X-native solver for spin-1/2 and spin-1 time-dependent Schroedinger
equations (method of arXiv:2204.05586: CF4 Magnus steps, Lie-Trotter
exponentiator with residual squaring, per-interval rotating frame, ordered
product of interval operators).

The compute path is the HIP library ``libmss.so`` (C ABI in
``include/mss.h``); ``native`` is its ctypes binding and ``Simulator`` the
paper-style front end.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads", "native", "Simulator", "Results"]


def __getattr__(name):
    import importlib
    if name == "native":
        return importlib.import_module(__name__ + ".native")
    if name in ("Simulator", "Results"):
        return getattr(importlib.import_module(__name__ + ".simulator"), name)
    raise AttributeError(name)
