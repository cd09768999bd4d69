"""MI355X-native CTIS EM reconstruction (HIP kernels behind a C ABI).

The binding (``Plan`` and friends, in ``ctis``) is imported lazily so that
importing the seeded workload generators does not load the HIP library.
"""
import importlib

__all__ = ["Plan", "CtisError", "PlanInfo", "load_library"]


def __getattr__(name):
    if name in __all__:
        return getattr(importlib.import_module(".ctis", __name__), name)
    raise AttributeError(name)
