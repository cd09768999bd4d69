"""MI355X-native CTIS EM reconstruction (HIP kernels behind a C ABI).

The binding (``Plan`` and friends) is imported lazily so that importing the
seeded workload generators does not load the HIP library.
"""
__all__ = ["Plan", "CtisError", "load_library", "workloads"]


def __getattr__(name):
    if name in ("Plan", "CtisError", "load_library", "PlanInfo"):
        from . import ctis
        return getattr(ctis, name)
    if name == "workloads":
        from . import workloads
        return workloads
    raise AttributeError(name)
