"""MI355X-native learned finite-temperature Fermi-operator expansion (arXiv 2605.08523).

The compute path is the HIP library ``libfe.so`` (C ABI in ``include/fe.h``); ``api`` is its
Python binding, ``models`` the coefficient bank and ``workloads`` the seeded synthetic inputs.
"""
from . import models, workloads  # noqa: F401

__all__ = ["api", "models", "workloads"]


def __getattr__(name):
    if name == "api":
        import importlib
        return importlib.import_module(__name__ + ".api")
    raise AttributeError(name)
