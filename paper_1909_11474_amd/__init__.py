"""MI355X (gfx950) library for batched minimal-Tersoff evaluation and GA fitting.

The compute path is the HIP library libmt_tersoff.so (C ABI in
include/mt_tersoff.h); ``api`` is its Python binding, ``ga`` the genetic
algorithm driver that calls it.  Submodules load lazily so that the package can
be imported to build the library on a machine without a GPU.
"""
__all__ = ["api", "ga", "build"]


def __getattr__(name):
    if name in ("api", "ga", "build", "_lib"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
