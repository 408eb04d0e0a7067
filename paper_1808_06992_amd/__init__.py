"""UoI_LASSO / UoI_VAR on MI355X (gfx950): hand-written HIP kernels behind a C ABI.

Importing the package loads nothing; ``paper_1808_06992_amd.api`` (the ctypes
binding of libuoi.so) is imported on first use and raises if the library has
not been built.  ``synth`` holds the seeded synthetic workloads.
"""
from . import synth  # noqa: F401

__all__ = ["synth", "api"]


def __getattr__(name):
    if name == "api":
        from . import _lib
        return _lib
    raise AttributeError(name)
