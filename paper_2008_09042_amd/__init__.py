"""MI355X-native (gfx950) encoding operator of Maxwell parallel imaging.

The compute path is libmaxwell.so (C ABI in include/maxwell.h, HIP kernels
under csrc/); ``encoding`` wraps it for PyTorch.  Importing this package does
not load the library; constructing a MaxwellPlan does, and raises if it is
missing.
"""
from . import _lib  # noqa: F401


def __getattr__(name):
    if name in ("MaxwellPlan", "MaxwellEncode", "MaxwellDataFidelity"):
        from . import encoding as _op
        return getattr(_op, name)
    raise AttributeError(name)
