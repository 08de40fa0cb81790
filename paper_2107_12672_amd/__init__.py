"""MI355X-native differentiable direct volume rendering (DiffDVR hot path).

The rendering and its adjoint run in the HIP library ``libddvr.so``
(C ABI in include/ddvr.h); :mod:`paper_2107_12672_amd.ddvr` is the ctypes
binding and :mod:`paper_2107_12672_amd.autograd` the PyTorch autograd wrapper.
"""
from . import ddvr  # noqa: F401
from . import autograd  # noqa: F401
