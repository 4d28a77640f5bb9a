"""MI355X-native radiation hot path of EMMA (Aubert, Deparis & Ocvirk 2015).

The M1 transport + hydrogen thermochemistry step on a uniform periodic grid,
as hand-written HIP kernels for gfx950 behind a C ABI (include/emma_rt.h),
with a thin ctypes/PyTorch binding.
"""
from . import _lib
from .rt import EmmaRT, RTStep, group_constants

__all__ = ["EmmaRT", "RTStep", "group_constants", "_lib"]
