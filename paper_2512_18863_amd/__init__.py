"""MI355X-native differentiable pencil-beam VMAT dose engine (arXiv:2512.18863).

The dose path is a C-ABI library of hand-written HIP kernels for gfx950
(``libpdrt.so``, declared in ``include/pdrt.h``); ``engine`` binds it to
PyTorch device memory and streams.  Importing this package loads nothing:
``engine`` loads the library on first use and raises if it is missing.
"""
__all__ = ["inputs", "engine"]
