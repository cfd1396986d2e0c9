"""hiz: MI355X-native error-bounded lossy compressor for FP32 3-D fields.

An implementation of the interpolation-based compressor of cuSZ-Hi
(arXiv 2507.11165) as hand-written HIP kernels for gfx950 behind a C ABI
(include/hiz.h); this package holds the HIP sources (csrc/), the build script
and the ctypes binding (hiz.py).
"""
from . import hiz  # noqa: F401
from .hiz import (ABS, REL, CUBIC, LINEAR, MD, SEQ, Context, HizError,  # noqa: F401
                  compress, compress_bound, decompress, inspect, make_params)
