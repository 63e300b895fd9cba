"""MI355X-native HPEZ: error-bounded lossy compression of float32/float64
fields with the auto-tuned multi-component interpolation predictor of Liu et
al. (SIGMOD 2024), as HIP kernels for gfx950 behind a C ABI (include/hpez.h).

    from paper_2311_12133_amd import compress, decompress, tune

The HIP library (libhpez.so) is loaded on first use; there is no CPU
fallback.
"""
from __future__ import annotations


def compress(x, cfg, stream=None, out=None):
    from .binding import compress as _c
    return _c(x, cfg, stream=stream, out=out)


def decompress(stream_t, stream=None, out=None):
    from .binding import decompress as _d
    return _d(stream_t, stream=stream, out=out)


def tune(x, cfg, opts=None, stream=None):
    from .binding import tune as _t
    return _t(x, cfg, opts=opts, stream=stream)


def build():
    from .build import build as _b
    return _b()
