"""YCbCr -> RGB colour conversion (oracle; test infrastructure only).

Paper Sec. 4.3, Algorithm 2: R = Y + 1.402 (Cr-128),
G = Y - 0.34414 (Cb-128) - 0.71414 (Cr-128), B = Y + 1.772 (Cb-128).
Reading (the paper gives only the real-valued formula): each constant is
taken to 16 fraction bits, K = round(k * 2^16) from the paper's printed
digits; each chroma term is rounded once, (sum + 2^15) >> 16 with an
arithmetic shift; the result is added to Y and clamped to 0..255.
"""
from __future__ import annotations

import numpy as np

SCALE_BITS = 16


def _k(x: float) -> int:
    return int(round(x * (1 << SCALE_BITS)))


K_CR_R = _k(1.402)
K_CB_G = _k(0.34414)
K_CR_G = _k(0.71414)
K_CB_B = _k(1.772)
_HALF = 1 << (SCALE_BITS - 1)


def ycc_to_rgb(y, cb, cr) -> np.ndarray:
    """Integer planes (any matching shapes) -> uint8[..., 3]."""
    y = np.asarray(y, dtype=np.int64)
    xb = np.asarray(cb, dtype=np.int64) - 128
    xr = np.asarray(cr, dtype=np.int64) - 128
    r = y + ((K_CR_R * xr + _HALF) >> SCALE_BITS)
    g = y + ((-K_CB_G * xb - K_CR_G * xr + _HALF) >> SCALE_BITS)
    b = y + ((K_CB_B * xb + _HALF) >> SCALE_BITS)
    return np.clip(np.stack([r, g, b], axis=-1), 0, 255).astype(np.uint8)
