"""Quantisation tables for the synthetic workloads.

The base tables are the example luminance and chrominance tables of the JPEG
standard (ITU-T T.81, Annex K.1), in natural (row-major) order.  Workloads
that say "quality q" scale them with the IJG rule: scale s = 5000/q for
q < 50, else 200 - 2q; entry = clamp(floor((base * s + 50) / 100), 1, 255).
These tables are inputs to the decoder, not part of its arithmetic.
"""
from __future__ import annotations

import numpy as np

ANNEX_K_LUMA = np.array([
    16, 11, 10, 16, 24, 40, 51, 61,
    12, 12, 14, 19, 26, 58, 60, 55,
    14, 13, 16, 24, 40, 57, 69, 56,
    14, 17, 22, 29, 51, 87, 80, 62,
    18, 22, 37, 56, 68, 109, 103, 77,
    24, 35, 55, 64, 81, 104, 113, 92,
    49, 64, 78, 87, 103, 121, 120, 101,
    72, 92, 95, 98, 112, 100, 103, 99,
], dtype=np.int64)

ANNEX_K_CHROMA = np.array([
    17, 18, 24, 47, 99, 99, 99, 99,
    18, 21, 26, 66, 99, 99, 99, 99,
    24, 26, 56, 99, 99, 99, 99, 99,
    47, 66, 99, 99, 99, 99, 99, 99,
    99, 99, 99, 99, 99, 99, 99, 99,
    99, 99, 99, 99, 99, 99, 99, 99,
    99, 99, 99, 99, 99, 99, 99, 99,
    99, 99, 99, 99, 99, 99, 99, 99,
], dtype=np.int64)


def quality_scale(quality: int) -> int:
    if not 1 <= quality <= 100:
        raise ValueError(f"quality {quality} outside 1..100")
    return 5000 // quality if quality < 50 else 200 - 2 * quality


def scaled_table(base: np.ndarray, quality: int) -> np.ndarray:
    s = quality_scale(quality)
    q = (base * s + 50) // 100
    return np.clip(q, 1, 255).astype(np.uint16)


def quant_tables(quality: int) -> np.ndarray:
    """uint16[4][64] natural order: slot 0 luma, slot 1 chroma, slots 2-3 all ones."""
    qt = np.ones((4, 64), dtype=np.uint16)
    qt[0] = scaled_table(ANNEX_K_LUMA, quality)
    qt[1] = scaled_table(ANNEX_K_CHROMA, quality)
    return qt


def zigzag_order() -> np.ndarray:
    """zz[i] = natural index (8*row + col) of the i-th coefficient in zig-zag order.

    Built by walking the anti-diagonals r + c = s, alternating direction
    (T.81 Figure 5)."""
    out = []
    for s in range(15):
        cells = [(r, s - r) for r in range(8) if 0 <= s - r < 8]
        if s % 2 == 0:  # even diagonals run bottom-left -> top-right
            cells.reverse()
        out.extend(8 * r + c for r, c in cells)
    return np.array(out, dtype=np.int64)
