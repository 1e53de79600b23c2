"""Encoder side of the synthetic workloads: RGB pixels -> quantised int16 blocks.

This produces the decoder's inputs (coefficient blocks in MCU order, quant
tables, frame description).  None of it is decoder arithmetic:

* RGB -> YCbCr with the JFIF forward equations in FP64, rounded half up and
  clamped to 0..255;
* every plane padded to whole MCUs by edge replication;
* chroma downsampled by the rounded-half-up mean of each 2x1 / 2x2 group;
* level shift by -128 and the forward DCT of T.81 (A.3.3) in FP64;
* quantisation c = sign(F) * floor(|F| / Q + 1/2).

Block order at the output is MCU order: MCUs in raster order, and inside an
MCU the luma blocks (v rows x h columns, raster), then one Cb and one Cr
block.  Each block is 64 int16 in natural order, index 8*row + col, where the
row is the vertical frequency.
"""
from __future__ import annotations

import math

import numpy as np

from .tables import quant_tables

SAMPLINGS = {
    "444": (1, 1),
    "422": (2, 1),
    "420": (2, 2),
}


def make_frame(width: int, height: int, sampling: str) -> dict:
    hy, vy = SAMPLINGS[sampling]
    return {"width": int(width), "height": int(height),
            "h": (hy, 1, 1), "v": (vy, 1, 1), "qsel": (0, 1, 1)}


def mcu_grid(frame: dict):
    hmax, vmax = max(frame["h"]), max(frame["v"])
    mx = -(-frame["width"] // (8 * hmax))
    my = -(-frame["height"] // (8 * vmax))
    return mx, my


def _round_half_up(x: np.ndarray) -> np.ndarray:
    return np.floor(x + 0.5)


def rgb_to_ycbcr(rgb: np.ndarray) -> np.ndarray:
    f = rgb.astype(np.float64)
    r, g, b = f[..., 0], f[..., 1], f[..., 2]
    y = 0.299 * r + 0.587 * g + 0.114 * b
    cb = -0.168736 * r - 0.331264 * g + 0.5 * b + 128.0
    cr = 0.5 * r - 0.418688 * g - 0.081312 * b + 128.0
    out = np.stack([y, cb, cr], axis=-1)
    return np.clip(_round_half_up(out), 0, 255).astype(np.int64)


def _pad_edge(plane: np.ndarray, ph: int, pw: int) -> np.ndarray:
    h, w = plane.shape
    return np.pad(plane, ((0, ph - h), (0, pw - w)), mode="edge")


def _downsample(plane: np.ndarray, fh: int, fv: int) -> np.ndarray:
    if fh == 1 and fv == 1:
        return plane
    h, w = plane.shape
    s = plane.reshape(h // fv, fv, w // fh, fh).sum(axis=(1, 3))
    n = fh * fv
    return (s + n // 2) // n


def _dct_matrix() -> np.ndarray:
    m = np.empty((8, 8), dtype=np.float64)
    for k in range(8):
        ck = math.sqrt(0.5) if k == 0 else 1.0
        for n in range(8):
            m[k, n] = 0.5 * ck * math.cos((2 * n + 1) * k * math.pi / 16.0)
    return m


_D = _dct_matrix()


def fdct_blocks(samples: np.ndarray) -> np.ndarray:
    """FP64 forward DCT of level-shifted 8x8 blocks; samples[..., 8, 8] in 0..255."""
    f = samples.astype(np.float64) - 128.0
    return np.einsum("vy,...yx,ux->...vu", _D, f, _D, optimize=True)


def quantise(coefs: np.ndarray, q: np.ndarray) -> np.ndarray:
    qq = q.reshape(8, 8).astype(np.float64)
    c = np.sign(coefs) * np.floor(np.abs(coefs) / qq + 0.5)
    return c.astype(np.int16)


def plane_to_blocks(plane: np.ndarray) -> np.ndarray:
    h, w = plane.shape
    return plane.reshape(h // 8, 8, w // 8, 8).transpose(0, 2, 1, 3)


def interleave_mcu(frame: dict, grids) -> np.ndarray:
    """grids[c]: int16[by, bx, 64] per component -> int16[n_blocks, 64] MCU order."""
    mx, my = mcu_grid(frame)
    parts = []
    for c, g in enumerate(grids):
        hc, vc = frame["h"][c], frame["v"][c]
        g = g.reshape(my, vc, mx, hc, 64).transpose(0, 2, 1, 3, 4)
        parts.append(g.reshape(my, mx, vc * hc, 64))
    return np.concatenate(parts, axis=2).reshape(-1, 64)


def encode_planes(frame: dict, ycc: np.ndarray, qt: np.ndarray) -> np.ndarray:
    """YCbCr int planes [H, W, 3] -> quantised blocks in MCU order."""
    mx, my = mcu_grid(frame)
    hmax, vmax = max(frame["h"]), max(frame["v"])
    pw, ph = mx * 8 * hmax, my * 8 * vmax
    grids = []
    for c in range(3):
        plane = _pad_edge(ycc[:, :, c], ph, pw)
        plane = _downsample(plane, hmax // frame["h"][c], vmax // frame["v"][c])
        blocks = plane_to_blocks(plane)
        coefs = fdct_blocks(blocks)
        qc = quantise(coefs, qt[frame["qsel"][c]])
        grids.append(qc.reshape(qc.shape[0], qc.shape[1], 64))
    return interleave_mcu(frame, grids)


def encode_rgb(rgb: np.ndarray, sampling: str, quality: int):
    """-> (frame, coef int16[n_blocks, 64], qt uint16[4, 64])."""
    h, w, _ = rgb.shape
    frame = make_frame(w, h, sampling)
    qt = quant_tables(quality)
    coef = encode_planes(frame, rgb_to_ycbcr(rgb), qt)
    return frame, coef, qt
