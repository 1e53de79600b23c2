"""The decoder's back half, end to end (oracle; test infrastructure only).

Input, as the paper states the problem (Sec. 7 and Sec. 4): an array of
16-bit quantised coefficients, the image's quantisation tables and the
components' sampling factors; output: interleaved 8-bit RGB (Sec. 4.3,
Fig. 4b and Fig. 5), rows top to bottom, one byte per channel.

Steps, in the order of the decoder path (Sec. 2, Fig. 1):
  1. un-interleave the MCU-order blocks into one block grid per component
     (reading: the interface takes MCU order; the paper's GPU buffer keeps all
     Y blocks, then Cb, then Cr, which is an internal layout choice, Sec. 4);
  2. dequantise (Sec. 2, Sec. 4.1);
  3. 2-D IDCT, columns then rows, +128, clamp (Sec. 4.1, Eqs. 1-2);
  4. crop each component plane to its true size (reading; fixes the edges
     the upsampling filter clamps at);
  5. upsample the chroma planes (Sec. 4.2, Algorithm 1 and readings);
  6. colour conversion (Sec. 4.3, Algorithm 2);
  7. interleave R, G, B and crop to W x H (Sec. 4.3, Fig. 4b, Fig. 5).
"""
from __future__ import annotations

import numpy as np

from .colour import ycc_to_rgb
from .geometry import geometry
from .idct import dequantise, idct_blocks
from .upsample import upsample

SUPPORTED_LUMA = {(1, 1), (2, 1), (2, 2)}


def check_frame(frame: dict) -> dict:
    hs, vs = tuple(frame["h"]), tuple(frame["v"])
    if (hs[0], vs[0]) not in SUPPORTED_LUMA or hs[1:] != (1, 1) or vs[1:] != (1, 1):
        raise ValueError(f"unsupported sampling h={hs} v={vs}")
    if not (1 <= frame["width"] <= 65535 and 1 <= frame["height"] <= 65535):
        raise ValueError("image dimensions must be 1..65535")
    if any(not 0 <= q <= 3 for q in frame["qsel"]):
        raise ValueError("quant table selectors must be 0..3")
    return geometry(frame)


def component_grids(frame: dict, coef: np.ndarray):
    """Step 1: MCU-order int16[n_blocks, 64] -> per component int16[gh, gw, 64]."""
    g = geometry(frame)
    mx, my, bpm = g["mcus_x"], g["mcus_y"], g["blocks_per_mcu"]
    coef = np.asarray(coef).reshape(my, mx, bpm, 64)
    grids = []
    first = 0
    for c in range(3):
        hc, vc = frame["h"][c], frame["v"][c]
        part = coef[:, :, first:first + hc * vc, :].reshape(my, mx, vc, hc, 64)
        grids.append(part.transpose(0, 2, 1, 3, 4).reshape(my * vc, mx * hc, 64))
        first += hc * vc
    return grids


def component_planes(frame: dict, coef: np.ndarray, qt: np.ndarray):
    """Steps 1-4: -> list of cropped uint8 planes [comp_h, comp_w]."""
    g = check_frame(frame)
    grids = component_grids(frame, coef)
    planes = []
    for c in range(3):
        d = dequantise(grids[c], np.asarray(qt)[frame["qsel"][c]])
        s = idct_blocks(d)                                  # [gh, gw, 8, 8]
        gh, gw = s.shape[:2]
        plane = s.transpose(0, 2, 1, 3).reshape(gh * 8, gw * 8)
        planes.append(plane[:g["comp_h"][c], :g["comp_w"][c]])
    return planes


def decode(frame: dict, coef: np.ndarray, qt: np.ndarray, mode: str = "simple") -> np.ndarray:
    """Quantised blocks (MCU order) -> uint8 RGB [H, W, 3]."""
    g = check_frame(frame)
    w, h = frame["width"], frame["height"]
    planes = component_planes(frame, coef, qt)
    full = []
    for c in range(3):
        fh = g["hmax"] // frame["h"][c]
        fv = g["vmax"] // frame["v"][c]
        full.append(upsample(planes[c], fh, fv, mode)[:h, :w])
    return ycc_to_rgb(full[0], full[1], full[2])


def decode_rows(frame: dict, coef: np.ndarray, qt: np.ndarray, mode: str,
                mcu_row0: int, mcu_row1: int) -> np.ndarray:
    """Output pixel rows of MCU rows [mcu_row0, mcu_row1) of the whole-image decode."""
    g = check_frame(frame)
    full = decode(frame, coef, qt, mode)
    y0 = g["mcu_h"] * mcu_row0
    y1 = min(frame["height"], g["mcu_h"] * mcu_row1)
    return full[y0:y1]
