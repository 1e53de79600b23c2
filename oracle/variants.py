"""Decoder variants (oracle; test infrastructure only).

The paper notes that libjpeg builds its IDCT from AAN 1-D transforms and
picks between integer and float IDCTs (Sec. 2, Sec. 3); its kernels decode
4:4:4 and 4:2:2 and treat the other samplings alike (Sec. 4.2).  This module
defines the variants beside the islow path of `oracle.idct`:

IDCT methods
  "islow"  oracle.idct (LL&M, 13-bit constants);
  "ifast"  the AAN flowgraph in fixed point;
  "float"  the AAN flowgraph in IEEE single precision.

The AAN 1-D IDCT used here is the transpose of the AAN forward DCT
flowgraph (Arai, Agui and Nakajima, 1988; as drawn in Pennebaker and
Mitchell's JPEG book).  The forward graph computes Y = A x with
A = diag(a) C, C the orthonormal 8-point DCT and a(k) = sqrt(8) s(k),
s(0) = 1, s(k) = sqrt(2) cos(k pi / 16).  Hence x = C^T F =
A^T diag(1/a) F, and A^T is the forward graph with its arrows reversed:
butterflies stay butterflies, constant multiplies stay, and branch points
become sums.  The graph's constants are cos(pi/4), cos(3 pi/8),
cos(pi/8) - cos(3 pi/8) and cos(pi/8) + cos(3 pi/8); five multiplies in
all.  The input scale 1/a(u) a(v) of the 2-D transform folds into the
dequantisation multipliers.

Readings (the paper names the methods only):
* ifast: multiplier M(u, v) = (q * A(u, v) + 2^7) >> 8 with
  A(u, v) = round(2^14 / (s(u) s(v))), i.e. q * 2^6 / (s(u) s(v)) with six
  fraction bits and a 2-D gain of 8 left in (2^9 x the sample value);
  graph constants round(c * 2^9); each product shifted right by 9
  (arithmetic, truncating); no descale between the passes; the result is
  ((v + 2^8) >> 9) + 128, clamped to 0..255.  Every intermediate is asserted
  to fit int32; on the input domain |coefficient * q| <= 1155 the largest
  is below 2^30.
* float: multiplier fp32(q / (8 * (s(u) * s(v)))), the fp64 product and
  quotient rounded once to fp32; the coefficient times the multiplier in
  fp32; the graph in fp32, one rounding per operation in the order written
  (sums left to right); constants fp32(c); the result is
  floor(v + 128.5) clamped to 0..255.  s(k) and the constants come from the
  C library's cos (Python's math module).

Scaled decoding (output 1/s of the image in each direction, s in 2, 4, 8;
N = 8 / s) takes each block's top-left N x N coefficients through the
N-point IDCT with the 8-point normalisation, so a constant block keeps its
value:
  x(m, n) = 1/4 sum_{u, v < N} c(u) c(v) F(u, v) cos((2m+1) u pi / 2N) cos((2n+1) v pi / 2N).
Readings: the fixed-point form follows islow (the 1-D transform
x0 * 2^13 + sum_{u >= 1} round(2^13 sqrt(2) cos((2m+1) u pi / 2N)) x_u,
columns then rows, pass 1 descaled by 11 and pass 2 by 18 with rounding,
+128, clamp), whatever the IDCT method of the full-size decode; the output
is ceil(W / s) x ceil(H / s) and component c's plane ceil(W h_c / (hmax s))
wide (likewise in height); upsampling and colour conversion then run at that
size.

Samplings
  luma (h, v) in {(1,1), (2,1), (1,2), (2,2), (4,1)}, chroma 1x1, and
  grayscale (one component, blocks in raster order).
Readings: fancy (1,2) is Algorithm 1's triangle filter turned vertical
(out[2r] = (3 C[r] + C[r-1] + 1) >> 2, out[2r+1] = (3 C[r] + C[r+1] + 2) >> 2,
rows clamped at the true component height); a factor of 4 replicates in
both modes (the triangle filter is defined for a factor of 2).  Grayscale
output is one byte per pixel.
"""
from __future__ import annotations

import math

import numpy as np

from .colour import ycc_to_rgb
from .geometry import ceil_div, geometry
from .idct import dequantise, idct_blocks
from .upsample import fancy_h2v1, fancy_h2v2, simple

VARIANT_LUMA = {(1, 1), (2, 1), (1, 2), (2, 2), (4, 1)}
IDCT_METHODS = ("islow", "ifast", "float")

_INT32_MIN, _INT32_MAX = -(1 << 31), (1 << 31) - 1

S = [1.0] + [math.sqrt(2.0) * math.cos(k * math.pi / 16.0) for k in range(1, 8)]
C_R = math.cos(math.pi / 4.0)
C_5 = math.cos(3.0 * math.pi / 8.0)
C_2 = math.cos(math.pi / 8.0) - math.cos(3.0 * math.pi / 8.0)
C_4 = math.cos(math.pi / 8.0) + math.cos(3.0 * math.pi / 8.0)


def _chk(a):
    a = np.asarray(a)
    if a.size and (a.min() < _INT32_MIN or a.max() > _INT32_MAX):
        raise OverflowError("IDCT intermediate leaves the int32 range")
    return a


def aan_1d(Y, mul, add=lambda a, b: a + b, sub=lambda a, b: a - b):
    """The transposed AAN flowgraph on 8 inputs (frequency order), with the
    arithmetic supplied: mul(v, name) multiplies by constant `name` in
    ("r", "c5", "c2", "c4"); add/sub give the rounding of the float form.
    Returns the 8 outputs (sample order)."""
    y0, y1, y2, y3, y4, y5, y6, y7 = Y
    # even part: the transpose of (t10, t11, t12, t13) -> (Y0, Y4, Y2, Y6)
    t10 = add(y0, y4)
    t11 = sub(y0, y4)
    u = mul(sub(y2, y6), "r")
    t13 = add(add(y2, y6), u)
    e0, e3 = add(t10, t13), sub(t10, t13)
    e1, e2 = add(t11, u), sub(t11, u)
    # odd part: the transpose of the rotation network -> (Y1, Y3, Y5, Y7)
    z13 = add(y5, y3)
    z2 = sub(y5, y3)
    z11 = add(y1, y7)
    z4 = sub(y1, y7)
    a11 = mul(sub(z11, z13), "r")
    t = mul(add(z2, z4), "c5")
    a10 = add(mul(z2, "c2"), t)
    a12 = sub(mul(z4, "c4"), t)
    o4 = a10
    o5 = add(a10, a11)
    o6 = add(a11, a12)
    o7 = add(add(z11, z13), a12)
    return [add(e0, o7), add(e1, o6), add(e2, o5), add(e3, o4),
            sub(e3, o4), sub(e2, o5), sub(e1, o6), sub(e0, o7)]


# ---- ifast ----------------------------------------------------------------------------------
IFAST_FRAC = 6
IFAST_CONST_BITS = 9
IFAST_CONST = {k: round(c * (1 << IFAST_CONST_BITS)) for k, c in (("r", C_R), ("c5", C_5), ("c2", C_2), ("c4", C_4))}
IFAST_SHIFT = IFAST_FRAC + 3


def ifast_multipliers(q: np.ndarray) -> np.ndarray:
    """uint16[64] natural-order table -> int64[64] multipliers M(u, v)."""
    a = np.array([[round((1 << 14) / (S[u] * S[v])) for v in range(8)] for u in range(8)], dtype=np.int64)
    return (np.asarray(q, dtype=np.int64).reshape(8, 8) * a + (1 << (13 - IFAST_FRAC))) >> (14 - IFAST_FRAC)


def _ifast_mul(v, name):
    return _chk(_chk(v * IFAST_CONST[name]) >> IFAST_CONST_BITS)


def _ifast_add(a, b):
    return _chk(a + b)


def _ifast_sub(a, b):
    return _chk(a - b)


def idct_ifast(coef: np.ndarray, q: np.ndarray) -> np.ndarray:
    """int16[..., 64] coefficients, uint16[64] table -> uint8[..., 8, 8]."""
    c = np.asarray(coef, dtype=np.int64)
    shape = c.shape[:-1]
    w = _chk(c.reshape(-1, 8, 8) * ifast_multipliers(q)[None])        # [n, u, v]
    cols = aan_1d([w[:, u, :] for u in range(8)], _ifast_mul, _ifast_add, _ifast_sub)  # y -> [n, v]
    ws = np.stack(cols, axis=1)                                          # [n, y, v]
    rows = aan_1d([ws[:, :, v] for v in range(8)], _ifast_mul, _ifast_add, _ifast_sub)  # x -> [n, y]
    out = np.stack(rows, axis=2)                                         # [n, y, x]
    out = (_chk(out + (1 << (IFAST_SHIFT - 1))) >> IFAST_SHIFT) + 128
    return np.clip(out, 0, 255).astype(np.uint8).reshape(shape + (8, 8))


# ---- float ----------------------------------------------------------------------------------
F32 = np.float32
FLOAT_CONST = {"r": F32(C_R), "c5": F32(C_5), "c2": F32(C_2), "c4": F32(C_4)}


def float_multipliers(q: np.ndarray) -> np.ndarray:
    """uint16[64] table -> float32[8, 8] multipliers."""
    qq = np.asarray(q).reshape(8, 8)
    return np.array([[F32(float(qq[u, v]) / (8.0 * (S[u] * S[v]))) for v in range(8)] for u in range(8)],
                    dtype=np.float32)


def idct_float(coef: np.ndarray, q: np.ndarray) -> np.ndarray:
    c = np.asarray(coef)
    shape = c.shape[:-1]
    w = c.reshape(-1, 8, 8).astype(np.float32) * float_multipliers(q)[None]
    assert w.dtype == np.float32
    mul = lambda v, name: v * FLOAT_CONST[name]  # noqa: E731
    cols = aan_1d([w[:, u, :] for u in range(8)], mul)
    ws = np.stack(cols, axis=1)
    rows = aan_1d([ws[:, :, v] for v in range(8)], mul)
    out = np.stack(rows, axis=2)
    assert out.dtype == np.float32
    out = np.floor(out + F32(128.5))
    return np.clip(out, 0, 255).astype(np.uint8).reshape(shape + (8, 8))


# ---- reduced (scaled) IDCT -------------------------------------------------------------------
SCALES = (1, 2, 4, 8)


def reduced_constants(n: int):
    """K[m][u] = round(2^13 sqrt(2) cos((2m+1) u pi / 2n)) for u >= 1."""
    return [[round((1 << 13) * math.sqrt(2.0) * math.cos((2 * m + 1) * u * math.pi / (2 * n))) for u in range(n)]
            for m in range(n)]


def _reduced_1d(x, K):
    n = len(x)
    return [_chk(sum((K[m][u] * x[u] for u in range(1, n)), _chk(x[0] << 13))) for m in range(n)]


def idct_reduced(coef: np.ndarray, q: np.ndarray, n: int) -> np.ndarray:
    """int16[..., 64], uint16[64] -> uint8[..., n, n] from the top-left n x n
    coefficients."""
    c = np.asarray(coef, dtype=np.int64)
    shape = c.shape[:-1]
    d = (c.reshape(-1, 8, 8) * np.asarray(q, dtype=np.int64).reshape(8, 8))[:, :n, :n]   # [k, u, v]
    K = reduced_constants(n)
    cols = _reduced_1d([d[:, u, :] for u in range(n)], K)                # m -> [k, v]
    ws = np.stack([_chk(_chk(y + (1 << 10)) >> 11) for y in cols], axis=1)  # [k, m, v]
    rows = _reduced_1d([ws[:, :, v] for v in range(n)], K)               # x -> [k, m]
    out = np.stack(rows, axis=2)                                         # [k, m, x]
    out = _chk(out + (1 << 17) + (128 << 18)) >> 18
    return np.clip(out, 0, 255).astype(np.uint8).reshape(shape + (n, n))


def idct(coef: np.ndarray, q: np.ndarray, method: str) -> np.ndarray:
    if method == "islow":
        return idct_blocks(dequantise(coef, q))
    if method == "ifast":
        return idct_ifast(coef, q)
    if method == "float":
        return idct_float(coef, q)
    raise ValueError(f"unknown IDCT method {method!r}")


# ---- frames, planes and the whole decode ----------------------------------------------------

def variant_geometry(frame: dict) -> dict:
    """geometry() for three-component frames; for grayscale (ncomp 1) one
    8x8 block per MCU."""
    if frame.get("ncomp", 3) == 1:
        w, h = int(frame["width"]), int(frame["height"])
        mx, my = ceil_div(w, 8), ceil_div(h, 8)
        return {"hmax": 1, "vmax": 1, "mcu_w": 8, "mcu_h": 8, "mcus_x": mx, "mcus_y": my, "blocks_per_mcu": 1,
                "n_blocks": mx * my, "comp_w": [w], "comp_h": [h], "grid_w": [mx], "grid_h": [my]}
    hs, vs = tuple(frame["h"]), tuple(frame["v"])
    if (hs[0], vs[0]) not in VARIANT_LUMA or hs[1:] != (1, 1) or vs[1:] != (1, 1):
        raise ValueError(f"unsupported sampling h={hs} v={vs}")
    return geometry(frame)


def planes(frame: dict, coef: np.ndarray, qt: np.ndarray, method: str, scale: int = 1):
    """MCU-order blocks -> cropped uint8 component planes (1/scale size)."""
    if scale not in SCALES:
        raise ValueError(f"scale 1/{scale} not supported")
    if scale > 1 and method != "islow":
        raise ValueError("scaled decoding has the islow-style reduced transform only")
    n = 8 // scale
    g = variant_geometry(frame)
    nc = frame.get("ncomp", 3)
    mx, my, bpm = g["mcus_x"], g["mcus_y"], g["blocks_per_mcu"]
    c = np.asarray(coef).reshape(my, mx, bpm, 64)
    out = []
    first = 0
    for k in range(nc):
        hc, vc = (1, 1) if nc == 1 else (frame["h"][k], frame["v"][k])
        part = c[:, :, first:first + hc * vc, :].reshape(my, mx, vc, hc, 64)
        grid = part.transpose(0, 2, 1, 3, 4).reshape(my * vc, mx * hc, 64)
        first += hc * vc
        q = np.asarray(qt)[frame["qsel"][k]]
        s = idct(grid, q, method) if n == 8 else idct_reduced(grid, q, n)   # [gh, gw, n, n]
        gh, gw = s.shape[:2]
        plane = s.transpose(0, 2, 1, 3).reshape(gh * n, gw * n)
        out.append(plane[:ceil_div(g["comp_h"][k], scale), :ceil_div(g["comp_w"][k], scale)])
    return out


def fancy_h1v2(c: np.ndarray) -> np.ndarray:
    """The vertical triangle filter: uint8[h, n] -> int64[2h, n]."""
    c = np.asarray(c, dtype=np.int64)
    up = np.concatenate([c[:1], c[:-1]], axis=0)
    down = np.concatenate([c[1:], c[-1:]], axis=0)
    out = np.empty((2 * c.shape[0], c.shape[1]), dtype=np.int64)
    out[0::2] = (3 * c + up + 1) >> 2
    out[1::2] = (3 * c + down + 2) >> 2
    return out


def upsample_variant(c: np.ndarray, fh: int, fv: int, mode: str) -> np.ndarray:
    if mode not in ("simple", "fancy"):
        raise ValueError(f"unknown upsampling mode {mode!r}")
    if (fh, fv) == (1, 1):
        return np.asarray(c, dtype=np.int64)
    if mode == "simple" or fh == 4:
        return simple(c, fh, fv)
    if (fh, fv) == (2, 1):
        return fancy_h2v1(c)
    if (fh, fv) == (1, 2):
        return fancy_h1v2(c)
    if (fh, fv) == (2, 2):
        return fancy_h2v2(c)
    raise ValueError(f"no filter for factors ({fh}, {fv})")


def decode_variant(frame: dict, coef: np.ndarray, qt: np.ndarray, method: str = "islow",
                   mode: str = "fancy", scale: int = 1) -> np.ndarray:
    """-> uint8[H', W', 3] (YCbCr frames) or uint8[H', W'] (grayscale),
    W' = ceil(W / scale), H' = ceil(H / scale)."""
    g = variant_geometry(frame)
    w, h = ceil_div(frame["width"], scale), ceil_div(frame["height"], scale)
    p = planes(frame, coef, qt, method, scale)
    if frame.get("ncomp", 3) == 1:
        return p[0][:h, :w].astype(np.uint8)
    full = []
    for k in range(3):
        full.append(upsample_variant(p[k], g["hmax"] // frame["h"][k], g["vmax"] // frame["v"][k], mode)[:h, :w])
    return ycc_to_rgb(full[0], full[1], full[2])
