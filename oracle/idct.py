"""Dequantisation and the fixed-point 8x8 inverse DCT (oracle; test infrastructure only).

Paper Sec. 2 and Sec. 4.1: the decoder dequantises each coefficient with the
image's quantisation table right after loading it, then forms the 2-D IDCT
separably: a 1-D IDCT down each of the eight columns (Eq. 1), then a 1-D IDCT
along each of the eight rows of that result (Eq. 2), with C = 1/sqrt(2) for
the zero frequency and 1 otherwise.

Readings where the paper is silent:
* normalisation as in T.81 A.3.3 (overall factor 1/4 * C_u * C_v), followed
  by the +128 level shift and a clamp to 0..255;
* the fixed-point form is the Loeffler-Ligtenberg-Moschytz (LL&M) 8-point
  flowgraph ("islow"), whose 1-D transform is sqrt(8) times the orthonormal
  1-D IDCT, so the zero-frequency path is a pure shift;
* every real constant k is replaced by round(k * 2^13); pass 1 keeps 2 extra
  fraction bits (descale by 13 - 2 = 11), pass 2 descales by 13 + 2 + 3 = 18
  (the +3 removes the 2-D gain of 8 left by two sqrt(8) passes);
* every descale adds half an LSB and shifts right arithmetically.

All arithmetic is in int64 and every intermediate is asserted to fit int32,
which is the domain the fixed-point design assumes.
"""
from __future__ import annotations

import math

import numpy as np

CONST_BITS = 13
PASS1_BITS = 2
PASS1_SHIFT = CONST_BITS - PASS1_BITS           # 11
PASS2_SHIFT = CONST_BITS + PASS1_BITS + 3       # 18

_INT32_MIN, _INT32_MAX = -(1 << 31), (1 << 31) - 1


def _fix(x: float) -> int:
    return int(round(x * (1 << CONST_BITS)))


# a[j] = sqrt(2) * cos(j*pi/16).  The sqrt(8)-scaled 1-D IDCT is
# y[n] = x[0] + sum_{k>=1} sqrt(2) * cos((2n+1)*k*pi/16) * x[k].
_A = [math.sqrt(2.0) * math.cos(j * math.pi / 16.0) for j in range(8)]

# Even part: rotation of (x2, x6) by 3 multiplies.
K_R = _fix(_A[6])                      # common term (x2 + x6) * a6
K_R2 = _fix(_A[2] - _A[6])             # x2 * (a2 - a6)
K_R6 = _fix(_A[2] + _A[6])             # x6 * (a2 + a6)
# Odd part: LL&M's network over the pair sums x7+x1, x5+x3, x7+x3, x5+x1,
# one shared product (x7+x3+x5+x1)*a3, four pair-sum products and four
# single-input products (12 multiplies in all).
K_Z5 = _fix(_A[3])
K_P7 = _fix(-_A[1] + _A[3] + _A[5] - _A[7])
K_P5 = _fix(_A[1] + _A[3] - _A[5] + _A[7])
K_P3 = _fix(_A[1] + _A[3] + _A[5] - _A[7])
K_P1 = _fix(_A[1] + _A[3] - _A[5] - _A[7])
K_Z1 = _fix(_A[3] - _A[7])
K_Z2 = _fix(_A[1] + _A[3])
K_Z3 = _fix(_A[3] + _A[5])
K_Z4 = _fix(_A[3] - _A[5])


def _chk(a):
    a = np.asarray(a)
    if a.size and (a.min() < _INT32_MIN or a.max() > _INT32_MAX):
        raise OverflowError("IDCT intermediate leaves the int32 range")
    return a


def _descale(x, n):
    return _chk(_chk(x + (1 << (n - 1))) >> n)


def llm_1d(x):
    """One LL&M 8-point 1-D IDCT, unscaled (results carry the 2^13 constant scale).

    x: sequence of 8 int64 arrays (frequency index 0..7, all the same shape).
    Returns 8 int64 arrays: sample index 0..7, each = 2^13 * sqrt(8) * IDCT_ortho
    (exactly, given the rounded constants), before any descale."""
    x = [np.asarray(v, dtype=np.int64) for v in x]
    # even part: x0, x4 through pure shifts; x2, x6 through the rotation
    z1 = _chk((x[2] + x[6]) * K_R)
    t2 = _chk(z1 + x[2] * K_R2)          # a2*x2 + a6*x6
    t3 = _chk(z1 - x[6] * K_R6)          # a6*x2 - a2*x6
    t0 = _chk((x[0] + x[4]) << CONST_BITS)
    t1 = _chk((x[0] - x[4]) << CONST_BITS)
    e0, e3 = _chk(t0 + t2), _chk(t0 - t2)
    e1, e2 = _chk(t1 + t3), _chk(t1 - t3)
    # odd part
    s17 = x[7] + x[1]
    s35 = x[5] + x[3]
    s37 = x[7] + x[3]
    s15 = x[5] + x[1]
    z5 = _chk((s37 + s15) * K_Z5)
    p7 = _chk(x[7] * K_P7)
    p5 = _chk(x[5] * K_P5)
    p3 = _chk(x[3] * K_P3)
    p1 = _chk(x[1] * K_P1)
    q17 = _chk(-s17 * K_Z1)
    q35 = _chk(-s35 * K_Z2)
    q37 = _chk(z5 - s37 * K_Z3)
    q15 = _chk(z5 - s15 * K_Z4)
    o0 = _chk(p1 + q17 + q15)
    o1 = _chk(p3 + q35 + q37)
    o2 = _chk(p5 + q35 + q15)
    o3 = _chk(p7 + q17 + q37)
    return [_chk(e0 + o0), _chk(e1 + o1), _chk(e2 + o2), _chk(e3 + o3),
            _chk(e3 - o3), _chk(e2 - o2), _chk(e1 - o1), _chk(e0 - o0)]


def dequantise(coef: np.ndarray, q: np.ndarray) -> np.ndarray:
    """coef int16[..., 64] natural order, q uint16[64] -> int64 products (Sec. 2)."""
    return np.asarray(coef, dtype=np.int64) * np.asarray(q, dtype=np.int64)


def idct_blocks(d: np.ndarray) -> np.ndarray:
    """Dequantised blocks int[..., 64] (natural order, row = vertical frequency)
    -> uint8 samples [..., 8, 8] (row = y, column = x)."""
    d = np.asarray(d, dtype=np.int64)
    shape = d.shape[:-1]
    b = d.reshape(-1, 8, 8)
    # pass 1: column u holds F(u, v) for v = 0..7 (Eq. 1); output rows keep 2 fraction bits
    ws = np.empty_like(b)
    cols = llm_1d([b[:, v, :] for v in range(8)])        # each [n, 8 columns]
    for y in range(8):
        ws[:, y, :] = _descale(cols[y], PASS1_SHIFT)
    # pass 2: each row y of the column results (Eq. 2); remove the gain, level shift, clamp
    out = np.empty(b.shape, dtype=np.int64)
    rows = llm_1d([ws[:, :, u] for u in range(8)])       # each [n, 8 rows]
    for x in range(8):
        out[:, :, x] = _descale(rows[x], PASS2_SHIFT) + 128
    return np.clip(out, 0, 255).astype(np.uint8).reshape(shape + (8, 8))
