"""Chroma upsampling (oracle; test infrastructure only).

Paper Sec. 4.2, Algorithm 1: the 4:2:2 triangle ("fancy") filter turns a row
of n samples into 2n: out[2k] = (3*In[k] + In[k-1] + 1) / 4,
out[2k+1] = (3*In[k] + In[k+1] + 2) / 4, and the two end outputs copy the
end inputs.  Readings (the paper prints only the one-block case and says the
other samplings are decoded similarly):
* the filter runs over the whole component row; only the true component edge
  (ceil(W*h/hmax) samples) is clamped, i.e. In[-1] = In[0], In[n] = In[n-1],
  which gives Algorithm 1's end copies exactly;
* 4:2:0 (h2v2): first an unrounded vertical triangle sum, S = 3*C[r] + C[r-1]
  for output row 2r and S = 3*C[r] + C[r+1] for row 2r+1 (rows clamped at the
  true component height), then horizontally out[2k] = (3*S[k] + S[k-1] + 8) >> 4
  and out[2k+1] = (3*S[k] + S[k+1] + 7) >> 4;
* "simple" upsampling replicates each sample over its 2x1 or 2x2 group.
"""
from __future__ import annotations

import numpy as np


def _clamped_neighbours(c: np.ndarray, axis: int):
    prev = np.concatenate([np.take(c, [0], axis=axis),
                           np.take(c, np.arange(c.shape[axis] - 1), axis=axis)], axis=axis)
    nxt = np.concatenate([np.take(c, np.arange(1, c.shape[axis]), axis=axis),
                          np.take(c, [c.shape[axis] - 1], axis=axis)], axis=axis)
    return prev, nxt


def _interleave_cols(even: np.ndarray, odd: np.ndarray) -> np.ndarray:
    h, n = even.shape
    out = np.empty((h, 2 * n), dtype=np.int64)
    out[:, 0::2] = even
    out[:, 1::2] = odd
    return out


def _interleave_rows(even: np.ndarray, odd: np.ndarray) -> np.ndarray:
    n, w = even.shape
    out = np.empty((2 * n, w), dtype=np.int64)
    out[0::2] = even
    out[1::2] = odd
    return out


def fancy_h2v1(c: np.ndarray) -> np.ndarray:
    """Algorithm 1 over whole rows: uint8[h, n] -> int64[h, 2n]."""
    c = np.asarray(c, dtype=np.int64)
    prev, nxt = _clamped_neighbours(c, axis=1)
    even = (3 * c + prev + 1) >> 2
    odd = (3 * c + nxt + 2) >> 2
    return _interleave_cols(even, odd)


def fancy_h2v2(c: np.ndarray) -> np.ndarray:
    """Triangle filter in both directions: uint8[h, n] -> int64[2h, 2n]."""
    c = np.asarray(c, dtype=np.int64)
    up, down = _clamped_neighbours(c, axis=0)
    s = _interleave_rows(3 * c + up, 3 * c + down)     # unrounded vertical sums
    prev, nxt = _clamped_neighbours(s, axis=1)
    even = (3 * s + prev + 8) >> 4
    odd = (3 * s + nxt + 7) >> 4
    return _interleave_cols(even, odd)


def simple(c: np.ndarray, fh: int, fv: int) -> np.ndarray:
    c = np.asarray(c, dtype=np.int64)
    return np.repeat(np.repeat(c, fv, axis=0), fh, axis=1)


def upsample(c: np.ndarray, fh: int, fv: int, mode: str) -> np.ndarray:
    """Upsample a cropped component plane by (fh, fv) in {1,2} x {1,2}."""
    if fh == 1 and fv == 1:
        return np.asarray(c, dtype=np.int64)
    if mode == "simple":
        return simple(c, fh, fv)
    if mode != "fancy":
        raise ValueError(f"unknown upsampling mode {mode!r}")
    if (fh, fv) == (2, 1):
        return fancy_h2v1(c)
    if (fh, fv) == (2, 2):
        return fancy_h2v2(c)
    raise ValueError(f"fancy upsampling of factors {(fh, fv)} is not defined here")
