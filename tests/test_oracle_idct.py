"""Pins for the oracle's dequantisation and fixed-point IDCT (Sec. 4.1, Eqs. 1-2).

Each check compares against something other than the oracle itself: the
closed form of a DC-only block, an FP64 IDCT from scipy, a brute-force FP64
double sum written from the T.81 definition, and an independent libjpeg-turbo
build run as a black box (see test_oracle_codec.py).
"""
import itertools
import math

import numpy as np
import pytest
from scipy.fft import idctn

from oracle.idct import dequantise, idct_blocks, llm_1d
from synth.encode import fdct_blocks, quantise
from synth.tables import quant_tables


def fp64_reference(d):
    """scipy orthonormal 2-D IDCT-II (== T.81's 1/4 C_u C_v normalisation), +128."""
    b = np.asarray(d, dtype=np.float64).reshape(-1, 8, 8)
    return idctn(b, type=2, norm="ortho", axes=(1, 2)) + 128.0


def brute_force(d):
    """T.81 A.3.3 written out: f(y,x) = 1/4 sum_v sum_u C_v C_u F(v,u) cos cos."""
    b = np.asarray(d, dtype=np.float64).reshape(8, 8)
    out = np.zeros((8, 8))
    for y in range(8):
        for x in range(8):
            s = 0.0
            for v in range(8):
                for u in range(8):
                    cv = 1 / math.sqrt(2) if v == 0 else 1.0
                    cu = 1 / math.sqrt(2) if u == 0 else 1.0
                    s += cv * cu * b[v, u] * math.cos((2 * y + 1) * v * math.pi / 16) * \
                        math.cos((2 * x + 1) * u * math.pi / 16)
            out[y, x] = s / 4 + 128
    return out


def rounded_clamped(f):
    return np.clip(np.floor(f + 0.5), 0, 255)


def test_dc_only_closed_form():
    # all-zero AC: pass 1 gives 4*d exactly, pass 2 gives floor((d + 4) / 8)
    d = np.arange(-2048, 2048, dtype=np.int64)
    blocks = np.zeros((d.size, 64), dtype=np.int64)
    blocks[:, 0] = d
    out = idct_blocks(blocks).reshape(d.size, 64).astype(np.int64)
    expect = np.clip(128 + np.floor_divide(d + 4, 8), 0, 255)
    assert np.array_equal(out, np.repeat(expect[:, None], 64, axis=1))


def test_zero_block_is_mid_grey():
    assert np.all(idct_blocks(np.zeros((1, 64))) == 128)


def test_dequantise_is_elementwise_product():
    rng = np.random.default_rng(0)
    c = rng.integers(-1023, 1024, size=(5, 64)).astype(np.int16)
    q = rng.integers(1, 256, size=64).astype(np.uint16)
    d = dequantise(c, q)
    for i in range(5):
        for k in range(64):
            assert d[i, k] == int(c[i, k]) * int(q[k])


def test_brute_force_matches_scipy():
    rng = np.random.default_rng(1)
    for _ in range(4):
        d = rng.integers(-300, 301, size=64)
        assert np.allclose(brute_force(d), fp64_reference(d)[0], atol=1e-9)


@pytest.mark.parametrize("seed", [2, 3])
def test_brute_force_vs_oracle_within_one(seed):
    rng = np.random.default_rng(seed)
    d = np.zeros(64, dtype=np.int64)
    d[0] = rng.integers(-1024, 1024)
    nz = rng.choice(np.arange(1, 64), 12, replace=False)
    d[nz] = rng.integers(-200, 201, size=12)
    ref = rounded_clamped(brute_force(d))
    got = idct_blocks(d[None, :])[0].astype(np.float64)
    assert np.abs(ref - got).max() <= 1


def test_single_nonzero_blocks_within_one_of_fp64():
    # every position, every value in the conforming range |d| <= 1152
    vals = np.arange(-1152, 1153, dtype=np.int64)
    for k in range(64):
        d = np.zeros((vals.size, 64), dtype=np.int64)
        d[:, k] = vals
        ref = rounded_clamped(fp64_reference(d))
        got = idct_blocks(d).reshape(-1, 8, 8).astype(np.float64)
        assert np.abs(ref - got).max() <= 1, f"position {k}"


def test_random_conforming_blocks_within_one_of_fp64():
    rng = np.random.default_rng(4)
    worst = 0
    mismatches = 0
    total = 0
    for q in range(1, 101):
        qt = quant_tables(q)[0]
        px = rng.integers(0, 256, size=(200, 8, 8))
        c = quantise(fdct_blocks(px), qt).reshape(-1, 64)
        d = dequantise(c, qt)
        ref = rounded_clamped(fp64_reference(d))
        got = idct_blocks(d).astype(np.float64)
        diff = np.abs(ref - got)
        worst = max(worst, diff.max())
        mismatches += int((diff > 0).sum())
        total += diff.size
    assert worst <= 1
    # the fixed-point transform should be exact on the vast majority of samples
    assert mismatches / total < 0.05


def test_ieee1180_style_error_statistics():
    """Per-position mean error and mean square error of the fixed-point IDCT
    against the FP64 IDCT on random spatial blocks in [-256, 255] (the IEEE
    1180 input recipe: FDCT, round, clip to +-2048).  The oracle's values are
    reported against the standard's published limits (peak 1, per-position
    MSE 0.06, overall MSE 0.02, per-position mean 0.015, overall mean 0.0015);
    this pins the rounding and constants to a well-behaved transform."""
    rng = np.random.default_rng(1180)
    n = 20000
    px = rng.integers(-256, 256, size=(n, 8, 8)).astype(np.float64) + 128.0
    F = np.clip(np.floor(fdct_blocks(px) + 0.5), -2048, 2047).reshape(n, 64)
    ref = np.floor(idctn(F.reshape(n, 8, 8), type=2, norm="ortho", axes=(1, 2)) + 0.5)
    # compare before the +128 and clamp: remove the level shift and use the
    # clamp-free range of the reference (the oracle clamps to 0..255)
    got = idct_blocks(F).astype(np.float64) - 128.0
    keep = (ref >= -128) & (ref <= 127)
    err = np.where(keep, got - ref, 0.0)
    cnt = keep.sum(axis=0)
    peak = np.abs(err).max()
    pmse = (err ** 2).sum(axis=0) / cnt
    pme = err.sum(axis=0) / cnt
    assert peak <= 1
    assert pmse.max() <= 0.06
    assert (err ** 2).sum() / cnt.sum() <= 0.02
    assert np.abs(pme).max() <= 0.015
    assert abs(err.sum() / cnt.sum()) <= 0.0015


DOMAIN_BOUND = 1173   # |dequantised coefficient| bound that keeps every intermediate in int32


def _vertex_bound_ok(bound):
    """Each LL&M intermediate is linear in its 8 inputs, so its extreme over the
    box |x_k| <= bound sits on one of the 256 sign vertices.  Pass 2 is checked
    on the box of pass-1 output bounds (a safe over-approximation)."""
    pats = np.array(list(itertools.product([-1, 1], repeat=8)), dtype=np.int64)
    try:
        out = llm_1d([pats[:, k] * bound for k in range(8)])
        m = [int(np.abs((o + 1024) >> 11).max()) + 1 for o in out]
        for y in range(8):
            llm_1d([pats[:, k] * m[y] for k in range(8)])
    except OverflowError:
        return False
    return True


def test_int32_domain_bound():
    # conforming 8-bit data: |F| <= 1024 (DC of a block at 0 or 255), so
    # |d| <= 1024 + Q/2 <= 1151 for baseline tables; the safe bound covers it
    assert _vertex_bound_ok(DOMAIN_BOUND)
    assert not _vertex_bound_ok(DOMAIN_BOUND + 1)
    # real worst-case blocks at the bound run through the oracle's own checks
    rng = np.random.default_rng(5)
    k = np.arange(64)
    for _ in range(200):
        idct_blocks((rng.choice([-1, 1], size=64) * DOMAIN_BOUND)[None, :])
    for y in range(8):
        for x in range(8):
            cy = np.cos((2 * y + 1) * (k // 8) * np.pi / 16)
            cx = np.cos((2 * x + 1) * (k % 8) * np.pi / 16)
            d = np.where(cy * cx >= 0, DOMAIN_BOUND, -DOMAIN_BOUND)[None, :]
            idct_blocks(d)
            idct_blocks(-d)
