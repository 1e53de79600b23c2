"""Pins for the oracle's chroma upsampling (Sec. 4.2, Algorithm 1) and colour
conversion (Sec. 4.3, Algorithm 2)."""
import os

import numpy as np

from oracle.colour import ycc_to_rgb
from oracle.upsample import fancy_h2v1, fancy_h2v2, simple, upsample

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_alg1():
    rows = []
    with open(os.path.join(GOLDEN, "alg1_h2v1.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            a, b = line.split("|")
            rows.append(([int(v) for v in a.split(":")[1].split()],
                         [int(v) for v in b.split(":")[1].split()]))
    return rows


def test_algorithm1_worked_rows():
    for inp, out in load_alg1():
        got = fancy_h2v1(np.array([inp]))[0]
        assert got.tolist() == out


def test_fancy_h2v1_whole_row_spans_blocks():
    # a 16-sample row (two blocks): the filter crosses the block edge and only
    # the true row ends copy their input
    rng = np.random.default_rng(0)
    c = rng.integers(0, 256, size=(3, 16))
    out = fancy_h2v1(c)
    assert np.array_equal(out[:, 0], c[:, 0])
    assert np.array_equal(out[:, -1], c[:, -1])
    # output 16 (even, k = 8) reads In[7] across the block edge
    assert np.array_equal(out[:, 16], (3 * c[:, 8] + c[:, 7] + 1) // 4)


def test_constant_planes_stay_constant():
    for v in (0, 1, 77, 128, 254, 255):
        c = np.full((5, 7), v)
        assert np.all(fancy_h2v1(c) == v)
        assert np.all(fancy_h2v2(c) == v)
        assert np.all(simple(c, 2, 2) == v)


def test_fancy_h2v2_separable_on_vertical_ramp():
    # rows r*16 (constant along x): horizontal pass must leave the vertical
    # triangle result, (3*C[r] + C[r+-1]) * 4 + bias >> 4
    c = np.repeat((np.arange(6) * 16)[:, None], 5, axis=1)
    out = fancy_h2v2(c)
    for r in range(6):
        up = c[max(r - 1, 0), 0]
        dn = c[min(r + 1, 5), 0]
        s_even = 3 * c[r, 0] + up
        s_odd = 3 * c[r, 0] + dn
        assert np.all(out[2 * r, 0::2] == (4 * s_even + 8) >> 4)
        assert np.all(out[2 * r, 1::2] == (4 * s_even + 7) >> 4)
        assert np.all(out[2 * r + 1, 0::2] == (4 * s_odd + 8) >> 4)


def test_fancy_h2v2_interpolates_within_rounding():
    # on a bilinear ramp, interior outputs equal the real triangle filter
    # value up to the final rounding
    y, x = np.mgrid[0:8, 0:8]
    c = 10 + 7 * x + 5 * y
    out = fancy_h2v2(c)
    for oy in range(2, 14):
        for ox in range(2, 14):
            ry = (oy - 0.5) / 2.0
            rx = (ox - 0.5) / 2.0
            exact = 10 + 7 * rx + 5 * ry
            assert abs(out[oy, ox] - exact) <= 0.5 + 1e-9


def test_upsample_identity_for_full_resolution():
    c = np.arange(12).reshape(3, 4)
    assert np.array_equal(upsample(c, 1, 1, "fancy"), c)


def test_colour_exhaustive_within_one_of_fp64():
    """All 2^24 (Y, Cb, Cr) triples against Algorithm 2 in FP64, rounded and clamped."""
    y = np.arange(256, dtype=np.int64)
    worst = 0
    mism = 0
    for cb in range(256):
        cr = np.arange(256, dtype=np.int64)[:, None]
        yy = y[None, :]
        got = ycc_to_rgb(yy + 0 * cr, np.full_like(yy + 0 * cr, cb), cr + 0 * yy).astype(np.int64)
        r = yy + 1.402 * (cr - 128)
        g = yy - 0.34414 * (cb - 128) - 0.71414 * (cr - 128)
        b = yy + 1.772 * (cb - 128) + 0 * cr
        ref = np.clip(np.floor(np.stack([r, g, b], -1) + 0.5), 0, 255)
        d = np.abs(got - ref)
        worst = max(worst, d.max())
        mism += int((d > 0).sum())
    assert worst <= 1
    # the fixed-point terms differ from the real formula only near rounding ties
    assert mism < 0.02 * 3 * (1 << 24)


def test_colour_neutral_chroma_is_grey():
    y = np.arange(256)
    rgb = ycc_to_rgb(y, np.full(256, 128), np.full(256, 128))
    assert np.array_equal(rgb[:, 0], y) and np.array_equal(rgb[:, 1], y) and np.array_equal(rgb[:, 2], y)


def test_colour_saturates():
    # extreme chroma drives R and B past 255 / below 0: both clamp
    hi = ycc_to_rgb(np.array([255]), np.array([255]), np.array([255]))[0]
    lo = ycc_to_rgb(np.array([0]), np.array([0]), np.array([0]))[0]
    assert hi[0] == 255 and hi[2] == 255
    assert lo[0] == 0 and lo[2] == 0
    # G: 255 - 0.34414*127 - 0.71414*127 = 120.6 -> fixed point rounds to 121
    assert hi[1] == 121
    # 0 + 0.34414*128 + 0.71414*128 = 135.5 -> 135 or 136 within rounding
    assert lo[1] in (135, 136)
    assert ycc_to_rgb(np.array([200]), np.array([128]), np.array([255]))[0, 0] == 255
    assert ycc_to_rgb(np.array([50]), np.array([128]), np.array([0]))[0, 0] == 0
