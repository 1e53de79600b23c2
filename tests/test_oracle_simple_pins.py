"""Pins for simple (replicating) chroma upsampling, paper Sec. 4.2.

- Hand-written outputs (tests/golden/simple_replicate.txt) on a non-square,
  non-constant plane for the factors (2,1), (2,2), (1,2) and (4,1), cropped
  to odd sizes: a swapped or wrong factor changes the shape or the values.
- Whole decodes of DC-only images: every block is a constant (the DC closed
  form, 128 + floor((c q + 4) / 8)), so with simple upsampling each output
  pixel takes the luma of its own 8x8 luma block and the chroma of its own
  MCU.  The expected image is assembled from block indices alone and
  converted by the exhaustively pinned colour oracle; it covers 4:2:0,
  4:2:2, 4:4:4 (main oracle) and h1v2, 4:1:1 (variant oracle), with partial
  MCUs on both edges.
"""
import os

import numpy as np
import pytest

import oracle
import oracle.variants as V
from oracle.upsample import simple, upsample

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "simple_replicate.txt")


def _rows(text):
    return np.array([[int(v) for v in r.split()] for r in text.split(";")], dtype=np.int64)


def load_cases():
    cases = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            head, src, want = line.split("|")
            fh, fv, cw, ch = (int(v) for v in head.split())
            cases.append((fh, fv, cw, ch, _rows(src), _rows(want)))
    return cases


def test_golden_cases_are_present():
    got = {(c[0], c[1]) for c in load_cases()}
    assert got == {(2, 1), (2, 2), (1, 2), (4, 1)}


@pytest.mark.parametrize("case", load_cases(), ids=lambda c: f"{c[0]}x{c[1]}_{c[2]}x{c[3]}")
def test_simple_matches_hand_written_outputs(case):
    fh, fv, cw, ch, src, want = case
    assert want.shape == (ch, cw)
    got = simple(src, fh, fv)[:ch, :cw]
    assert np.array_equal(got, want)
    # the variant dispatcher takes the same path for every factor
    assert np.array_equal(V.upsample_variant(src, fh, fv, "simple")[:ch, :cw], want)
    if fh <= 2 and fv <= 2 and (fh, fv) != (1, 2):
        assert np.array_equal(upsample(src, fh, fv, "simple")[:ch, :cw], want)


def _dc_only(rng, frame, qdc):
    g = V.variant_geometry(frame)
    coef = np.zeros((g["n_blocks"], 64), np.int16)
    lim = 1024 // qdc
    coef[:, 0] = rng.integers(-lim, lim + 1, g["n_blocks"])
    return coef


def _expected_dc_only(frame, coef, qt):
    """Expected RGB of a DC-only image decoded with simple upsampling,
    from block indices: luma block (y // 8, x // 8) of the luma grid and the
    chroma blocks of MCU (y // mcu_h, x // mcu_w)."""
    g = V.variant_geometry(frame)
    w, h = frame["width"], frame["height"]
    hy, vy = frame["h"][0], frame["v"][0]
    bpm = g["blocks_per_mcu"]
    dc = coef[:, 0].astype(np.int64).reshape(g["mcus_y"], g["mcus_x"], bpm)

    def level(d, sel):
        return np.clip(128 + np.floor_divide(d * int(qt[sel][0]) + 4, 8), 0, 255)

    yy, xx = np.mgrid[0:h, 0:w]
    my, mx = yy // g["mcu_h"], xx // g["mcu_w"]
    # luma block inside its MCU: row (y % mcu_h) // 8, column (x % mcu_w) // 8
    by, bx = (yy % g["mcu_h"]) // 8, (xx % g["mcu_w"]) // 8
    Y = level(dc[my, mx, by * hy + bx], frame["qsel"][0])
    ny = hy * vy
    Cb = level(dc[my, mx, ny], frame["qsel"][1])
    Cr = level(dc[my, mx, ny + 1], frame["qsel"][2])
    return oracle.ycc_to_rgb(Y, Cb, Cr)


@pytest.mark.parametrize("hy,vy", [(2, 2), (2, 1), (1, 1)])
@pytest.mark.parametrize("w,h", [(37, 21), (16, 16), (1, 1), (50, 9)])
def test_dc_only_simple_decode_main_oracle(hy, vy, w, h):
    rng = np.random.default_rng(hy * 100 + vy * 10 + w + h)
    qt = rng.integers(1, 9, (4, 64)).astype(np.uint16)
    frame = {"width": w, "height": h, "h": (hy, 1, 1), "v": (vy, 1, 1), "qsel": (0, 1, 2)}
    coef = _dc_only(rng, frame, int(qt[:3, 0].max()))
    assert np.array_equal(oracle.decode(frame, coef, qt, "simple"), _expected_dc_only(frame, coef, qt))


@pytest.mark.parametrize("hy,vy", [(4, 1), (1, 2), (2, 2), (2, 1)])
@pytest.mark.parametrize("w,h", [(45, 35), (33, 17), (3, 2)])
def test_dc_only_simple_decode_variant_oracle(hy, vy, w, h):
    rng = np.random.default_rng(7 + hy * 100 + vy * 10 + w + h)
    qt = rng.integers(1, 9, (4, 64)).astype(np.uint16)
    frame = {"width": w, "height": h, "h": (hy, 1, 1), "v": (vy, 1, 1), "qsel": (0, 1, 1)}
    coef = _dc_only(rng, frame, int(qt[:2, 0].max()))
    got = V.decode_variant(frame, coef, qt, "islow", "simple")
    assert np.array_equal(got, _expected_dc_only(frame, coef, qt))
    if (hy, vy) == (4, 1):
        # the factor-4 chroma is replicated in both modes
        assert np.array_equal(V.decode_variant(frame, coef, qt, "islow", "fancy"), got)
