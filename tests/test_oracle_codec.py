"""Whole-decode pins for the oracle: round trips with closed-form answers, the
baseline Huffman codec, and an independent libjpeg-turbo build (through
Pillow) run as a black box on the project's own bitstreams."""
import io

import numpy as np
import pytest

import oracle
from oracle.geometry import geometry
from synth import bitstream, encode, images
from synth.tables import quant_tables
from tests.conftest import requires_pillow


def test_geometry_small_cases():
    for samp, (mw, mh) in (("444", (8, 8)), ("422", (16, 8)), ("420", (16, 16))):
        for w in range(1, 41):
            for h in (1, 7, 8, 9, 16, 17, 33):
                g = geometry(encode.make_frame(w, h, samp))
                assert (g["mcu_w"], g["mcu_h"]) == (mw, mh)
                assert g["mcus_x"] == -(-w // mw) and g["mcus_y"] == -(-h // mh)
                assert g["comp_w"][0] == w and g["comp_h"][0] == h
                assert g["comp_w"][1] == -(-w // (mw // 8))
                assert g["comp_h"][1] == -(-h // (mh // 8))
                assert g["n_blocks"] == g["mcus_x"] * g["mcus_y"] * (mw * mh // 64 + 2)


def test_fig4_block_order_to_pixel_order():
    """Fig. 4: a 16x8 image is stored as two 8x8 blocks (block order) and
    leaves colour conversion as pixel rows one image width apart."""
    frame = encode.make_frame(16, 8, "444")
    qt = np.ones((4, 64), dtype=np.uint16)
    coef = np.zeros((6, 64), dtype=np.int16)      # 2 MCUs x (Y, Cb, Cr)
    coef[0, 0] = -800                             # left Y block dark
    coef[3, 0] = 800                              # right Y block bright
    rgb = oracle.decode(frame, coef, qt)
    assert rgb.shape == (8, 16, 3)
    assert np.all(rgb[:, :8] == 128 - 100) and np.all(rgb[:, 8:] == 128 + 100)


def test_flat_images_round_trip_exactly():
    # a flat level-k block has DC exactly 8(k-128) and zero AC; with Q_DC <= 8
    # the decoder returns k exactly (128 + floor((d+4)/8) with |d - 8(k-128)| <= 3)
    for qdc in range(1, 9):
        qt = np.full((4, 64), 16, dtype=np.uint16)
        qt[:, 0] = qdc
        for samp in ("444", "422", "420"):
            for k in (0, 1, 77, 128, 200, 255):
                frame = encode.make_frame(24, 20, samp)
                ycc = np.zeros((20, 24, 3), dtype=np.int64)
                ycc[..., 0] = k
                ycc[..., 1] = 255 - k
                ycc[..., 2] = (k * 7) % 256
                coef = encode.encode_planes(frame, ycc, qt)
                planes = oracle.component_planes(frame, coef, qt)
                assert np.all(planes[0] == k)
                assert np.all(planes[1] == 255 - k)
                assert np.all(planes[2] == (k * 7) % 256)


def test_block_aligned_steps_round_trip_exactly():
    rng = np.random.default_rng(7)
    qt = np.full((4, 64), 99, dtype=np.uint16)
    qt[:, 0] = 8
    frame = encode.make_frame(64, 48, "444")
    ycc = np.repeat(np.repeat(rng.integers(0, 256, size=(6, 8, 3)), 8, axis=0), 8, axis=1)
    coef = encode.encode_planes(frame, ycc, qt)
    planes = oracle.component_planes(frame, coef, qt)
    for c in range(3):
        assert np.array_equal(planes[c], ycc[..., c])


@pytest.mark.parametrize("ri", [0, 1, 5])
def test_huffman_round_trip_is_lossless(ri):
    for samp in ("444", "422", "420"):
        rgb = images.texture_rgb(45, 38, 11, sigma=12)
        frame, coef, qt = encode.encode_rgb(rgb, samp, 85)
        data = bitstream.write_jpeg(frame, coef, qt, restart_interval=ri)
        f2, c2, q2 = oracle.parse_and_decode(data)
        assert f2 == frame
        assert np.array_equal(c2, coef)
        assert np.array_equal(q2[:2], qt[:2])


def test_huffman_extreme_values_round_trip():
    # DC differences up to category 11, AC magnitudes up to category 10, long zero runs
    frame = encode.make_frame(16, 8, "444")
    coef = np.zeros((6, 64), dtype=np.int16)
    coef[0, 0], coef[1, 0], coef[2, 0] = 1023, -1024, 0
    coef[3, 0], coef[4, 0], coef[5, 0] = -1024, 1023, 1
    coef[0, 63] = -1023
    coef[1, 17] = 1023
    coef[2, 1:64] = np.arange(1, 64)
    qt = np.ones((4, 64), dtype=np.uint16)
    data = bitstream.write_jpeg(frame, coef, qt)
    _, c2, _ = oracle.parse_and_decode(data)
    assert np.array_equal(c2, coef)


def test_corrupt_stream_is_rejected():
    rgb = images.gradient_rgb(32, 32, 3)
    frame, coef, qt = encode.encode_rgb(rgb, "420", 75)
    data = bytearray(bitstream.write_jpeg(frame, coef, qt, restart_interval=2))
    with pytest.raises(oracle.JpegError):
        oracle.parse_and_decode(bytes(data[:len(data) // 2]))
    # renumber the first restart marker
    i = data.index(b"\xFF\xD0")
    data[i + 1] = 0xD3
    with pytest.raises(oracle.JpegError):
        oracle.parse_and_decode(bytes(data))


@requires_pillow
def test_quant_tables_match_libjpeg_scaling():
    from PIL import Image
    for q in range(1, 101):
        b = io.BytesIO()
        Image.fromarray(np.full((8, 8, 3), 100, np.uint8)).save(b, "JPEG", quality=q)
        b.seek(0)
        pil_q = Image.open(b).quantization
        ours = quant_tables(q)
        # Pillow reports the tables in natural order
        assert list(pil_q[0]) == ours[0].tolist(), q
        assert list(pil_q[1]) == ours[1].tolist(), q


@requires_pillow
@pytest.mark.parametrize("samp", ["444", "422", "420"])
def test_libjpeg_decodes_our_streams_to_the_oracle_bits(samp):
    """The project's bitstreams, decoded by libjpeg-turbo (islow IDCT, fancy
    upsampling, its integer colour converter), agree bit for bit with the
    oracle's fancy decode, including odd sizes and partial MCUs."""
    from PIL import Image
    for (w, h, seed) in ((256, 256, 1), (123, 77, 2), (17, 9, 3), (1, 1, 4), (33, 200, 5), (250, 2, 6)):
        rgb = images.texture_rgb(w, h, seed, sigma=12)
        frame, coef, qt = encode.encode_rgb(rgb, samp, 90)
        data = bitstream.write_jpeg(frame, coef, qt, restart_interval=3)
        pil = np.asarray(Image.open(io.BytesIO(data)).convert("RGB"))
        assert np.array_equal(pil, oracle.decode(frame, coef, qt, "fancy")), (w, h)


@requires_pillow
def test_oracle_reads_libjpeg_written_files():
    from PIL import Image
    rgb = images.texture_rgb(77, 61, 9, sigma=12)
    for sub in (0, 1, 2):   # Pillow: 0 = 4:4:4, 1 = 4:2:2, 2 = 4:2:0
        b = io.BytesIO()
        Image.fromarray(rgb).save(b, "JPEG", quality=80, subsampling=sub)
        data = b.getvalue()
        frame, coef, qt = oracle.parse_and_decode(data)
        pil = np.asarray(Image.open(io.BytesIO(data)).convert("RGB"))
        assert np.array_equal(pil, oracle.decode(frame, coef, qt, "fancy"))


@requires_pillow
def test_dc_only_levels_match_libjpeg():
    """Every reachable level 0..255 through DC-only blocks (Q_DC = 1), so no
    IDCT factorisation is involved; exercises upsampling and colour only."""
    from PIL import Image
    rng = np.random.default_rng(12)
    for samp in ("444", "422", "420"):
        frame = encode.make_frame(37, 29, samp)
        g = geometry(frame)
        coef = np.zeros((g["n_blocks"], 64), dtype=np.int16)
        coef[:, 0] = rng.integers(-1024, 1017, size=g["n_blocks"])
        qt = np.ones((4, 64), dtype=np.uint16)
        data = bitstream.write_jpeg(frame, coef, qt)
        pil = np.asarray(Image.open(io.BytesIO(data)).convert("RGB"))
        assert np.array_equal(pil, oracle.decode(frame, coef, qt, "fancy"))
