"""The back half on host cores (CPU only), the CPU side of the paper's
CPU-GPU partitioning (Sec. 5.2): bit-exact against the oracle for every
sampling and upsampling mode, band by band, for any thread count."""
import numpy as np
import pytest

import oracle
from synth import encode, images, workloads


@pytest.fixture(scope="module")
def M():
    import paper_1311_5304_amd as mod
    return mod


CASES = [(257, 190, "420"), (333, 47, "422"), (100, 121, "444"), (17, 9, "420"), (1, 1, "420"), (16, 16, "420"),
         (200, 33, "422"), (31, 64, "444")]


@pytest.mark.parametrize("mode", ["simple", "fancy"])
@pytest.mark.parametrize("case", CASES)
def test_whole_image_matches_oracle(M, case, mode):
    w, h, samp = case
    frame, coef, qt = encode.encode_rgb(images.texture_rgb(w, h, 5, sigma=12), samp, 85)
    g = M.mjd_geometry_of(frame)
    for nt in (1, 3):
        out = np.zeros((h, w, 3), np.uint8)
        M.mjd_decode_host(frame, coef, qt, M.UPSAMPLE[mode], out, 3 * w, 0, g["mcus_y"], nt)
        assert np.array_equal(out, oracle.decode(frame, coef.reshape(-1, 64), qt, mode))


@pytest.mark.parametrize("samp", ["420", "422", "444"])
def test_bands_write_only_their_rows(M, samp):
    w, h = 190, 101
    frame, coef, qt = encode.encode_rgb(images.gradient_rgb(w, h, 6, sigma=8), samp, 75)
    g = M.mjd_geometry_of(frame)
    full = oracle.decode(frame, coef.reshape(-1, 64), qt, "fancy")
    mh = g["mcu_h"]
    for r0, r1 in ((0, 1), (1, 3), (g["mcus_y"] - 1, g["mcus_y"]), (2, g["mcus_y"])):
        pitch = 3 * w + 7
        out = np.full((h, pitch), 9, np.uint8)
        M.mjd_decode_host(frame, coef, qt, M.MJD_UPSAMPLE_FANCY, out, pitch, r0, r1, 4)
        y0, y1 = r0 * mh, min(h, r1 * mh)
        assert np.array_equal(out[y0:y1, :3 * w].reshape(y1 - y0, w, 3), full[y0:y1])
        assert np.all(out[:y0] == 9) and np.all(out[y1:] == 9) and np.all(out[:, 3 * w:] == 9)


def test_random_coefficients(M):
    for samp in ("420", "422", "444"):
        frame = encode.make_frame(120, 72, samp)
        coef = workloads.random_coefficients(frame, seed=3, scale=20.0, density=0.3)
        qt = np.full((4, 64), 3, np.uint16)
        g = M.mjd_geometry_of(frame)
        for mode in ("simple", "fancy"):
            out = np.zeros((72, 120, 3), np.uint8)
            M.mjd_decode_host(frame, coef, qt, M.UPSAMPLE[mode], out, 360, 0, g["mcus_y"], 2)
            assert np.array_equal(out, oracle.decode(frame, coef.reshape(-1, 64), qt, mode))


def test_argument_errors(M):
    frame, coef, qt = encode.encode_rgb(images.gradient_rgb(16, 16, 1, sigma=8), "420", 75)
    out = np.zeros((16, 16, 3), np.uint8)
    for args, code in (((M.MJD_UPSAMPLE_FANCY, out, 47, 0, 1, 1), -1),   # pitch below 3*width
                       ((M.MJD_UPSAMPLE_FANCY, out, 48, 0, 2, 1), -1),   # rows past the image
                       ((M.MJD_UPSAMPLE_FANCY, out, 48, 0, 1, 0), -1),   # no threads
                       ((7, out, 48, 0, 1, 1), -1)):                     # unknown mode
        with pytest.raises(M.MjdError) as ei:
            M.mjd_decode_host(frame, coef, qt, *args)
        assert ei.value.code == code
