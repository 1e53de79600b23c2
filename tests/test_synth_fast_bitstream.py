"""The C++ corpus writer produces the same bytes as the Python JPEG writer."""
import numpy as np
import pytest

from synth import bitstream, encode, fast_bitstream, images, workloads


@pytest.mark.parametrize("samp", ["444", "422", "420"])
@pytest.mark.parametrize("ri", [0, 1, 7, 32])
def test_same_bytes_as_python_writer(samp, ri):
    for (w, h, seed) in ((1, 1, 1), (23, 17, 2), (90, 41, 3)):
        rgb = images.texture_rgb(w, h, seed, sigma=12)
        frame, coef, qt = encode.encode_rgb(rgb, samp, 85)
        assert fast_bitstream.write_jpeg(frame, coef, qt, ri) == bitstream.write_jpeg(frame, coef, qt, ri)


def test_same_bytes_on_extreme_and_random_blocks():
    frame = encode.make_frame(40, 24, "420")
    coef = workloads.random_coefficients(frame, seed=5, scale=300.0, density=0.6)
    coef[3, 1:64] = 0
    coef[3, 63] = -1023          # a long zero run before the last coefficient
    qt = np.ones((4, 64), dtype=np.uint16)
    for ri in (0, 2):
        assert fast_bitstream.write_jpeg(frame, coef, qt, ri) == bitstream.write_jpeg(frame, coef, qt, ri)
