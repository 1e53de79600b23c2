"""The torch encoder used for the large batch workloads follows the same
recipe as the numpy encoder: on identical YCbCr planes the two give the same
quantised blocks (run here on torch's CPU device)."""
import numpy as np
import pytest

from synth import encode, images

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("w,h,sampling,q", [(37, 29, "420", 75), (70, 33, "422", 90), (41, 50, "444", 55)])
def test_torch_encoder_matches_numpy_encoder(w, h, sampling, q):
    from synth import gpu_encode
    from synth.tables import quant_tables
    rgb = images.gradient_rgb(w, h, 1234 + w, sigma=8.0)
    ycc = encode.rgb_to_ycbcr(rgb)
    frame = encode.make_frame(w, h, sampling)
    qt = quant_tables(q)
    want = encode.encode_planes(frame, ycc, qt)
    t = torch.from_numpy(np.ascontiguousarray(ycc.transpose(2, 0, 1)).astype(np.float64))
    got = gpu_encode.encode_ycc(torch, frame, t, qt, "cpu").numpy()
    assert got.shape == want.shape
    # FP64 sums in another order may flip a rounding tie of the quantiser
    assert np.count_nonzero(got != want) <= 2
    assert np.abs(got.astype(int) - want).max() <= 1


def test_torch_gradient_content_is_seeded():
    from synth import gpu_encode
    a = gpu_encode.gradient_ycc(torch, 40, 24, 7, 8.0, "cpu")
    b = gpu_encode.gradient_ycc(torch, 40, 24, 7, 8.0, "cpu")
    c = gpu_encode.gradient_ycc(torch, 40, 24, 8, 8.0, "cpu")
    assert torch.equal(a, b) and not torch.equal(a, c)
    assert float(a.min()) >= 0 and float(a.max()) <= 255
