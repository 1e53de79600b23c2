"""GPU parity of the CPU-GPU partitioned decode (paper Sec. 5.2): every
split of an image between the GPU (first MCU rows) and the host threads
(the rest), under both schemes, gives the oracle's bytes."""
import numpy as np
import pytest

import oracle
from synth import bitstream, encode, images

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-hetero] {msg}", flush=True)


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1311_5304_amd as mod
    return mod


@pytest.fixture(scope="module")
def ctx(M):
    c = M.Context(0)
    yield c
    c.close()


SPECS = [(257, 190, "420", 85, 4), (333, 47, "422", 90, 0), (100, 121, "444", 60, 3), (640, 480, "420", 75, 32)]


@pytest.mark.parametrize("scheme", ["sps", "pps"])
def test_every_split_matches_oracle(M, ctx, scheme):
    code = M.MJD_PART_SPS if scheme == "sps" else M.MJD_PART_PPS
    h = M.Hetero(ctx, max_blocks=640 * 480 * 6 // 256 + 4096, max_pixels=640 * 480, n_threads=4)
    try:
        for i, (w, hh, samp, q, ri) in enumerate(SPECS):
            frame, coef, qt = encode.encode_rgb(images.texture_rgb(w, hh, 300 + i, sigma=12), samp, q)
            data = bitstream.write_jpeg(frame, coef, qt, restart_interval=ri)
            f, c, qq = oracle.parse_and_decode(data)
            exp = oracle.decode(f, c, qq, "fancy")
            g = oracle.geometry(f)
            splits = sorted({0, hh} | {hh - min(hh, r * g["mcu_h"]) for r in (1, g["mcus_y"] // 2, g["mcus_y"] - 1)})
            for cpu_rows in splits:
                say(f"{w}x{hh} {samp} {scheme} cpu_rows={cpu_rows}")
                out = torch.full((hh, 3 * w + 5), 7, dtype=torch.uint8).pin_memory()
                t = h.decode(data, out, 3 * w + 5, cpu_rows, code)
                o = out.numpy()
                assert np.array_equal(o[:, :3 * w].reshape(hh, w, 3), exp), (w, hh, cpu_rows)
                assert np.all(o[:, 3 * w:] == 7)
                assert t["total_s"] > 0
        with pytest.raises(M.MjdError):  # a split inside an MCU row
            h.decode(data, out, 3 * w + 5, 3, code)
    finally:
        h.close()
