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


SPECS = [(257, 190, "420", 85, 4), (333, 47, "422", 90, 0), (100, 121, "444", 60, 3), (640, 480, "420", 75, 32),
         (1, 1, "420", 80, 0), (17, 300, "422", 70, 1)]


def _streams():
    out = []
    for i, (w, hh, samp, q, ri) in enumerate(SPECS):
        frame, coef, qt = encode.encode_rgb(images.texture_rgb(w, hh, 300 + i, sigma=12), samp, q)
        data = bitstream.write_jpeg(frame, coef, qt, restart_interval=ri)
        f, c, qq = oracle.parse_and_decode(data)
        out.append((w, hh, samp, data, oracle.decode(f, c, qq, "fancy"), oracle.geometry(f)))
    return out


@pytest.fixture(scope="module")
def hetero(M, ctx):
    h = M.Hetero(ctx, max_blocks=640 * 480 * 6 // 256 + 4096, max_pixels=640 * 480, n_threads=4)
    yield h
    h.close()


def _check(out, w, hh, exp):
    o = out.numpy()
    assert np.array_equal(o[:, :3 * w].reshape(hh, w, 3), exp)
    assert np.all(o[:, 3 * w:] == 7)  # the pitch padding is untouched


@pytest.mark.parametrize("scheme", ["sps", "overlap", "pps"])
def test_every_split_matches_oracle(M, hetero, scheme):
    code = {"sps": M.MJD_PART_SPS, "overlap": M.MJD_PART_OVERLAP, "pps": M.MJD_PART_PPS}[scheme]
    for w, hh, samp, data, exp, g in _streams():
        splits = sorted({0, hh} | {hh - min(hh, r * g["mcu_h"]) for r in (1, g["mcus_y"] // 2, g["mcus_y"] - 1)})
        for cpu_rows in splits:
            for chunk in ((0, 1, 3) if scheme == "pps" else (0,)):
                say(f"{w}x{hh} {samp} {scheme} cpu_rows={cpu_rows} chunk={chunk}")
                out = torch.full((hh, 3 * w + 5), 7, dtype=torch.uint8).pin_memory()
                t = hetero.decode(data, out, 3 * w + 5, cpu_rows, code, chunk_mcu_rows=chunk)
                _check(out, w, hh, exp)
                gpu_mcu_rows = -(-(hh - cpu_rows) // g["mcu_h"])
                want = -(-gpu_mcu_rows // chunk) if chunk else min(1, gpu_mcu_rows)
                assert t["chunks"] == want and t["cpu_rows"] == cpu_rows
                assert t["total_s"] > 0
    with pytest.raises(M.MjdError):  # a split inside an MCU row
        hetero.decode(data, out, 3 * w + 5, 3, code)


def _model(M, cpu_rate, gpu_rate):
    """P_cpu and P_gpu linear in the pixels, no dispatch, a small Huffman rate."""
    m = M.mjd_model()
    m.huff_per_pixel.degree = 0
    m.huff_per_pixel.c[0] = 1e-9
    for name, val in (("o_w", 0.0), ("t_kernel", gpu_rate), ("o_r", 0.0), ("p_cpu", cpu_rate), ("t_dispatch", 0.0)):
        p = getattr(m, name)
        p.degree = 2
        p.c[4] = val  # the a*b term
    return m


def test_pps_repartitioning_matches_oracle(M, hetero):
    # a model with a slow GPU hands the last chunk's rows to the CPU, one with
    # a slow CPU keeps them on the GPU; either way the bytes are the oracle's
    for cpu_rate, gpu_rate in ((1e-6, 1.0), (1.0, 1e-6)):
        m = _model(M, cpu_rate, gpu_rate)
        for w, hh, samp, data, exp, g in _streams():
            if g["mcus_y"] < 3:
                continue
            cpu_rows = hh - min(hh, (g["mcus_y"] - 1) * g["mcu_h"])  # one MCU row for the CPU
            say(f"{w}x{hh} {samp} pps repartition cpu_rate={cpu_rate}")
            out = torch.full((hh, 3 * w + 5), 7, dtype=torch.uint8).pin_memory()
            t = hetero.decode(data, out, 3 * w + 5, cpu_rows, M.MJD_PART_PPS, chunk_mcu_rows=1, model=m,
                              huff_threads=4.0)
            _check(out, w, hh, exp)
            assert t["cpu_rows"] in (0, hh) or (hh - t["cpu_rows"]) % g["mcu_h"] == 0
            if cpu_rate < gpu_rate:  # the CPU takes the whole remainder at the last chunk
                assert t["cpu_rows"] > cpu_rows and t["chunks"] == g["mcus_y"] - 2
            else:  # the GPU takes every row, the last chunk two MCU rows
                assert t["cpu_rows"] == 0 and t["chunks"] == g["mcus_y"] - 1
