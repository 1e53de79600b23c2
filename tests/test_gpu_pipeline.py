"""GPU tests of the pipelined end-to-end decode: bitstreams in host memory ->
RGB8 in host memory through host entropy workers, three HIP streams and the
fused kernel, bit-exact against the oracle's own reader and decoder."""
import numpy as np
import pytest

import oracle
from synth import bitstream, encode, fast_bitstream, images

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-pipeline] {msg}", flush=True)


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


SPECS = [(257, 190, "420", 85, 32), (64, 64, "420", 75, 0), (333, 47, "422", 90, 3), (100, 121, "444", 60, 1),
         (17, 300, "420", 95, 5), (512, 384, "420", 85, 32), (1, 1, "420", 50, 0), (200, 33, "422", 70, 2)]


@pytest.fixture(scope="module")
def corpus():
    out = []
    for i, (w, h, samp, q, ri) in enumerate(SPECS):
        rgb = images.texture_rgb(w, h, 100 + i, sigma=12)
        frame, coef, qt = encode.encode_rgb(rgb, samp, q)
        out.append((frame, bitstream.write_jpeg(frame, coef, qt, restart_interval=ri)))
    return out


def expected(corpus, mode):
    exp = []
    for frame, jpg in corpus:
        f, c, q = oracle.parse_and_decode(jpg)
        exp.append(oracle.decode(f, c, q, mode))
    return exp


def slot_sizes(corpus):
    blocks = max(oracle.geometry(f)["n_blocks"] for f, _ in corpus)
    pixels = max(f["width"] * f["height"] for f, _ in corpus)
    return blocks, pixels


@pytest.mark.parametrize("mode", ["fancy", "simple"])
def test_pipeline_matches_oracle(M, ctx, corpus, mode):
    exp = expected(corpus, mode)
    blocks, pixels = slot_sizes(corpus)
    for threads, slots, band in ((1, 2, 1), (4, 3, 0), (3, 2, 2), (8, 4, 5)):
        say(f"{mode} threads={threads} slots={slots} band={band}")
        p = M.Pipeline(ctx, threads, blocks, pixels, M.UPSAMPLE[mode], n_slots=slots, band_mcu_rows=band)
        try:
            for rep in range(2):
                outs = [torch.full((f["height"], f["width"], 3), 7, dtype=torch.uint8).pin_memory()
                        for f, _ in corpus]
                st = p.run([j for _, j in corpus], outs)
                assert st["images"] == len(corpus)
                for i, (o, e) in enumerate(zip(outs, exp)):
                    assert np.array_equal(o.numpy(), e), (i, SPECS[i], threads, slots, band, rep)
        finally:
            p.close()


def test_pitch_padding_untouched_and_pageable_outputs(M, ctx, corpus):
    exp = expected(corpus, "fancy")
    blocks, pixels = slot_sizes(corpus)
    p = M.Pipeline(ctx, 2, blocks, pixels, M.MJD_UPSAMPLE_FANCY)
    try:
        outs = [np.full((f["height"], 3 * f["width"] + 13), 9, dtype=np.uint8) for f, _ in corpus]
        p.run([j for _, j in corpus], outs, pitches=[o.shape[1] for o in outs])
        for o, e, (f, _) in zip(outs, exp, corpus):
            w = f["width"]
            assert np.array_equal(o[:, :3 * w].reshape(f["height"], w, 3), e)
            assert np.all(o[:, 3 * w:] == 9)
    finally:
        p.close()


def test_entropy_only_leaves_outputs_alone(M, ctx, corpus):
    blocks, pixels = slot_sizes(corpus)
    p = M.Pipeline(ctx, 3, blocks, pixels, M.MJD_UPSAMPLE_FANCY)
    try:
        outs = [np.full((f["height"], f["width"], 3), 5, dtype=np.uint8) for f, _ in corpus]
        st = p.run([j for _, j in corpus], outs, entropy_only=True)
        assert st["images"] == len(corpus) and st["entropy_ms"] > 0 and st["kernel_ms"] == 0
        assert all(np.all(o == 5) for o in outs)
    finally:
        p.close()


def test_errors_name_the_image_and_the_pipeline_recovers(M, ctx, corpus):
    exp = expected(corpus, "fancy")
    blocks, pixels = slot_sizes(corpus)
    p = M.Pipeline(ctx, 2, blocks, pixels, M.MJD_UPSAMPLE_FANCY, n_slots=2, band_mcu_rows=1)
    try:
        jpgs = [j for _, j in corpus]
        outs = [np.zeros((f["height"], f["width"], 3), dtype=np.uint8) for f, _ in corpus]
        bad = bytearray(jpgs[2])
        scan, _ = M.mjd_parse(bytes(bad))
        # a long run of 1-bits (stuffed 0xFF bytes): no code word is all ones
        bad[scan.data_offset + 5: scan.data_offset + 45] = b"\xFF\x00" * 20
        with pytest.raises(M.MjdError) as ei:
            p.run(jpgs[:2] + [bytes(bad)] + jpgs[3:], outs)
        assert "image 2" in str(ei.value) and ei.value.code == -5
        with pytest.raises(M.MjdError) as ei:
            p.run([jpgs[0][:len(jpgs[0]) // 2]], outs[:1])
        assert "image 0" in str(ei.value)
        # a frame larger than the slots
        big = encode.encode_rgb(images.gradient_rgb(700, 700, 1), "444", 75)
        with pytest.raises(M.MjdError) as ei:
            p.run([fast_bitstream.write_jpeg(*big)], [np.zeros((700, 700, 3), np.uint8)])
        assert ei.value.code == -6
        # still decodes correctly afterwards
        st = p.run(jpgs, outs)
        assert st["images"] == len(jpgs)
        for o, e in zip(outs, exp):
            assert np.array_equal(o, e)
    finally:
        p.close()
