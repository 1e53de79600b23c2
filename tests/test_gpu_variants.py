"""GPU parity of the decoder variants (mjd_decode_variant) against the
variant oracle, byte for byte: every IDCT method (islow, ifast, float) on
every sampling ((1,1), (2,1), (1,2), (2,2), (4,1)) in both upsampling modes,
and grayscale; ragged sizes spanning several workgroups, a 1x1 image,
segments of one sub-tile up to a whole strip under several launch tunings,
extreme coefficients of the whole input domain, padded and misaligned
output rows, the largest widths and heights, and a 4096x3072 image per
method.  islow through the variants
path also equals mjd_decode on the samplings both serve."""
import numpy as np
import pytest

import oracle.variants as V

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

SAMPLINGS = [(1, 1), (2, 1), (1, 2), (2, 2), (4, 1)]
SIZES = [(257, 190), (33, 47), (1, 1)]


def say(msg):
    print(f"[gpu-variants] {msg}", flush=True)


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


def _case(seed, frame):
    """Quant tables 1..16 and coefficients on the domain |c * q| <= 1155:
    mostly decaying blocks, a tenth of them at the domain's extremes."""
    rng = np.random.default_rng(seed)
    qt = rng.integers(1, 17, (4, 64)).astype(np.uint16)
    n = V.variant_geometry(frame)["n_blocks"]
    lim = (1155 // qt.max(axis=0)).astype(np.int64)  # per position, safe for every table
    c = (rng.standard_normal((n, 64)) * lim / (1 + np.arange(64) / 6)).astype(np.int64)
    c[:, 0] = rng.integers(-lim[0], lim[0] + 1, n)
    ext = rng.random(n) < 0.1
    c[ext] = rng.choice([-1, 1], (int(ext.sum()), 64)) * lim
    return np.clip(c, -lim, lim).astype(np.int16), qt


def _run(M, ctx, frame, coef, qt, method, mode, ncomp=3):
    cd = torch.from_numpy(coef.reshape(-1)).cuda()
    qd = torch.from_numpy(qt.view(np.int16).reshape(-1)).cuda()
    out = M.decode_variant(ctx, frame, cd, qd, method, mode, ncomp)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("method", V.IDCT_METHODS)
def test_every_sampling_and_mode_matches_oracle(M, ctx, method):
    for i, (hy, vy) in enumerate(SAMPLINGS):
        for w, h in SIZES:
            fr = {"width": w, "height": h, "h": (hy, 1, 1), "v": (vy, 1, 1), "qsel": (0, 1, 2)}
            coef, qt = _case(1000 * i + w, fr)
            for mode in ("simple", "fancy"):
                say(f"{method} {hy}x{vy} {w}x{h} {mode}")
                got = _run(M, ctx, fr, coef, qt, method, mode)
                exp = V.decode_variant(fr, coef, qt, method, mode)
                assert np.array_equal(got, exp), (method, hy, vy, w, h, mode, int((got != exp).sum()))


# launch tunings: (sub-tiles per segment, workgroups, shape index).  Long
# segments wrap every luma/chroma ring of the segment walk several times
# (the 190-pixel image holds 6 sub-tiles of 2 MCU rows per strip); 8
# workgroups walk many segments each; the shape index picks among the
# single-image kernel's shapes where the islow class has several.
TUNINGS = [(1, 8, 0), (3, 0, 1), (64, 0, 2), (64, 8, 0)]


@pytest.mark.parametrize("method", V.IDCT_METHODS)
def test_long_segments_and_tunings_match_oracle(M, ctx, method):
    w, h = 257, 190
    try:
        for i, (hy, vy) in enumerate(SAMPLINGS):
            fr = {"width": w, "height": h, "h": (hy, 1, 1), "v": (vy, 1, 1), "qsel": (0, 1, 2)}
            coef, qt = _case(5000 + 100 * i, fr)
            for mode in ("simple", "fancy"):
                exp = V.decode_variant(fr, coef, qt, method, mode)
                for seg, wg, shape in TUNINGS:
                    say(f"{method} {hy}x{vy} {mode} seg={seg} wg={wg} shape={shape}")
                    M.mjd_ctx_set_tuning(ctx, seg, wg, shape)
                    got = _run(M, ctx, fr, coef, qt, method, mode)
                    assert np.array_equal(got, exp), (method, hy, vy, mode, seg, wg, shape,
                                                      int((got != exp).sum()))
    finally:
        M.mjd_ctx_set_tuning(ctx, 0, 0, 0)


@pytest.mark.parametrize("method", V.IDCT_METHODS)
def test_grayscale_matches_oracle(M, ctx, method):
    for w, h in SIZES + [(640, 480)]:
        fr = {"width": w, "height": h, "ncomp": 1, "h": (1, 1, 1), "v": (1, 1, 1), "qsel": (3, 0, 0)}
        coef, qt = _case(77 + w, fr)
        say(f"{method} grayscale {w}x{h}")
        got = _run(M, ctx, fr, coef, qt, method, "fancy", ncomp=1)
        assert got.shape == (h, w)
        assert np.array_equal(got, V.decode_variant(fr, coef, qt, method)), (method, w, h)


def test_islow_variant_equals_the_fused_kernel(M, ctx):
    for hy, vy in ((1, 1), (2, 1), (2, 2)):
        fr = {"width": 333, "height": 97, "h": (hy, 1, 1), "v": (vy, 1, 1), "qsel": (0, 1, 1)}
        coef, qt = _case(5 + hy + vy, fr)
        for mode in ("simple", "fancy"):
            say(f"islow vs fused {hy}x{vy} {mode}")
            cd = torch.from_numpy(coef.reshape(-1)).cuda()
            qd = torch.from_numpy(qt.view(np.int16).reshape(-1)).cuda()
            a = M.decode_variant(ctx, fr, cd, qd, "islow", mode)
            b = M.decode(ctx, fr, cd, qd, mode)
            torch.cuda.synchronize()
            assert torch.equal(a, b)


def test_padded_and_misaligned_rows(M, ctx):
    # rows of pitch 3w + 5 starting one byte past an aligned address: the
    # bytes between rows and around the image stay untouched
    for method, ncomp, (hy, vy) in (("float", 3, (2, 2)), ("float", 3, (4, 1)), ("float", 1, (1, 1)),
                                    ("islow", 3, (2, 2)), ("islow", 1, (1, 1))):
        w, h = 61, 35
        fr = {"width": w, "height": h, "h": (hy, 1, 1), "v": (vy, 1, 1), "qsel": (0, 1, 1), "ncomp": ncomp}
        coef, qt = _case(31 + hy, fr)
        v = M.make_variant(fr, ncomp, method, "fancy")
        g, wb = M.mjd_variant_geometry(v)
        pitch = ncomp * w + 5
        buf = torch.full((h * pitch + 64,), 0xA5, dtype=torch.uint8, device="cuda")
        work = torch.empty(max(wb, 16), dtype=torch.uint8, device="cuda")
        cd = torch.from_numpy(coef.reshape(-1)).cuda()
        qd = torch.from_numpy(qt.view(np.int16).reshape(-1)).cuda()
        say(f"misaligned {method} ncomp={ncomp} {hy}x{vy}")
        M.mjd_decode_variant(ctx, v, cd, qd, buf.data_ptr() + 1, pitch, work, wb)
        torch.cuda.synchronize()
        b = buf.cpu().numpy()
        rows = b[1:1 + h * pitch].reshape(h, pitch)
        exp = V.decode_variant(fr, coef, qt, method, "fancy")
        assert np.array_equal(rows[:, :ncomp * w].reshape(exp.shape), exp), method
        assert np.all(rows[:, ncomp * w:] == 0xA5) and b[0] == 0xA5 and np.all(b[1 + h * pitch:] == 0xA5)


def test_bad_calls_are_refused(M, ctx):
    fr = {"width": 64, "height": 64, "h": (2, 1, 1), "v": (2, 1, 1), "qsel": (0, 1, 1)}
    v = M.make_variant(fr, 3, "ifast")
    g, wb = M.mjd_variant_geometry(v)
    assert wb == 0  # full size: the fused pass needs no workspace
    cd = torch.zeros(g["n_blocks"] * 64, dtype=torch.int16, device="cuda")
    qd = torch.ones(256, dtype=torch.int16, device="cuda")
    out = torch.empty((64, 64, 3), dtype=torch.uint8, device="cuda")
    for args in ((cd, qd, out, 191, 0, 0),                # pitch below 3 * width
                 (cd, qd, out, 1 << 24, 0, 0),            # pitch not below 2^24 (fused pass)
                 (cd.data_ptr() + 2, qd, out, 192, 0, 0)):  # misaligned coefficients
        with pytest.raises(M.MjdError):
            M.mjd_decode_variant(ctx, v, *args)
    vs = M.make_variant(fr, 3, "islow", "fancy", 2)
    gs, wbs = M.mjd_variant_geometry(vs)
    work = torch.empty(wbs, dtype=torch.uint8, device="cuda")
    small = torch.empty((32, 32, 3), dtype=torch.uint8, device="cuda")
    for args in ((cd, qd, small, 96, work, wbs - 1),      # workspace too small
                 (cd, qd, small, 96, 0, wbs)):            # no workspace
        with pytest.raises(M.MjdError):
            M.mjd_decode_variant(ctx, vs, *args)
    torch.cuda.synchronize()


@pytest.mark.parametrize("w,h,hy,vy,ncomp", [(65535, 16, 4, 1, 3), (65535, 9, 1, 2, 3), (17, 65535, 2, 2, 3),
                                             (65535, 11, 1, 1, 1)])
def test_maximum_sizes(M, ctx, w, h, hy, vy, ncomp):
    fr = {"width": w, "height": h, "h": (hy, 1, 1), "v": (vy, 1, 1), "qsel": (0, 1, 1), "ncomp": ncomp}
    coef, qt = _case(w + h + hy, fr)
    for method in V.IDCT_METHODS:
        say(f"{method} {w}x{h} {hy}x{vy} ncomp={ncomp}")
        got = _run(M, ctx, fr, coef, qt, method, "fancy", ncomp)
        assert np.array_equal(got, V.decode_variant(fr, coef, qt, method, "fancy")), (method, w, h)


@pytest.mark.parametrize("scale", [2, 4, 8])
def test_scaled_decoding_matches_oracle(M, ctx, scale):
    # every sampling in both modes, grayscale, ragged sizes and the full image
    for i, (hy, vy) in enumerate(SAMPLINGS):
        for w, h in SIZES + [(65, 9)]:
            fr = {"width": w, "height": h, "h": (hy, 1, 1), "v": (vy, 1, 1), "qsel": (0, 1, 2)}
            coef, qt = _case(500 * i + w + scale, fr)
            for mode in ("simple", "fancy"):
                say(f"1/{scale} {hy}x{vy} {w}x{h} {mode}")
                cd = torch.from_numpy(coef.reshape(-1)).cuda()
                qd = torch.from_numpy(qt.view(np.int16).reshape(-1)).cuda()
                got = M.decode_variant(ctx, fr, cd, qd, "islow", mode, scale=scale).cpu().numpy()
                exp = V.decode_variant(fr, coef, qt, "islow", mode, scale)
                assert np.array_equal(got, exp), (scale, hy, vy, w, h, mode)
    for w, h in ((257, 190), (1, 1), (65535, 9)):
        fr = {"width": w, "height": h, "ncomp": 1, "h": (1, 1, 1), "v": (1, 1, 1), "qsel": (1, 0, 0)}
        coef, qt = _case(w * scale, fr)
        say(f"1/{scale} grayscale {w}x{h}")
        cd = torch.from_numpy(coef.reshape(-1)).cuda()
        qd = torch.from_numpy(qt.view(np.int16).reshape(-1)).cuda()
        got = M.decode_variant(ctx, fr, cd, qd, "islow", ncomp=1, scale=scale).cpu().numpy()
        assert np.array_equal(got, V.decode_variant(fr, coef, qt, "islow", scale=scale))
    from synth import workloads
    frame, coef, qt = workloads.large_420_fancy()
    say(f"1/{scale} 4096x3072 4:2:0 fancy")
    cd = torch.from_numpy(coef.reshape(-1)).cuda()
    qd = torch.from_numpy(qt.view(np.int16).reshape(-1)).cuda()
    got = M.decode_variant(ctx, frame, cd, qd, "islow", "fancy", scale=scale).cpu().numpy()
    assert np.array_equal(got, V.decode_variant(frame, coef, qt, "islow", "fancy", scale))


def test_variant_bitstreams_decode_on_the_device(M, ctx):
    # h1v2 and 4:1:1 bitstreams: the GPU entropy kernel returns the encoded
    # coefficients, and the variants path turns them into the oracle's RGB
    from synth import bitstream
    rng = np.random.default_rng(61)
    for hy, vy in ((1, 2), (4, 1)):
        for w, h, ri in ((97, 61, 4), (640, 480, 32)):
            fr = {"width": w, "height": h, "h": (hy, 1, 1), "v": (vy, 1, 1), "qsel": (0, 1, 1)}
            coef, qt = _case(w + hy, fr)
            coef[rng.random(coef.shape) < 0.5] = 0
            coef = np.clip(coef, -1023, 1023)  # baseline ranges: AC and DC-difference categories
            data = bitstream.write_jpeg(fr, coef, qt, restart_interval=ri)
            scan, q = M.mjd_parse(data)
            off = M.mjd_restart_index(data, scan)
            d_jpg = torch.zeros(-(-len(data) // 16) * 16, dtype=torch.uint8, device="cuda")
            d_jpg[:len(data)] = torch.from_numpy(np.frombuffer(data, dtype=np.uint8).copy()).cuda()
            d_coef = torch.full((coef.size,), 0x5A5A, dtype=torch.int16, device="cuda")
            say(f"bitstream {hy}x{vy} {w}x{h} ri={ri}")
            b = M.EntropyBatch(ctx, [(scan, off, d_jpg, len(data), d_coef)])
            b.launch()
            assert b.status() == -1
            b.close()
            assert np.array_equal(d_coef.cpu().numpy().reshape(-1, 64), coef)
            qd = torch.from_numpy(q.view(np.int16).reshape(-1)).cuda()
            got = M.decode_variant(ctx, M.scan_frame(scan), d_coef, qd, "islow", "fancy").cpu().numpy()
            assert np.array_equal(got, V.decode_variant(fr, coef, qt, "islow", "fancy"))
    # grayscale: one component, one block per MCU
    for w, h, ri in ((97, 61, 3), (640, 480, 40)):
        fr = {"width": w, "height": h, "ncomp": 1, "h": (1, 1, 1), "v": (1, 1, 1), "qsel": (1, 1, 1)}
        coef, qt = _case(w + 7, fr)
        coef[rng.random(coef.shape) < 0.5] = 0
        coef = np.clip(coef, -1023, 1023)
        data = bitstream.write_jpeg(fr, coef, qt, restart_interval=ri)
        scan, q = M.mjd_parse(data)
        off = M.mjd_restart_index(data, scan)
        d_jpg = torch.zeros(-(-len(data) // 16) * 16, dtype=torch.uint8, device="cuda")
        d_jpg[:len(data)] = torch.from_numpy(np.frombuffer(data, dtype=np.uint8).copy()).cuda()
        d_coef = torch.full((coef.size,), 0x5A5A, dtype=torch.int16, device="cuda")
        say(f"grayscale bitstream {w}x{h} ri={ri}")
        b = M.EntropyBatch(ctx, [(scan, off, d_jpg, len(data), d_coef)])
        b.launch()
        assert b.status() == -1
        b.close()
        assert np.array_equal(d_coef.cpu().numpy().reshape(-1, 64), coef)
        qd = torch.from_numpy(q.view(np.int16).reshape(-1)).cuda()
        for method in V.IDCT_METHODS:
            got = M.decode_variant(ctx, M.scan_frame(scan), d_coef, qd, method, ncomp=1).cpu().numpy()
            assert np.array_equal(got, V.decode_variant(fr, coef, qt, method))


def test_mixed_sampling_entropy_batch(M, ctx):
    # one GPU entropy launch over 4:2:0, h1v2, 4:1:1 and grayscale streams:
    # every job's coefficients come back as encoded
    from synth import bitstream
    rng = np.random.default_rng(83)
    jobs, want = [], []
    for i, (hy, vy, nc) in enumerate(((2, 2, 3), (1, 2, 3), (4, 1, 3), (1, 1, 1), (2, 2, 3))):
        w, h = (131 + 40 * i, 77 + 13 * i)
        fr = {"width": w, "height": h, "h": (hy, 1, 1), "v": (vy, 1, 1), "qsel": (0, 1, 1), "ncomp": nc}
        coef, qt = _case(900 + i, fr)
        coef[rng.random(coef.shape) < 0.5] = 0
        coef = np.clip(coef, -1023, 1023)
        data = bitstream.write_jpeg(fr, coef, qt, restart_interval=(0, 3, 8, 1, 64)[i])
        scan, _ = M.mjd_parse(data)
        off = M.mjd_restart_index(data, scan)
        d_jpg = torch.zeros(-(-len(data) // 16) * 16, dtype=torch.uint8, device="cuda")
        d_jpg[:len(data)] = torch.from_numpy(np.frombuffer(data, dtype=np.uint8).copy()).cuda()
        jobs.append((scan, off, d_jpg, len(data), torch.full((coef.size,), 0x5A5A, dtype=torch.int16, device="cuda")))
        want.append(coef)
    say("mixed-sampling entropy batch")
    b = M.EntropyBatch(ctx, jobs)
    b.launch()
    assert b.status() == -1
    b.close()
    for j, coef in zip(jobs, want):
        assert np.array_equal(j[4].cpu().numpy().reshape(-1, 64), coef)


@pytest.mark.parametrize("method", V.IDCT_METHODS)
def test_full_size_image(M, ctx, method):
    from synth import workloads
    frame, coef, qt = workloads.large_420_fancy()
    say(f"{method} 4096x3072 4:2:0 fancy")
    got = _run(M, ctx, frame, coef, qt, method, "fancy")
    exp = V.decode_variant(frame, coef, qt, method, "fancy")
    assert np.array_equal(got, exp), int((got != exp).sum())
