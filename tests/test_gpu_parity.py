"""GPU parity: the fused HIP kernel, called through the C ABI, against the
oracle, element by element.  All of the path is integer arithmetic, so the
bar is bit-exact (tolerance 0)."""
import numpy as np
import pytest

import oracle
from synth import encode, images, workloads

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-parity] {msg}", flush=True)


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


def to_dev(coef, qt):
    c = torch.from_numpy(np.ascontiguousarray(coef, dtype=np.int16)).cuda()
    q = torch.from_numpy(np.ascontiguousarray(qt, dtype=np.uint16).view(np.int16)).cuda()
    return c, q


def gpu_decode(M, ctx, frame, coef, qt, mode, rows=None):
    c, q = to_dev(coef, qt)
    out = M.decode(ctx, frame, c, q, mode, rows=rows)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def assert_same(got, exp, what):
    if not np.array_equal(got, exp):
        bad = np.argwhere(got != exp)
        y, x, ch = bad[0]
        raise AssertionError(f"{what}: {len(bad)} bytes differ; first at y={y} x={x} ch={ch}: "
                             f"gpu {got[y, x]} oracle {exp[y, x]}")


def test_small_420_simple_bit_exact(M, ctx):
    say("256x256 4:2:0 q75 simple")
    frame, coef, qt = workloads.small_420_simple()
    assert_same(gpu_decode(M, ctx, frame, coef, qt, "simple"), oracle.decode(frame, coef, qt, "simple"),
                "256x256 simple")
    assert_same(gpu_decode(M, ctx, frame, coef, qt, "fancy"), oracle.decode(frame, coef, qt, "fancy"),
                "256x256 fancy")


SIZES = [(1, 1), (2, 3), (7, 9), (8, 8), (16, 16), (17, 33), (31, 17), (100, 75), (129, 333),
         (257, 130), (640, 480), (1000, 8), (8, 1000), (511, 513)]


@pytest.mark.parametrize("samp", ["444", "422", "420"])
@pytest.mark.parametrize("mode", ["simple", "fancy"])
def test_sizes_and_edges_bit_exact(M, ctx, samp, mode):
    for i, (w, h) in enumerate(SIZES):
        say(f"{samp} {mode} {w}x{h}")
        rgb = images.texture_rgb(w, h, 1000 + i, sigma=12)
        frame, coef, qt = encode.encode_rgb(rgb, samp, 50 + 3 * i)
        assert_same(gpu_decode(M, ctx, frame, coef, qt, mode), oracle.decode(frame, coef, qt, mode),
                    f"{samp} {mode} {w}x{h}")


@pytest.mark.parametrize("samp", ["444", "422", "420"])
def test_random_coefficients_bit_exact(M, ctx, samp):
    # dense random blocks across the conforming range, all-ones tables
    for w, h in ((203, 77), (64, 64)):
        say(f"random coefficients {samp} {w}x{h}")
        frame = encode.make_frame(w, h, samp)
        coef = workloads.random_coefficients(frame, seed=7 * w + h, density=0.6)
        qt = np.ones((4, 64), dtype=np.uint16)
        for mode in ("simple", "fancy"):
            assert_same(gpu_decode(M, ctx, frame, coef, qt, mode), oracle.decode(frame, coef, qt, mode),
                        f"random {samp} {mode}")


@pytest.mark.parametrize("samp", ["444", "422", "420"])
def test_dot_product_and_int32_row_pass_paths_bit_exact(M, ctx, samp):
    """The row pass runs as int16 dot products for a wave whose dequantised
    coefficients all lie in [-1024, 1023] and in int32 otherwise; both give
    the oracle's bits.  Cases: every coefficient at the ends of that range
    (the largest pass-1 results the dot-product path meets), a few blocks
    reaching 1024..1155 among conforming ones (mixed waves), and the whole
    documented domain (+-1155) densely."""
    w, h = 203, 77
    frame = encode.make_frame(w, h, samp)
    base = workloads.random_coefficients(frame, seed=w * 31 + h, density=0.6)
    rng = np.random.default_rng(4242)
    extremes = rng.choice(np.array([-1024, 1023], dtype=np.int16), size=base.shape)
    mixed = base.copy()
    few = rng.random(len(mixed)) < 0.02
    mixed[few, rng.integers(0, 64, few.sum())] = rng.choice(np.array([-1155, -1100, 1024, 1155], dtype=np.int16),
                                                           few.sum())
    dense = rng.integers(-1155, 1156, size=base.shape).astype(np.int16)
    qt = np.ones((4, 64), dtype=np.uint16)
    for name, coef in (("extremes", extremes), ("mixed", mixed), ("dense", dense)):
        for mode in ("simple", "fancy"):
            say(f"row-pass paths {samp} {mode} {name}")
            assert_same(gpu_decode(M, ctx, frame, coef, qt, mode), oracle.decode(frame, coef, qt, mode),
                        f"{name} {samp} {mode}")
    # the same ranges reached through quantisation factors: c * Q near the ends
    q2 = np.full((4, 64), 5, dtype=np.uint16)
    coef = rng.choice(np.array([-231, -205, 204, 231], dtype=np.int16), size=base.shape)
    for mode in ("simple", "fancy"):
        say(f"row-pass paths {samp} {mode} c*Q")
        assert_same(gpu_decode(M, ctx, frame, coef, q2, mode), oracle.decode(frame, coef, q2, mode),
                    f"c*Q {samp} {mode}")


@pytest.mark.parametrize("samp", ["422", "420"])
def test_band_decode_equals_whole_decode(M, ctx, samp):
    rgb = images.texture_rgb(300, 203, 77, sigma=12)
    frame, coef, qt = encode.encode_rgb(rgb, samp, 88)
    g = oracle.geometry(frame)
    whole = oracle.decode(frame, coef, qt, "fancy")
    c, q = to_dev(coef, qt)
    for r0, r1 in ((0, 1), (1, 3), (2, g["mcus_y"]), (g["mcus_y"] - 1, g["mcus_y"]), (0, g["mcus_y"])):
        say(f"band {samp} rows [{r0},{r1})")
        out = torch.full((frame["height"], frame["width"], 3), 7, dtype=torch.uint8, device="cuda")
        M.decode(ctx, frame, c, q, "fancy", out=out, rows=(r0, r1))
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        y0, y1 = r0 * g["mcu_h"], min(frame["height"], r1 * g["mcu_h"])
        assert_same(got[y0:y1], whole[y0:y1], f"band rows {r0}..{r1}")
        assert np.all(got[:y0] == 7) and np.all(got[y1:] == 7), "band wrote outside its rows"


@pytest.mark.parametrize("samp,mode", [("420", "fancy"), ("420", "simple"), ("422", "fancy"), ("444", "simple")])
def test_unaligned_output_pitch_and_base(M, ctx, samp, mode):
    """Every row start alignment (pitch and base offsets 0..3 mod 4) gives
    the oracle's bytes and leaves the padding and the bytes before the image
    untouched; widths span several strips and end in a ragged MCU."""
    rgb = images.texture_rgb(301, 45, 5, sigma=12)
    frame, coef, qt = encode.encode_rgb(rgb, samp, 80)
    exp = oracle.decode(frame, coef, qt, mode)
    c, q = to_dev(coef, qt)
    w, h = frame["width"], frame["height"]
    for pitch, base in ((3 * w + 1, 0), (3 * w + 2, 2), (3 * w + 4, 1), (3 * w + 5, 3), (3 * w + 3, 0)):
        say(f"{samp} {mode} pitch {pitch} base offset {base}")
        buf = torch.full((h * pitch + base + 16,), 9, dtype=torch.uint8, device="cuda")
        M.mjd_decode(ctx, frame, c, q, M.UPSAMPLE[mode], buf.data_ptr() + base, pitch, 0,
                     oracle.geometry(frame)["mcus_y"])
        torch.cuda.synchronize()
        host = buf.cpu().numpy()
        assert np.all(host[:base] == 9), "wrote before the image"
        for y in range(h):
            row = host[base + y * pitch: base + y * pitch + 3 * w].reshape(w, 3)
            assert np.array_equal(row, exp[y]), f"row {y}"
            pad = host[base + y * pitch + 3 * w: base + (y + 1) * pitch] if y < h - 1 else []
            assert np.all(np.asarray(pad) == 9), "wrote into row padding"
        assert np.all(host[base + (h - 1) * pitch + 3 * w:] == 9), "wrote past the image"


def test_large_420_fancy_full_image_bit_exact(M, ctx):
    """The headline image whole, under the library's default launch, under
    every sub-tile shape at the launch sizes the autotuner searches (fewer,
    as many and more workgroups than stay resident), and under the launch
    the tuning cache holds for this workload on this device, if any."""
    from paper_1311_5304_amd import autotune
    say("4096x3072 4:2:0 q90 fancy (full image)")
    frame, coef, qt = workloads.large_420_fancy()
    exp = oracle.decode(frame, coef, qt, "fancy")
    assert_same(gpu_decode(M, ctx, frame, coef, qt, "fancy"), exp, "4096x3072 fancy")
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    try:
        for shape in range(M.mjd_shape_count(2, 2, M.MJD_UPSAMPLE_FANCY)):
            for seg, k in ((3, 2), (1, 1), (6, 4)):
                M.mjd_ctx_set_tuning(ctx, seg, k * cus, shape)
                say(f"4096x3072 fancy shape {shape} seg {seg} workgroups {k * cus}")
                assert_same(gpu_decode(M, ctx, frame, coef, qt, "fancy"), exp,
                            f"4096x3072 fancy shape={shape} seg={seg} wgs={k * cus}")
        if autotune.apply_cached(ctx, frame, M.MJD_UPSAMPLE_FANCY):
            say(f"4096x3072 fancy cached tuning {M.mjd_ctx_get_tuning(ctx)}")
            assert_same(gpu_decode(M, ctx, frame, coef, qt, "fancy"), exp, "4096x3072 fancy, cached tuning")
    finally:
        M.mjd_ctx_set_tuning(ctx, 0, 0, 0)


@pytest.mark.parametrize("w,h,samp", [(65535, 16, "420"), (16, 65535, "422"), (65535, 9, "444")])
def test_maximum_dimensions(M, ctx, w, h, samp):
    say(f"max dims {w}x{h} {samp}")
    frame = encode.make_frame(w, h, samp)
    coef = workloads.random_coefficients(frame, seed=w ^ h, density=0.2)
    qt = np.ones((4, 64), dtype=np.uint16)
    for mode in ("simple", "fancy"):
        assert_same(gpu_decode(M, ctx, frame, coef, qt, mode), oracle.decode(frame, coef, qt, mode),
                    f"max {w}x{h} {samp} {mode}")


def test_invalid_arguments_are_rejected(M, ctx):
    frame, coef, qt = workloads.small_420_simple()
    c, q = to_dev(coef, qt)
    out = torch.empty((256, 256, 3), dtype=torch.uint8, device="cuda")
    with pytest.raises(M.MjdError):
        M.mjd_decode(ctx, frame, c, q, 1, out, 3 * 256, 3, 3)            # empty band
    with pytest.raises(M.MjdError):
        M.mjd_decode(ctx, frame, c, q, 1, out, 3 * 256, 0, 17)           # past the last MCU row
    with pytest.raises(M.MjdError):
        M.mjd_decode(ctx, frame, c.data_ptr() + 2, q, 1, out, 3 * 256, 0, 16)  # misaligned
    with pytest.raises(M.MjdError):
        M.mjd_decode(ctx, frame, c, q, 1, out, 3 * 256 - 1, 0, 16)       # pitch too small
    with pytest.raises(M.MjdError):
        M.mjd_decode(ctx, frame, c, q, 2, out, 3 * 256, 0, 16)           # unknown mode


def test_copy_probe_copies(M, ctx):
    src = torch.randint(0, 255, (1 << 20,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(src)
    M.mjd_copy(ctx, dst, src, src.numel())
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


@pytest.mark.parametrize("samp,mode", [("420", "fancy"), ("420", "simple"), ("422", "fancy"),
                                       ("422", "simple"), ("444", "simple")])
def test_launch_shapes_bit_exact(M, ctx, samp, mode):
    """Every sub-tile shape of the class, segments of several sub-tiles (the
    prefetch pipeline and the chroma ring), few workgroups (each takes many
    segments), more workgroups than stay resident, and bands: the output
    never depends on the launch shape."""
    rgb = images.texture_rgb(523, 437, 31, sigma=12)
    frame, coef, qt = encode.encode_rgb(rgb, samp, 83)
    exp = oracle.decode(frame, coef, qt, mode)
    g = oracle.geometry(frame)
    c, q = to_dev(coef, qt)
    h, v = frame["h"][0], frame["v"][0]
    n_shapes = M.mjd_shape_count(h, v, M.UPSAMPLE[mode])
    try:
        for shape in range(n_shapes):
            info = M.mjd_shape_info(ctx, h, v, M.UPSAMPLE[mode], shape)
            for seg, wgs in ((1, 0), (2, 0), (3, 8), (7, 0), (64, 0), (5, 16), (0, 8), (1, 4096)):
                M.mjd_ctx_set_tuning(ctx, seg, wgs, shape)
                say(f"shape {samp} {mode} {info} seg_subtiles={seg} workgroups={wgs}")
                out = M.decode(ctx, frame, c, q, mode)
                torch.cuda.synchronize()
                assert_same(out.cpu().numpy(), exp, f"{samp} {mode} shape={shape} seg={seg} wgs={wgs}")
                for r0, r1 in ((3, g["mcus_y"] - 2), (g["mcus_y"] - 5, g["mcus_y"])):
                    band = torch.full((frame["height"], frame["width"], 3), 5, dtype=torch.uint8, device="cuda")
                    M.decode(ctx, frame, c, q, mode, out=band, rows=(r0, r1))
                    torch.cuda.synchronize()
                    got = band.cpu().numpy()
                    y0, y1 = r0 * g["mcu_h"], min(frame["height"], r1 * g["mcu_h"])
                    assert_same(got[y0:y1], exp[y0:y1], f"band {r0}..{r1} shape={shape} seg={seg} wgs={wgs}")
                    assert np.all(got[:y0] == 5) and np.all(got[y1:] == 5)
    finally:
        M.mjd_ctx_set_tuning(ctx, 0, 0)
