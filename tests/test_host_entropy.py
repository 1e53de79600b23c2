"""Host side of the library (CPU only): the JPEG marker parser, the
restart-interval index and the threaded Huffman decoder, against the
oracle's own reader on the project's bitstreams and on libjpeg-written
files.  Integer work, so the bar is equality."""
import io

import numpy as np
import pytest

import oracle
from oracle.geometry import geometry
from synth import bitstream, encode, images
from tests.conftest import requires_pillow


@pytest.fixture(scope="module")
def M():
    import paper_1311_5304_amd as mod
    return mod


def _stream(w, h, samp, q, ri, seed=3, texture=True):
    rgb = images.texture_rgb(w, h, seed, sigma=12) if texture else images.gradient_rgb(w, h, seed, sigma=8)
    frame, coef, qt = encode.encode_rgb(rgb, samp, q)
    return frame, coef, qt, bitstream.write_jpeg(frame, coef, qt, restart_interval=ri)


@pytest.mark.parametrize("samp", ["444", "422", "420"])
@pytest.mark.parametrize("ri", [0, 1, 3, 32])
def test_decode_matches_oracle_reader(M, samp, ri):
    for (w, h, seed) in ((1, 1, 1), (17, 9, 2), (45, 38, 3), (130, 67, 4)):
        frame, coef, qt, data = _stream(w, h, samp, 85, ri, seed)
        f_or, c_or, q_or = oracle.parse_and_decode(data)
        f, c, q = M.entropy_decode(data, n_threads=3)
        assert f == f_or == frame
        assert np.array_equal(q, q_or)
        assert np.array_equal(c, c_or)
        assert np.array_equal(c, coef)


def test_extreme_values(M):
    frame = encode.make_frame(16, 8, "444")
    coef = np.zeros((6, 64), dtype=np.int16)
    coef[0, 0], coef[1, 0], coef[2, 0] = 1023, -1024, 0
    coef[3, 0], coef[4, 0], coef[5, 0] = -1024, 1023, 1
    coef[0, 63] = -1023
    coef[1, 17] = 1023
    coef[2, 1:64] = np.arange(1, 64)
    coef[5, 1:64:17] = -700          # long zero runs (ZRL)
    qt = np.ones((4, 64), dtype=np.uint16)
    for ri in (0, 1):
        data = bitstream.write_jpeg(frame, coef, qt, restart_interval=ri)
        _, c, _ = M.entropy_decode(data)
        assert np.array_equal(c, coef)


def test_threads_and_bands_agree(M):
    frame, coef, qt, data = _stream(300, 170, "420", 90, 7, seed=9)
    scan, _ = M.mjd_parse(data)
    off = M.mjd_restart_index(data, scan)
    g = M.mjd_geometry_of(frame)
    per_row = g["mcus_x"] * g["blocks_per_mcu"]
    for nt in (1, 2, 5, 16):
        out = np.full((g["n_blocks"], 64), 7, dtype=np.int16)
        M.mjd_entropy_decode(data, scan, off, out, 0, g["mcus_y"], nt)
        assert np.array_equal(out, coef)
    # bands: only the band's blocks are written, with the same values
    for r0, r1 in ((0, 1), (2, 5), (g["mcus_y"] - 1, g["mcus_y"])):
        out = np.full((g["n_blocks"], 64), 7, dtype=np.int16)
        M.mjd_entropy_decode(data, scan, None, out, r0, r1, 4)
        assert np.array_equal(out[r0 * per_row:r1 * per_row], coef[r0 * per_row:r1 * per_row])
        assert np.all(out[:r0 * per_row] == 7) and np.all(out[r1 * per_row:] == 7)


def test_restart_index_points_past_each_marker(M):
    frame, coef, qt, data = _stream(64, 48, "422", 75, 5)
    scan, _ = M.mjd_parse(data)
    n_mcus = geometry(frame)["mcus_x"] * geometry(frame)["mcus_y"]
    assert scan.restart_interval == 5 and scan.n_intervals == -(-n_mcus // 5)
    off = M.mjd_restart_index(data, scan)
    assert off[0] == scan.data_offset
    for i in range(1, scan.n_intervals):
        assert data[off[i] - 2] == 0xFF and data[off[i] - 1] == 0xD0 + ((i - 1) & 7)
    assert off[-1] == len(data) and data[-2:] == b"\xFF\xD9"


def test_parse_fields(M):
    frame, coef, qt, data = _stream(77, 20, "420", 60, 4)
    scan, q = M.mjd_parse(data)
    assert M.scan_frame(scan) == frame
    assert np.array_equal(q[:2], qt[:2]) and np.all(q[2:] == 1)
    assert tuple(scan.dc_sel) == (0, 1, 1) and tuple(scan.ac_sel) == (0, 1, 1)
    assert scan.dc[0].defined and scan.ac[1].defined and not scan.dc[2].defined


def test_corrupt_and_truncated_streams_fail_cleanly(M):
    frame, coef, qt, data = _stream(40, 40, "420", 75, 2, seed=5)
    for cut in list(range(0, 40)) + list(range(len(data) // 2, len(data) - 1, 7)):
        with pytest.raises(M.MjdError):
            M.entropy_decode(data[:cut])
    # a renumbered restart marker
    bad = bytearray(data)
    i = bad.index(b"\xFF\xD0")
    bad[i + 1] = 0xD3
    with pytest.raises(M.MjdError) as ei:
        M.entropy_decode(bytes(bad))
    assert ei.value.code == -5
    # random byte damage in the entropy-coded data: an error or some result,
    # never a crash
    scan, _ = M.mjd_parse(data)
    rng = np.random.default_rng(1)
    for _ in range(300):
        bad = bytearray(data)
        for _ in range(int(rng.integers(1, 4))):
            bad[int(rng.integers(scan.data_offset, scan.data_end))] = int(rng.integers(0, 256))
        try:
            M.entropy_decode(bytes(bad), n_threads=2)
        except M.MjdError as e:
            assert e.code in (-5, -1)


@pytest.mark.parametrize("hy,vy", [(1, 2), (4, 1)])
@pytest.mark.parametrize("ri", [0, 2, 5])
def test_variant_samplings_decode_to_the_encoded_coefficients(M, hy, vy, ri):
    # h1v2 and 4:1:1 streams: the parser and the threaded decoder return the
    # coefficients the writer encoded; the fused decoder refuses the frame
    import oracle.variants as V
    rng = np.random.default_rng(hy * 10 + vy + ri)
    for w, h in ((45, 35), (8, 8), (97, 61)):
        fr = {"width": w, "height": h, "h": (hy, 1, 1), "v": (vy, 1, 1), "qsel": (0, 1, 1)}
        n = V.variant_geometry(fr)["n_blocks"]
        coef = rng.integers(-30, 31, (n, 64)).astype(np.int16)
        coef[:, 0] = rng.integers(-500, 501, n)
        coef[rng.random((n, 64)) < 0.6] = 0
        qt = rng.integers(1, 50, (4, 64)).astype(np.uint16)
        data = bitstream.write_jpeg(fr, coef, qt, restart_interval=ri)
        f, c, q = M.entropy_decode(data, n_threads=3)
        assert (f["h"], f["v"]) == ((hy, 1, 1), (vy, 1, 1))
        assert np.array_equal(c, coef.reshape(c.shape))
        with pytest.raises(M.MjdError) as ei:
            M.mjd_geometry_of(f)
        assert ei.value.code == -2


@pytest.mark.parametrize("ri", [0, 1, 7])
def test_grayscale_streams_decode_to_the_encoded_coefficients(M, ri):
    import oracle.variants as V
    rng = np.random.default_rng(70 + ri)
    for w, h in ((45, 35), (8, 8), (1, 1), (130, 9)):
        fr = {"width": w, "height": h, "ncomp": 1, "h": (1, 1, 1), "v": (1, 1, 1), "qsel": (2, 2, 2)}
        n = V.variant_geometry(fr)["n_blocks"]
        coef = rng.integers(-40, 41, (n, 64)).astype(np.int16)
        coef[:, 0] = rng.integers(-900, 901, n)
        coef[rng.random((n, 64)) < 0.5] = 0
        qt = rng.integers(1, 50, (4, 64)).astype(np.uint16)
        data = bitstream.write_jpeg(fr, coef, qt, restart_interval=ri)
        scan, q = M.mjd_parse(data)
        assert scan.ncomp == 1 and scan.n_intervals == (-(-n // ri) if ri else 1)
        f, c, q = M.entropy_decode(data, n_threads=3)
        assert f["ncomp"] == 1 and f["qsel"][0] == 2
        assert np.array_equal(c, coef.reshape(c.shape)) and np.array_equal(q[2], qt[2])


def test_unsupported_streams(M):
    frame, coef, qt, data = _stream(16, 16, "444", 75, 0)
    bad = bytearray(data)
    i = bad.index(b"\xFF\xC0")
    bad[i + 1] = 0xC2   # progressive
    with pytest.raises(M.MjdError) as ei:
        M.mjd_parse(bytes(bad))
    assert ei.value.code == -2
    with pytest.raises(M.MjdError) as ei:
        M.mjd_parse(b"\xFF\xD8\xFF\xD9")
    assert ei.value.code == -5


@requires_pillow
def test_reads_libjpeg_written_files(M):
    from PIL import Image
    rgb = images.texture_rgb(97, 61, 9, sigma=12)
    for sub in (0, 1, 2):
        b = io.BytesIO()
        Image.fromarray(rgb).save(b, "JPEG", quality=80, subsampling=sub)
        data = b.getvalue()
        f_or, c_or, q_or = oracle.parse_and_decode(data)
        f, c, q = M.entropy_decode(data, n_threads=2)
        assert f == f_or and np.array_equal(c, c_or) and np.array_equal(q, q_or)
    b = io.BytesIO()
    Image.fromarray(rgb).save(b, "JPEG", quality=80, progressive=True)
    with pytest.raises(M.MjdError) as ei:
        M.mjd_parse(b.getvalue())
    assert ei.value.code == -2
    # a libjpeg-written grayscale file: one component, one block per MCU;
    # its coefficients through the variant oracle land within a level of
    # libjpeg's own decode (the IDCT factorisations differ)
    import oracle.variants as V
    b = io.BytesIO()
    Image.fromarray(rgb[..., 0]).save(b, "JPEG", quality=80)
    f, c, q = M.entropy_decode(b.getvalue(), n_threads=2)
    assert f.get("ncomp") == 1 and c.shape == (-(-97 // 8) * -(-61 // 8), 64)
    ours = V.decode_variant(f, c, q, "islow").astype(np.int64)
    theirs = np.asarray(Image.open(io.BytesIO(b.getvalue()))).astype(np.int64)
    assert ours.shape == theirs.shape == (61, 97)
    assert np.abs(ours - theirs).max() <= 1


def _with_16bit_dqt(data: bytes, value_of=lambda v: v) -> bytes:
    """The stream with its first DQT table rewritten with Pq = 1 (16-bit
    entries, big-endian), each entry mapped by value_of."""
    i = data.index(b"\xFF\xDB")
    seglen = (data[i + 2] << 8) | data[i + 3]
    seg = data[i + 4:i + 2 + seglen]
    tq, vals, rest = seg[0] & 15, seg[1:65], seg[65:]
    wide = bytes([0x10 | tq]) + b"".join(int(value_of(v)).to_bytes(2, "big") for v in vals)
    body = wide + rest
    return data[:i] + b"\xFF\xDB" + (len(body) + 2).to_bytes(2, "big") + body + data[i + 2 + seglen:]


def test_16bit_quant_tables_are_refused(M):
    # T.81 B.2.4.1: Pq = 1 only with 12-bit samples; an 8-bit stream carrying
    # one is corrupt, whatever its values (small ones included)
    frame, coef, qt, data = _stream(24, 16, "420", 75, 0)
    for value_of in (lambda v: v, lambda v: 300 + v):
        bad = _with_16bit_dqt(data, value_of)
        assert oracle.parse_and_decode(bad)[0] == frame   # the oracle's reader still parses the layout
        with pytest.raises(M.MjdError) as ei:
            M.mjd_parse(bad)
        assert ei.value.code == -5 and "16-bit" in str(ei.value)


def _intervals(M, data):
    scan, _ = M.mjd_parse(data)
    off = M.mjd_restart_index(data, scan)
    return scan, [int(o) for o in off]


@pytest.mark.parametrize("samp,ri", [("420", 2), ("444", 5), ("422", 1)])
def test_corrupt_interval_is_cleared_and_the_rest_decodes(M, samp, ri):
    # Interval k's entropy-coded bytes replaced by all-ones (0xFF stuffed
    # as 0xFF 0x00): no valid code is sixteen 1-bits, so it is corrupt from
    # its first code.  The restart marker after it resynchronises the
    # decoder: every other interval decodes to the encoded coefficients,
    # interval k's MCUs come back as zero blocks, and MJD_ECORRUPT names k.
    frame, coef, qt, data = _stream(70, 45, samp, 80, ri, seed=11)
    scan, off = _intervals(M, data)
    g = geometry(frame)
    per_mcu = g["blocks_per_mcu"]
    n_int = scan.n_intervals
    for k in sorted({0, n_int // 2, n_int - 1}):
        bad = bytearray(data)
        a, b = off[k], off[k + 1] - 2
        fill = (b"\xFF\x00" * ((b - a) // 2 + 1))[:b - a]
        if fill.endswith(b"\xFF"):
            fill = fill[:-1] + b"\x00"
        bad[a:b] = fill
        for threads in (1, 3):
            with pytest.raises(M.MjdError) as ei:
                M.entropy_decode(bytes(bad), n_threads=threads)
            assert ei.value.code == -5 and f"interval {k}" in str(ei.value)
            c = np.full_like(coef.reshape(-1, 64), 0x5A5A)
            rc_err = None
            try:
                M.mjd_entropy_decode(bytes(bad), scan, None, c, 0, g["mcus_y"], threads)
            except M.MjdError as e:
                rc_err = e.code
            assert rc_err == -5
            want = coef.reshape(-1, 64).copy()
            m0, m1 = k * ri, min((k + 1) * ri, g["mcus_x"] * g["mcus_y"])
            want[m0 * per_mcu:m1 * per_mcu] = 0
            assert np.array_equal(c, want)


def test_two_corrupt_intervals_report_the_first(M):
    frame, coef, qt, data = _stream(64, 48, "420", 80, 1, seed=12)
    scan, off = _intervals(M, data)
    bad = bytearray(data)
    for k in (5, 2):
        a, b = off[k], off[k + 1] - 2
        bad[a:b] = (b"\xFF\x00" * (b - a))[:b - a] if (b - a) % 2 == 0 else (b"\xFF\x00" * (b - a))[:b - a - 1] + b"\x00"
    with pytest.raises(M.MjdError) as ei:
        M.entropy_decode(bytes(bad), n_threads=4)
    assert "interval 2" in str(ei.value)
