"""GPU parity of the entropy kernel (one lane per restart interval): every
job of a mixed batch decodes to exactly the coefficients the oracle's reader
(T.81 Annex F.2.2, bit by bit) finds in the stream and the encoder put in
it; corrupt data is reported for the right job without touching the others;
a whole bitstream decodes to RGB on the device through the entropy kernel
and the fused back half, bit-exact against the oracle."""
import random

import numpy as np
import pytest

import oracle
from synth import bitstream, encode, images

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

SENTINEL = 0x5A5A


def say(msg):
    print(f"[gpu-entropy] {msg}", flush=True)


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


# (width, height, sampling, quality, restart interval): tiny and ragged
# frames, every sampling, one MCU per interval, odd intervals, no markers
SPECS = [(257, 190, "420", 85, 32), (64, 64, "420", 75, 0), (333, 47, "422", 90, 3), (100, 121, "444", 60, 1),
         (17, 300, "420", 95, 5), (1, 1, "420", 50, 0), (200, 33, "422", 70, 2), (640, 480, "444", 85, 1),
         (999, 17, "420", 80, 7)]


@pytest.fixture(scope="module")
def streams():
    out = []
    for i, (w, h, samp, q, ri) in enumerate(SPECS):
        rgb = images.texture_rgb(w, h, 200 + i, sigma=12)
        frame, coef, qt = encode.encode_rgb(rgb, samp, q)
        out.append((frame, coef, qt, bitstream.write_jpeg(frame, coef, qt, restart_interval=ri)))
    return out


def device_job(M, data):
    scan, qt = M.mjd_parse(data)
    off = M.mjd_restart_index(data, scan)
    # the kernel reads the stream in 16-byte chunks: pad the buffer to 16
    d_jpg = torch.zeros(-(-len(data) // 16) * 16, dtype=torch.uint8, device="cuda")
    d_jpg[:len(data)] = torch.from_numpy(np.frombuffer(data, dtype=np.uint8).copy()).cuda()
    n_blocks = M.mjd_geometry_of(M.scan_frame(scan))["n_blocks"]
    d_coef = torch.full((n_blocks * 64,), SENTINEL, dtype=torch.int16, device="cuda")
    return (scan, off, d_jpg, len(data), d_coef), qt


def test_batch_matches_oracle_reader(M, ctx, streams):
    jobs = [device_job(M, data)[0] for *_, data in streams]
    say(f"one entropy batch of {len(jobs)} jobs")
    b = M.EntropyBatch(ctx, jobs)
    info = b.info()
    assert info["intervals"] == sum(j[0].n_intervals for j in jobs)
    for rep in range(2):  # the second launch finds the queue rearmed
        for j in jobs:
            j[4].fill_(SENTINEL)
        b.launch()
        assert b.status() == -1
        for i, ((frame, coef, qt, data), j) in enumerate(zip(streams, jobs)):
            _, c_or, _ = oracle.parse_and_decode(data)
            got = j[4].cpu().numpy().reshape(-1, 64)
            assert np.array_equal(got, c_or), (rep, i)
            assert np.array_equal(got, coef), (rep, i)
    b.close()


def test_jobs_in_separate_batches_and_orders(M, ctx, streams):
    """The same jobs, one batch each and in reverse order within one batch."""
    exp = [coef for _, coef, _, _ in streams]
    for order in (list(range(len(streams))), list(reversed(range(len(streams))))):
        jobs = [device_job(M, streams[i][3])[0] for i in order]
        b = M.EntropyBatch(ctx, jobs)
        b.launch()
        b.status()
        for i, j in zip(order, jobs):
            assert np.array_equal(j[4].cpu().numpy().reshape(-1, 64), exp[i]), i
        b.close()
    for i in (0, 5, 7):
        j = device_job(M, streams[i][3])[0]
        b = M.EntropyBatch(ctx, [j])
        b.launch()
        b.status()
        b.close()
        assert np.array_equal(j[4].cpu().numpy().reshape(-1, 64), exp[i]), i


def _rejected_mutation(M, data, seed):
    """A copy of `data` with entropy-coded bytes replaced that the host
    decoder rejects (markers and stuffing untouched)."""
    scan, _ = M.mjd_parse(data)
    off = M.mjd_restart_index(data, scan)
    g = M.mjd_geometry_of(M.scan_frame(scan))
    rnd = random.Random(seed)
    for _ in range(200):
        b = bytearray(data)
        for _ in range(4):
            p = rnd.randrange(scan.data_offset, scan.data_end)
            if b[p] != 0xFF and b[p - 1] != 0xFF:
                b[p] = rnd.randrange(255)
        try:
            M.mjd_entropy_decode(bytes(b), scan, off, np.zeros((g["n_blocks"], 64), np.int16), 0, g["mcus_y"], 1)
        except M.MjdError as e:
            if e.code == -5:
                return bytes(b)
    raise AssertionError("no rejected mutation found")


def test_corrupt_job_is_reported_and_others_decode(M, ctx, streams):
    bad = _rejected_mutation(M, streams[2][3], seed=3)
    datas = [streams[0][3], bad, streams[3][3]]
    jobs = [device_job(M, d)[0] for d in datas]
    say("batch with a corrupt middle job")
    b = M.EntropyBatch(ctx, jobs)
    b.launch()
    with pytest.raises(M.MjdError) as ei:
        b.status()
    assert ei.value.code == -5 and ei.value.bad_job == 1
    assert np.array_equal(jobs[0][4].cpu().numpy().reshape(-1, 64), streams[0][1])
    assert np.array_equal(jobs[2][4].cpu().numpy().reshape(-1, 64), streams[3][1])
    b.close()
    # a truncated stream (one interval, its last 6 bytes gone): more bits
    # are needed than the interval holds
    frame, coef, qt, data = streams[1]
    scan, _ = M.mjd_parse(data)
    assert scan.n_intervals == 1
    cut = data[:scan.data_end - 6] + data[scan.data_end:]
    j = device_job(M, cut)[0]
    b = M.EntropyBatch(ctx, [j])
    b.launch()
    with pytest.raises(M.MjdError) as ei:
        b.status()
    assert ei.value.code == -5 and ei.value.bad_job == 0
    b.close()


def _segments(d):
    out, i = [], 2
    while i < len(d):
        m, L = d[i + 1], d[i + 2] << 8 | d[i + 3]
        out.append((m, i, L))
        if m == 0xDA:
            break
        i += 2 + L
    return out


def _six_tables(d):
    """The same scan with its third component on copies (id 2) of the chroma
    DC and AC tables: six distinct tables, valid for the host decoder."""
    segs = _segments(d)
    extra = b""
    for m, i, L in segs:
        if m == 0xC4 and d[i + 4] in (0x01, 0x11):
            pay = bytearray(d[i + 4:i + 2 + L])
            pay[0] = (pay[0] & 0xF0) | 2
            extra += b"\xFF\xC4" + (len(pay) + 2).to_bytes(2, "big") + bytes(pay)
    m, i, L = segs[-1]
    sos = bytearray(d[i:i + 2 + L])
    sos[10] = 0x22  # component 3: DC 2, AC 2
    return d[:i] + extra + bytes(sos) + d[i + 2 + L:]


def test_dense_random_streams(M, ctx):
    """Random large coefficients: long codes, many stuffed bytes and dense
    intervals in which lanes outrun their stream ring and wait for it."""
    rng = np.random.default_rng(17)
    qt = np.ones((4, 64), dtype=np.uint16)
    jobs, exp = [], []
    for samp, w, h, ri in (("420", 160, 96, 1), ("422", 120, 40, 3), ("444", 72, 56, 0), ("420", 200, 120, 2)):
        fr = encode.make_frame(w, h, samp)
        nb = oracle.geometry(fr)["n_blocks"]
        size = np.minimum(rng.geometric(0.3, size=(nb, 64)), 10)
        mag = (1 << (size - 1)) + (rng.random((nb, 64)) * (1 << (size - 1))).astype(np.int64)
        c = np.where(rng.random((nb, 64)) < 0.5, -mag, mag).astype(np.int16)
        c[:, 0] = rng.integers(-1023, 1024, size=nb)
        c[rng.random((nb, 64)) < 0.2] = 0
        data = bitstream.write_jpeg(fr, c, qt, restart_interval=ri)
        assert data.count(b"\xFF\x00") > 10
        jobs.append(device_job(M, data)[0])
        exp.append(c)
    b = M.EntropyBatch(ctx, jobs)
    b.launch()
    b.status()
    for j, c in zip(jobs, exp):
        assert np.array_equal(j[4].cpu().numpy().reshape(-1, 64), c)
    b.close()


def test_scan_with_more_than_four_tables_is_refused(M, ctx, streams):
    data = _six_tables(streams[0][3])
    scan, _ = M.mjd_parse(data)
    assert len({(0, x) for x in scan.dc_sel} | {(1, x) for x in scan.ac_sel}) == 6
    with pytest.raises(M.MjdError) as ei:
        M.EntropyBatch(ctx, [device_job(M, data)[0]])
    assert ei.value.code == -2


def test_create_rejects_bad_jobs(M, ctx, streams):
    data = streams[0][3]
    j, _ = device_job(M, data)
    scan, off, d_jpg, n, d_coef = j
    with pytest.raises(M.MjdError) as ei:   # stream not 4-byte aligned
        M.EntropyBatch(ctx, [(scan, off, d_jpg[1:], n - 1, d_coef)])
    assert ei.value.code == -1
    bad_off = off.copy()
    bad_off[-1] = n + 10                    # restart index past the stream
    with pytest.raises(M.MjdError) as ei:
        M.EntropyBatch(ctx, [(scan, bad_off, d_jpg, n, d_coef)])
    assert ei.value.code == -1
    with pytest.raises(M.MjdError) as ei:
        M.EntropyBatch(ctx, [])
    assert ei.value.code == -1


@pytest.mark.parametrize("mode", ["fancy", "simple"])
def test_bitstreams_to_rgb_on_the_device(M, ctx, streams, mode):
    """Entropy kernel then the batched back half, all on the device."""
    jobs, qts = [], []
    for *_, data in streams:
        j, qt = device_job(M, data)
        jobs.append(j)
        qts.append(torch.from_numpy(qt.view(np.int16)).cuda())
    eb = M.EntropyBatch(ctx, jobs)
    outs = []
    djobs = []
    for (frame, coef, qt, data), j, q in zip(streams, jobs, qts):
        o = torch.full((frame["height"], frame["width"], 3), 3, dtype=torch.uint8, device="cuda")
        djobs.append((frame, j[4], q, o, 3 * frame["width"]))
        outs.append(o)
    db = M.Batch(ctx, djobs, M.UPSAMPLE[mode])
    eb.launch()
    db.launch()
    eb.status()
    torch.cuda.synchronize()
    for (frame, coef, qt, data), o in zip(streams, outs):
        f, c, q = oracle.parse_and_decode(data)
        assert np.array_equal(o.cpu().numpy(), oracle.decode(f, c, q, mode)), frame
    db.close()
    eb.close()


def test_corpus_size_image(M, ctx):
    """A 4000x3000 4:2:0 stream with a marker every 32 MCUs (the corpus's
    largest kind): every coefficient equals the encoder's."""
    from synth import fast_bitstream, gpu_encode
    frame, c, qt = gpu_encode.batch_image_gpu(torch, (4000, 3000, "420", 85, 77), "cuda", sigma=12.0,
                                              content="texture")
    coef = c.cpu().numpy()
    data = fast_bitstream.write_jpeg(frame, coef, qt, 32)
    say(f"4000x3000 stream of {len(data)} bytes")
    j, _ = device_job(M, data)
    b = M.EntropyBatch(ctx, [j])
    b.launch()
    b.status()
    assert torch.equal(j[4], c.to(torch.int16))
    b.close()
