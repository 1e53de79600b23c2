"""GPU parity of the batched persistent launch: every image of a mixed batch
(sizes with partial MCUs, 4:4:4 / 4:2:2 / 4:2:0, per-image quant tables)
bit-exact against the oracle, through direct launches and hipGraph replays,
under several queue shapes."""
import numpy as np
import pytest

import oracle
from synth import encode, images, workloads

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-batch] {msg}", flush=True)


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


@pytest.fixture(scope="module")
def batch_inputs():
    specs = workloads.batch_specs(n=15, lo=17, hi=700, workload_id=9)
    out = []
    for spec in specs:
        w, h, samp, q, seed = spec
        rgb = images.gradient_rgb(w, h, seed, sigma=8)
        frame, coef, qt = encode.encode_rgb(rgb, samp, q)
        out.append((frame, coef, qt))
    return out


def _device_jobs(batch_inputs):
    jobs, outs = [], []
    for frame, coef, qt in batch_inputs:
        c = torch.from_numpy(coef).cuda()
        q = torch.from_numpy(qt.view(np.int16)).cuda()
        o = torch.full((frame["height"], frame["width"], 3), 3, dtype=torch.uint8, device="cuda")
        jobs.append((frame, c, q, o, 3 * frame["width"]))
        outs.append(o)
    return jobs, outs


@pytest.mark.parametrize("mode", ["fancy", "simple"])
def test_batch_matches_oracle(M, ctx, batch_inputs, mode):
    exp = [oracle.decode(f, c, q, mode) for f, c, q in batch_inputs]
    jobs, outs = _device_jobs(batch_inputs)
    # workgroups 2048: more than stay resident, the rest start as others leave
    for seg, wgs, graph in ((0, 0, False), (1, 0, False), (3, 8, False), (0, 0, True), (2, 16, True),
                            (1, 2048, False), (1, 2048, True)):
        M.mjd_ctx_set_tuning(ctx, seg, wgs)
        say(f"batch {mode} seg={seg} wgs={wgs} graph={graph}")
        b = M.Batch(ctx, jobs, M.UPSAMPLE[mode])
        M.mjd_ctx_set_tuning(ctx, 0, 0)
        try:
            for rep in range(2 if graph else 1):
                for o in outs:
                    o.fill_(3)
                b.launch(use_graph=graph)
                torch.cuda.synchronize()
                for i, (o, e) in enumerate(zip(outs, exp)):
                    got = o.cpu().numpy()
                    assert np.array_equal(got, e), f"image {i} {batch_inputs[i][0]} seg={seg} rep={rep}"
        finally:
            b.close()


@pytest.mark.parametrize("mode", ["fancy", "simple"])
def test_batch_rows_at_any_byte_address(M, ctx, batch_inputs, mode):
    """Every image written at a base 1..3 bytes past a 4-byte boundary with
    a padded pitch (3W + 1..5 bytes): whole units take dword stores at those
    unaligned addresses; every RGB byte equals the oracle's and no byte of
    the padding or around the image changes."""
    exp = [oracle.decode(f, c, q, mode) for f, c, q in batch_inputs]
    jobs, bufs, geo = [], [], []
    for i, (frame, coef, qt) in enumerate(batch_inputs):
        w, h = frame["width"], frame["height"]
        off, pitch = 1 + i % 3, 3 * w + 1 + i % 5
        buf = torch.full((h * pitch + off + 16,), 0xA5, dtype=torch.uint8, device="cuda")
        c = torch.from_numpy(coef).cuda()
        q = torch.from_numpy(qt.view(np.int16)).cuda()
        jobs.append((frame, c, q, buf.data_ptr() + off, pitch))
        bufs.append(buf)
        geo.append((off, pitch, w, h))
    say(f"batch {mode} at unaligned bases and pitches")
    b = M.Batch(ctx, jobs, M.UPSAMPLE[mode])
    try:
        b.launch()
        torch.cuda.synchronize()
    finally:
        b.close()
    for i, (buf, e, (off, pitch, w, h)) in enumerate(zip(bufs, exp, geo)):
        got = buf.cpu().numpy()
        rows = got[off:off + h * pitch].reshape(h, pitch)
        assert np.array_equal(rows[:, :3 * w].reshape(h, w, 3), e), (i, off, pitch)
        assert (rows[:, 3 * w:] == 0xA5).all() and (got[:off] == 0xA5).all() and (got[off + h * pitch:] == 0xA5).all(), \
            (i, off, pitch)


def test_batch_equals_per_image_calls(M, ctx, batch_inputs):
    jobs, outs = _device_jobs(batch_inputs)
    b = M.Batch(ctx, jobs, M.MJD_UPSAMPLE_FANCY)
    b.launch()
    torch.cuda.synchronize()
    batched = [o.cpu().numpy() for o in outs]
    b.close()
    for (frame, c, q, o, pitch), ref in zip(jobs, batched):
        o.fill_(0)
        M.decode(ctx, frame, c, q, "fancy", out=o)
    torch.cuda.synchronize()
    for o, ref in zip(outs, batched):
        assert np.array_equal(o.cpu().numpy(), ref)


def test_batch_rejects_bad_job(M, ctx, batch_inputs):
    jobs, _ = _device_jobs(batch_inputs[:3])
    frame, c, q, o, pitch = jobs[1]
    jobs[1] = (frame, c, q, o, 3 * frame["width"] - 1)
    with pytest.raises(M.MjdError) as ei:
        M.Batch(ctx, jobs, M.MJD_UPSAMPLE_FANCY)
    assert "job 1" in str(ei.value)
    with pytest.raises(M.MjdError):
        M.Batch(ctx, [], M.MJD_UPSAMPLE_FANCY)
