"""GPU: the no-allocation batch entry point (mjd_decode_batch_noalloc), called
through the C ABI, against the allocating batch path (mjd_batch_create +
direct launch) on the same inputs, byte for byte, over two calls in a row
(the second with a smaller batch, so stale scratch contents would show), and
the rejection of a batch whose tables exceed the fixed scratch."""
import numpy as np
import pytest

import oracle
from synth import encode, images, workloads

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-noalloc] {msg}", flush=True)


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


def _inputs(n, workload_id):
    specs = workloads.batch_specs(n=n, lo=17, hi=520, workload_id=workload_id)
    out = []
    for w, h, samp, q, seed in specs:
        rgb = images.gradient_rgb(w, h, seed, sigma=8)
        out.append(encode.encode_rgb(rgb, samp, q))
    return out


def _jobs(inputs, fill):
    jobs, outs = [], []
    for frame, coef, qt in inputs:
        c = torch.from_numpy(coef).cuda()
        q = torch.from_numpy(qt.view(np.int16)).cuda()
        o = torch.full((frame["height"], frame["width"], 3), fill, dtype=torch.uint8, device="cuda")
        jobs.append((frame, c, q, o, 3 * frame["width"]))
        outs.append(o)
    return jobs, outs


def _allocating(M, ctx, jobs, upsample):
    b = M.mjd_batch_create(ctx, jobs, upsample)
    try:
        M.mjd_batch_launch(b, use_graph=False)
        torch.cuda.synchronize()
    finally:
        M.mjd_batch_destroy(b)


@pytest.mark.parametrize("mode", ["fancy", "simple"])
def test_noalloc_matches_allocating_batch_twice(M, ctx, mode):
    up = M.UPSAMPLE[mode]
    for call, (n, wid) in enumerate(((14, 31), (5, 32))):  # the second batch is smaller
        inputs = _inputs(n, wid)
        say(f"{mode} call {call}: {n} images")
        ref_jobs, ref_outs = _jobs(inputs, 11)
        _allocating(M, ctx, ref_jobs, up)
        jobs, outs = _jobs(inputs, 29)
        M.mjd_decode_batch_noalloc(ctx, jobs, up)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(ref_outs, outs)):
            assert torch.equal(a, b), f"{mode} call {call} image {i}: no-allocation output differs"
        # and one image of each call against the oracle
        f, c, q = inputs[0]
        assert np.array_equal(outs[0].cpu().numpy(), oracle.decode(f, c, q, mode)), "differs from the oracle"


def test_noalloc_rejects_tables_beyond_the_scratch(M, ctx):
    # 60000 tiny images (their views alone exceed 4 MiB); every job may share
    # one set of buffers, since nothing is enqueued
    frame = encode.make_frame(8, 8, "444")
    c = torch.zeros(3 * 64, dtype=torch.int16, device="cuda")
    q = torch.ones(4 * 64, dtype=torch.int16, device="cuda")
    o = torch.full((8, 8, 3), 77, dtype=torch.uint8, device="cuda")
    jobs = [(frame, c, q, o, 24)] * 60000
    with pytest.raises(M.MjdError) as ei:
        M.mjd_decode_batch_noalloc(ctx, jobs, M.MJD_UPSAMPLE_FANCY)
    assert "4194304" in str(ei.value) or "at most" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((o == 77).all()), "a rejected call wrote output"
