"""GPU parity at the full sizes of the batch and serving workloads: images of
320..4096 px (widths and heights not multiples of 16, plus 4095- and
4096-wide ones) of all three samplings, quality 50..95 with per-image
tables, decoded by one persistent batch launch under the planner's segment
length, the autotuner's usual choice (12 sub-tiles) and a longer one; and a
serving mix that holds requests of 4 MP and more.  Small images are compared
with the oracle whole; large ones on MCU-row bands the oracle decodes from
the band and one neighbour row on each side (all a band depends on)."""
import numpy as np
import pytest

import oracle
from synth import gpu_encode, workloads

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

WHOLE_MAX_PIXELS = 700_000


def say(msg):
    print(f"[gpu-full-size] {msg}", flush=True)


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


def _specs():
    specs = list(workloads.batch_specs(n=12, lo=320, hi=4096, workload_id=21))
    # the widest frames: one not a multiple of 16, one exactly 4096
    specs[0] = (4095, 1203, "420", 90, 7001)
    specs[1] = (4096, 777, "422", 61, 7002)
    specs[2] = (4095, 333, "444", 77, 7003)
    return specs


@pytest.fixture(scope="module")
def images_gpu():
    dev = torch.device("cuda:0")
    out = []
    for spec in _specs():
        frame, coef, qt = gpu_encode.batch_image_gpu(torch, spec, dev, sigma=8.0)
        out.append((frame, coef, torch.from_numpy(qt.view(np.int16)).to(dev), qt, coef.cpu().numpy().reshape(-1, 64)))
    torch.cuda.synchronize()
    return out


def oracle_rows(frame, coef_host, qt, mode, r0, r1):
    """Oracle RGB of MCU rows [r0, r1) from those rows and one neighbour row on each side."""
    g = oracle.geometry(frame)
    mh, H = g["mcu_h"], frame["height"]
    per_row = g["mcus_x"] * g["blocks_per_mcu"]
    a, b = max(r0 - 1, 0), min(r1 + 1, g["mcus_y"])
    sub = dict(frame, height=min(H, b * mh) - a * mh)
    rgb = oracle.decode(sub, coef_host[a * per_row:b * per_row], qt, mode)
    y0, y1 = r0 * mh, min(H, r1 * mh)
    return rgb[y0 - a * mh:y1 - a * mh], (y0, y1)


def check_image(got, frame, coef_host, qt, mode, what):
    W, H = frame["width"], frame["height"]
    if W * H <= WHOLE_MAX_PIXELS:
        exp = oracle.decode(frame, coef_host, qt, mode)
        assert np.array_equal(got, exp), f"{what}: whole image differs"
        return
    g = oracle.geometry(frame)
    n = g["mcus_y"]
    for r0, r1 in ((0, 2), (n // 2 - 1, n // 2 + 1), (n - 2, n)):
        exp, (y0, y1) = oracle_rows(frame, coef_host, qt, mode, max(r0, 0), min(r1, n))
        assert np.array_equal(got[y0:y1], exp), f"{what}: MCU rows {r0}..{r1} differ"


@pytest.mark.parametrize("seg", [0, 12, 24])
def test_full_size_batch_bit_exact(M, ctx, images_gpu, seg):
    mode = "fancy"
    jobs, outs = [], []
    for frame, c, q, _, _ in images_gpu:
        o = torch.full((frame["height"], frame["width"], 3), 13, dtype=torch.uint8, device="cuda")
        jobs.append((frame, c, q, o, 3 * frame["width"]))
        outs.append(o)
    M.mjd_ctx_set_tuning(ctx, seg, 0)
    try:
        b = M.mjd_batch_create(ctx, jobs, M.UPSAMPLE[mode])
        try:
            say(f"segment length {seg}: {b.info()}")
            M.mjd_batch_launch(b, use_graph=True)
            M.mjd_batch_launch(b, use_graph=True)  # a replay rewrites the same bytes
            torch.cuda.synchronize()
        finally:
            M.mjd_batch_destroy(b)
    finally:
        M.mjd_ctx_set_tuning(ctx, 0, 0)
    for i, ((frame, _, _, qt, ch), o) in enumerate(zip(images_gpu, outs)):
        check_image(o.cpu().numpy(), frame, ch, qt, mode, f"seg {seg} image {i} {frame['width']}x{frame['height']}")


def test_serving_mix_with_large_requests(M, ctx, images_gpu):
    """Continuous batching over requests that include 4 MP and larger ones:
    every result equals the oracle, alone and in the mix."""
    reqs = []
    big = 0
    for frame, c, q, qt, ch in images_gpu:
        reqs.append((frame, c.cpu().pin_memory(), q.cpu().pin_memory(), qt, ch))
        big += frame["width"] * frame["height"] >= 4_000_000
    assert big >= 1, "the mix has no request of 4 MP or more"
    srv = M.Server(ctx, 1 << 30, M.MJD_UPSAMPLE_FANCY, max_batch=16, max_inflight=2)
    try:
        outs = [torch.full((f["height"], f["width"], 3), 1, dtype=torch.uint8).pin_memory() for f, *_ in reqs]
        t0 = srv.now_ns()
        ids = [srv.submit(f, c, q, o, 3 * f["width"], t0 + 20_000 * i)
               for i, ((f, c, q, _, _), o) in enumerate(zip(reqs, outs))]
        times = [srv.wait(i) for i in ids]
        assert all(t["status"] == 0 for t in times)
        say(f"batches: {[t['batch'] for t in times]}")
        for i, ((f, _, _, qt, ch), o) in enumerate(zip(reqs, outs)):
            check_image(o.numpy(), f, ch, qt, "fancy", f"served {i} {f['width']}x{f['height']}")
    finally:
        srv.close()
