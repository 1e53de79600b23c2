"""GPU tests of the serving loop: requests of mixed sizes and samplings,
decoded alone and in a continuous-batching mix (arrivals overlapping device
work, admission limited by the device budget), give the same bytes as each
other and as the oracle; the synchronous server too."""
import numpy as np
import pytest

import oracle
from synth import encode, images, workloads

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-server] {msg}", flush=True)


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
def requests():
    specs = workloads.batch_specs(n=24, lo=9, hi=520, workload_id=12)
    out = []
    for w, h, samp, q, seed in specs:
        rgb = images.gradient_rgb(w, h, seed, sigma=8)
        frame, coef, qt = encode.encode_rgb(rgb, samp, q)
        out.append((frame, torch.from_numpy(coef.reshape(-1)).pin_memory(),
                    torch.from_numpy(qt.view(np.int16).reshape(-1)).pin_memory(), coef, qt))
    return out


def expected(requests, mode):
    return [oracle.decode(f, c, q, mode) for f, _, _, c, q in requests]


def outputs(requests):
    return [torch.full((f["height"], f["width"], 3), 1, dtype=torch.uint8).pin_memory() for f, *_ in requests]


def need(frame):
    g = oracle.geometry(frame)
    return g["n_blocks"] * 128 + 512 + -(-3 * frame["width"] // 16) * 16 * frame["height"] + 1024


def check_times(t):
    assert t["status"] == 0
    assert t["arrival_ns"] <= t["admit_ns"] <= t["launch_ns"] <= t["done_ns"]
    assert t["batch"] >= 1


@pytest.mark.parametrize("mode", ["fancy", "simple"])
def test_alone_and_in_the_mix_are_identical(M, ctx, requests, mode):
    exp = expected(requests, mode)
    srv = M.Server(ctx, 256 << 20, M.UPSAMPLE[mode], max_batch=64, max_inflight=2)
    try:
        say(f"{mode}: alone")
        alone = outputs(requests)
        for (f, c, q, _, _), o in zip(requests, alone):
            rid = srv.submit(f, c, q, o, 3 * f["width"])
            t = srv.wait(rid)
            check_times(t)
            assert t["batch"] == 1
        say(f"{mode}: mix")
        mix = outputs(requests)
        t0 = srv.now_ns()
        ids = [srv.submit(f, c, q, o, 3 * f["width"], t0 + 5_000 * i)
               for i, ((f, c, q, _, _), o) in enumerate(zip(requests, mix))]
        times = [srv.wait(i) for i in ids]
        for t in times:
            check_times(t)
        assert max(t["batch"] for t in times) > 1, "no request shared a batch"
        for i, (a, m, e) in enumerate(zip(alone, mix, exp)):
            assert np.array_equal(a.numpy(), e), i
            assert np.array_equal(m.numpy(), a.numpy()), i
    finally:
        srv.close()


def test_budget_admission_serialises_without_changing_results(M, ctx, requests):
    exp = expected(requests, "fancy")
    budget = int(1.2 * max(need(f) for f, *_ in requests))
    srv = M.Server(ctx, budget, M.MJD_UPSAMPLE_FANCY, max_batch=8, max_inflight=3)
    try:
        outs = outputs(requests)
        ids = [srv.submit(f, c, q, o, 3 * f["width"]) for (f, c, q, _, _), o in zip(requests, outs)]
        times = [srv.wait(i) for i in ids]
        admits = [t["admit_ns"] for t in times]
        assert admits == sorted(admits)  # admission keeps submission order
        for t in times:
            check_times(t)
        for o, e in zip(outs, exp):
            assert np.array_equal(o.numpy(), e)
    finally:
        srv.close()


def test_model_caps_the_predicted_batch_time(M, ctx, requests):
    """Batch sizing by the performance model: with every request predicted
    at 1 ms of GPU time and a 2.5 ms cap, no batch holds more than two
    requests, and the results do not change."""
    exp = expected(requests, "fancy")
    model = M.mjd_model()
    model.o_w.degree = model.t_kernel.degree = model.o_r.degree = 0
    model.o_w.c[0] = 1e-3
    assert M.mjd_model_predict(model, 100, 100, 0)["p_gpu"] == 1e-3
    srv = M.Server(ctx, 256 << 20, M.MJD_UPSAMPLE_FANCY, max_batch=64, max_inflight=1, model=model,
                   max_batch_s=2.5e-3)
    try:
        outs = outputs(requests)
        ids = [srv.submit(f, c, q, o, 3 * f["width"]) for (f, c, q, _, _), o in zip(requests, outs)]
        times = [srv.wait(i) for i in ids]
        for t in times:
            check_times(t)
        assert max(t["batch"] for t in times) == 2
        for o, e in zip(outs, exp):
            assert np.array_equal(o.numpy(), e)
    finally:
        srv.close()
    with pytest.raises(M.MjdError) as ei:
        M.Server(ctx, 256 << 20, M.MJD_UPSAMPLE_FANCY, model=model, max_batch_s=-1.0)
    assert ei.value.code == -1


def test_sync_server_and_padded_pitch(M, ctx, requests):
    exp = expected(requests, "fancy")
    srv = M.Server(ctx, 64 << 20, M.MJD_UPSAMPLE_FANCY, mode=M.MJD_SERVE_SYNC)
    try:
        outs = [np.full((f["height"], 3 * f["width"] + 5), 4, dtype=np.uint8) for f, *_ in requests]
        ids = [srv.submit(f, c, q, o, o.shape[1]) for (f, c, q, _, _), o in zip(requests, outs)]
        srv.drain()
        for i, o, e, (f, *_) in zip(ids, outs, exp, requests):
            t = srv.wait(i)
            check_times(t)
            assert t["batch"] == 1
            w = f["width"]
            assert np.array_equal(o[:, :3 * w].reshape(f["height"], w, 3), e)
            assert np.all(o[:, 3 * w:] == 4)
    finally:
        srv.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_device_outputs_match_host_outputs(M, ctx, requests, mode):
    """Requests whose RGB goes to device memory (written by the kernel, not
    copied back), mixed with host-output requests in one trace: both equal
    the oracle; a padded device pitch keeps its padding bytes."""
    exp = expected(requests, "fancy")
    srv = M.Server(ctx, 64 << 20, M.MJD_UPSAMPLE_FANCY, mode=mode, max_batch=8)
    try:
        outs, ids = [], []
        t0 = srv.now_ns() + 1_000_000
        for i, (f, c, q, _, _) in enumerate(requests):
            w, h = f["width"], f["height"]
            if i % 2 == 0:
                o = torch.full((h, 3 * w + 7), 6, dtype=torch.uint8, device="cuda")
                pitch = 3 * w + 7
            else:
                o = torch.full((h, w, 3), 1, dtype=torch.uint8).pin_memory()
                pitch = 3 * w
            say(f"device-output mix mode {mode} request {i} {w}x{h} {'device' if i % 2 == 0 else 'host'}")
            outs.append(o)
            ids.append(srv.submit(f, c, q, o, pitch, t0 + 20_000 * i))
        srv.drain()
        torch.cuda.synchronize()
        for i, (rid, o, e, (f, *_)) in enumerate(zip(ids, outs, exp, requests)):
            check_times(srv.wait(rid))
            w, h = f["width"], f["height"]
            got = o.cpu().numpy()
            if i % 2 == 0:
                assert np.array_equal(got[:, :3 * w].reshape(h, w, 3), e), i
                assert np.all(got[:, 3 * w:] == 6), i
            else:
                assert np.array_equal(got, e), i
    finally:
        srv.close()


def test_server_rejects_bad_requests(M, ctx, requests):
    f, c, q, _, _ = requests[0]
    srv = M.Server(ctx, 64 << 20, M.MJD_UPSAMPLE_FANCY)
    try:
        big = encode.make_frame(4000, 4000, "444")  # 96 MB of coefficients alone
        with pytest.raises(M.MjdError) as ei:
            srv.submit(big, c, q, np.zeros(1, np.uint8), 12000)
        assert ei.value.code == -6
        o = np.zeros((f["height"], f["width"], 3), np.uint8)
        with pytest.raises(M.MjdError):
            srv.submit(f, c, q, o, 3 * f["width"] - 1)
        import ctypes

        from paper_1311_5304_amd import _binding as B
        rid = ctypes.c_uint64()
        for h_rgb, d_rgb in ((None, None), (o.ctypes.data, o.ctypes.data)):  # no output, or both
            r = B.mjd_request(frame=B.make_frame(f), h_coef=c.data_ptr(), h_qt=q.data_ptr(), h_rgb=h_rgb,
                              d_rgb=d_rgb, pitch=3 * f["width"], arrival_ns=0)
            assert B.lib().mjd_server_submit(srv.handle, ctypes.byref(r), ctypes.byref(rid)) == B.MJD_EINVAL
        t = srv.now_ns()
        srv.wait(srv.submit(f, c, q, o, 3 * f["width"], t + 1000))
        with pytest.raises(M.MjdError):
            srv.submit(f, c, q, o, 3 * f["width"], t)  # earlier than the last arrival
    finally:
        srv.close()
