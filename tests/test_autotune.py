"""The launch-shape autotuner: interior test, cache keys and round trip on
the CPU; on the GPU, a search that stores its winner and a second lookup
that is served from the cache (and decodes bit-exactly with it)."""
import json
import os

import numpy as np
import pytest

from paper_1311_5304_amd import autotune


def test_interior_is_strict_on_each_axis():
    table = [{"seg_subtiles": s, "workgroups_per_cu": k} for s in (1, 2, 4) for k in (1, 2, 3)]
    assert autotune.interior({"seg_subtiles": 2, "workgroups_per_cu": 2}, table, "seg_subtiles")
    assert not autotune.interior({"seg_subtiles": 1, "workgroups_per_cu": 2}, table, "seg_subtiles")
    assert not autotune.interior({"seg_subtiles": 4, "workgroups_per_cu": 2}, table, "seg_subtiles")
    assert not autotune.interior({"seg_subtiles": 2, "workgroups_per_cu": 3}, table, "workgroups_per_cu")
    # fewer than three values searched: nothing is interior
    assert not autotune.interior({"seg_subtiles": 2}, [{"seg_subtiles": 2}, {"seg_subtiles": 3}], "seg_subtiles")


def test_refine_picks_the_fastest_retimed_row():
    table = [{"id": i, "ms": ms} for i, ms in enumerate((5.0, 1.0, 1.1, 1.2, 9.0))]
    retimed = {1: 1.3, 2: 1.05, 3: 1.2}
    best = autotune._refine(table, lambda r, n: retimed[r["id"]], 50, 3)
    assert best["id"] == 2
    assert "ms_refined" not in table[0] and "ms_refined" not in table[4]


def test_cache_round_trip_and_key(tmp_path):
    path = tmp_path / "cache.json"
    c = autotune.TuneCache(str(path))
    frame = {"width": 4096, "height": 3072, "h": (2, 1, 1), "v": (2, 1, 1)}
    key = autotune.TuneCache.key("gpu-x", autotune.TuneCache.image_workload(frame, 1))
    assert "gpu-x" in key and autotune.kernel_hash()[:16] in key and "h2v2_w2^12_h2^11" in key
    assert c.get(key) is None
    c.put(key, {"seg_subtiles": 3, "workgroups": 512, "shape": 1})
    again = autotune.TuneCache(str(path))
    assert again.get(key) == {"seg_subtiles": 3, "workgroups": 512, "shape": 1}
    assert json.loads(path.read_text())[key]["shape"] == 1


def test_image_launch_matches_the_launcher_arithmetic():
    g = {"mcus_x": 256, "mcus_y": 192}
    shape = {"mcus_x": 16, "mcus_y": 2, "resident_per_cu": 2, "cu_count": 256}
    assert autotune.image_launch(g, shape, 3, 0) == (512, 512)        # 16 strips x 32 segments
    assert autotune.image_launch(g, shape, 1, 1024) == (1536, 1024)   # more workgroups than resident
    assert autotune.image_launch(g, shape, 3, 1024) == (512, 512)     # capped at the segments
    assert autotune.image_launch(g, shape, 500, 0) == (16, 16)        # one segment per strip
    g = {"mcus_x": 33, "mcus_y": 28}
    assert autotune.image_launch(g, shape, 5, 256) == (3 * 3, 16)     # rounded up to a multiple of 8


def test_kernel_hash_covers_every_listed_source():
    for f in autotune.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(autotune.PKG, "csrc", f)), f
    assert len(autotune.kernel_hash()) == 64


@pytest.mark.gpu
def test_tuned_then_cached(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import paper_1311_5304_amd as M
    from synth import encode, images

    print("[autotune] 1000x700 4:2:0 fancy: search, then cache", flush=True)
    rgb = images.texture_rgb(1000, 700, 3, sigma=10)
    frame, coef, qt = encode.encode_rgb(rgb, "420", 88)
    exp = oracle.decode(frame, coef, qt, "fancy")
    ctx = M.Context(0)
    try:
        c = [torch.from_numpy(coef).cuda() for _ in range(2)]
        q = torch.from_numpy(qt.view(np.int16)).cuda()
        o = [torch.empty((700, 1000, 3), dtype=torch.uint8, device="cuda") for _ in range(2)]
        cache = autotune.TuneCache(str(tmp_path / "t.json"))
        e1, src1 = autotune.tuned_image(ctx, frame, M.MJD_UPSAMPLE_FANCY, c, q, o, cache=cache)
        assert src1 == "tuned"
        n_shapes = M.mjd_shape_count(2, 2, M.MJD_UPSAMPLE_FANCY)
        # every distinct launch once (asking more workgroups than segments repeats a launch)
        assert n_shapes * len(autotune.SEG_CANDIDATES) <= e1["candidates"] <= \
            n_shapes * len(autotune.WG_PER_CU) * len(autotune.SEG_CANDIDATES)
        keys = {(r["shape"], r["seg_subtiles"], r["launched"]) for r in e1["table"]}
        assert len(keys) == e1["candidates"]
        assert e1["ranges"]["seg_subtiles"] == sorted(autotune.SEG_CANDIDATES)
        M.mjd_ctx_set_tuning(ctx, 0, 0, 0)
        e2, src2 = autotune.tuned_image(ctx, frame, M.MJD_UPSAMPLE_FANCY, c, q, o,
                                        cache=autotune.TuneCache(cache.path))
        assert src2 == "cache"
        t = M.mjd_ctx_get_tuning(ctx)
        assert (t["seg_subtiles"], t["workgroups"], t["shape"]) == (e1["seg_subtiles"], e1["workgroups"],
                                                                     e1["shape"])
        out = M.decode(ctx, frame, c[0], q, "fancy")
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), exp)
    finally:
        ctx.close()
