"""Launch-shape autotuner for the decode kernels.

The paper picks its work-group size per platform by profiling (Sec. 4.1 and
Sec. 5.1).  Here the free choices are, per sampling class:
  - the sub-tile shape of the single-image kernel (SX x SY MCUs, lanes per
    workgroup; the class's list comes from `mjd_shape_info`),
  - the number of workgroups launched, as a multiple of the compute units
    (below, at or above what stays resident),
  - the segment length (sub-tile rows a workgroup walks, prefetching the
    next while decoding the current).
None of them changes the output.  `tune()` / `tune_batch()` time every
candidate with HIP events on the caller's buffers; `TuneCache` keeps the
winner in a JSON file keyed by device, a hash of the kernel sources and the
workload class, so a second run takes it from the file without timing.
"""
from __future__ import annotations

import hashlib
import json
import math
import os

from . import _binding as B

PKG = os.path.dirname(os.path.abspath(__file__))
# sources the decode kernels are built from: a change to any of them
# invalidates every cached choice
KERNEL_SOURCES = ("segment.h", "decode_kernel.h", "aan.h", "decode.hip", "batch.hip", "mjd_internal.h", "mjd_common.h")
DEFAULT_CACHE = os.path.join(PKG, "tune_cache.json")

SEG_CANDIDATES = (1, 2, 3, 4, 6, 8, 12, 16)
WG_PER_CU = (1, 2, 3, 4)
BATCH_SEG_CANDIDATES = (1, 2, 3, 4, 6, 8, 12, 16, 24, 32)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(PKG, "csrc", f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def device_name(device: int = 0) -> str:
    """The device's architecture (without its feature flags) and compute-unit
    count: what a launch shape depends on.  (The marketing name is left out:
    it reads differently depending on the installed ID tables and tools.)"""
    import torch
    p = torch.cuda.get_device_properties(device)
    arch = getattr(p, "gcnArchName", "?").split(":")[0]
    return f"{arch}|{p.multi_processor_count}CU"


def _time_ms(fn, reps: int, warmup: int = 3) -> float:
    import torch
    for _ in range(warmup):
        fn()
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def interior(best: dict, table: list, axis: str) -> bool:
    """True when the winner's value on an ordered axis lies strictly inside
    the range searched on that axis."""
    vals = sorted({r[axis] for r in table})
    return len(vals) >= 3 and vals[0] < best[axis] < vals[-1]


def _refine(table, time_of, reps_top, top, rounds: int = 5):
    """Re-time the `top` fastest rows, interleaved over several rounds (so a
    drift of the clock hits every row alike), and keep each row's median;
    the winner is the row with the lowest median."""
    order = sorted(table, key=lambda r: r["ms"])[:top]
    runs = {id(r): [] for r in order}
    for _ in range(rounds):
        for r in order:
            runs[id(r)].append(time_of(r, max(1, reps_top // rounds)))
    for r in order:
        r["ms_refined"] = sorted(runs[id(r)])[len(runs[id(r)]) // 2]
    return min(order, key=lambda r: r["ms_refined"])


def image_launch(g, shape: dict, seg: int, workgroups: int) -> tuple:
    """(segments, workgroups launched) of the single-image kernel for MCU
    rows [0, mcus_y): the launcher's own arithmetic (segments of `seg`
    sub-tile rows of every strip, the grid capped at the segment count and
    rounded up to a multiple of 8)."""
    sx, sy = shape["mcus_x"], shape["mcus_y"]
    strips = -(-g["mcus_x"] // sx)
    sub_rows = -(-g["mcus_y"] // sy)
    seg_rows = min(seg, sub_rows) * sy
    segments = strips * -(-g["mcus_y"] // seg_rows)
    wg = workgroups if workgroups > 0 else shape["resident_per_cu"] * shape["cu_count"]
    return segments, (min(wg, segments) + 7) & ~7


def shapes(ctx, frame, mode: int) -> list:
    h, v = int(frame["h"][0]), int(frame["v"][0])
    return [B.mjd_shape_info(ctx, h, v, mode, i) for i in range(B.mjd_shape_count(h, v, mode))]


def tune(ctx, frame, coef_sets, qt, mode: int, out_sets, reps: int = 10, reps_top: int = 100, top: int = 6,
         seg_candidates=SEG_CANDIDATES, wg_per_cu=WG_PER_CU, shape_ids=None):
    """Time every (shape, workgroups per CU, seg_subtiles) of the
    single-image kernel on rotating buffer sets (so caches do not hold the
    working set), then re-time the fastest few.

    coef_sets / out_sets: lists of device tensors.  Returns (best, table):
    rows are dicts {shape, sx, sy, threads, resident_per_cu, seg_subtiles,
    workgroups (asked), segments, launched, workgroups_per_cu (launched per
    CU), ms[, ms_refined]}.  A candidate whose launch equals one already
    timed (more workgroups asked than there are segments) is skipped."""
    g = B.mjd_geometry_of(frame)
    w = int(frame["width"])
    shp = shapes(ctx, frame, mode)
    ids = range(len(shp)) if shape_ids is None else shape_ids
    saved = B.mjd_ctx_get_tuning(ctx)
    it = [0]

    def run():
        k = it[0] % len(coef_sets)
        it[0] += 1
        B.mjd_decode(ctx, frame, coef_sets[k], qt, mode, out_sets[k], 3 * w, 0, g["mcus_y"])

    def time_of(r, n):
        B.mjd_ctx_set_tuning(ctx, r["seg_subtiles"], r["workgroups"], r["shape"])
        return _time_ms(run, n)

    table = []
    seen = set()
    try:
        for si in ids:
            s = shp[si]
            for seg in seg_candidates:
                for k in wg_per_cu:
                    segments, launched = image_launch(g, s, seg, k * s["cu_count"])
                    if (si, seg, launched) in seen:
                        continue  # the same launch as a row already timed
                    seen.add((si, seg, launched))
                    r = {"shape": si, "sx": s["mcus_x"], "sy": s["mcus_y"], "threads": s["threads"],
                         "resident_per_cu": s["resident_per_cu"], "seg_subtiles": seg,
                         "workgroups": k * s["cu_count"], "segments": segments, "launched": launched,
                         "workgroups_per_cu": round(launched / s["cu_count"], 3)}
                    r["ms"] = time_of(r, reps)
                    table.append(r)
        best = _refine(table, time_of, reps_top, top)
    finally:
        B.mjd_ctx_set_tuning(ctx, saved["seg_subtiles"], saved["workgroups"], saved["shape"])
    return best, table


def tune_batch(ctx, jobs, mode: int, reps: int = 4, reps_top: int = 25, top: int = 4,
               seg_candidates=BATCH_SEG_CANDIDATES, wg_per_cu=WG_PER_CU, cu_count=None, use_graph: bool = True):
    """Plan the batch once per (seg_subtiles, workgroups per CU) and time its
    persistent launch, then re-time the fastest few.  Rows hold the
    workgroups asked and launched (per CU); a candidate whose plan equals
    one already timed is skipped.  Returns (best, table); the planned Batch
    objects are released."""
    if cu_count is None:
        import torch
        cu_count = torch.cuda.get_device_properties(0).multi_processor_count
    saved = B.mjd_ctx_get_tuning(ctx)

    def time_of(r, n):
        B.mjd_ctx_set_tuning(ctx, r["seg_subtiles"], r["workgroups"], 0)
        b = B.Batch(ctx, jobs, mode)
        try:
            info = b.info()
            r["segments"], r["launched"] = info["segments"], info["workgroups"]
            return _time_ms(lambda: b.launch(use_graph=use_graph), n, warmup=2)
        finally:
            b.close()

    table = []
    seen = set()
    try:
        for seg in seg_candidates:
            for k in wg_per_cu:
                r = {"seg_subtiles": seg, "workgroups": k * cu_count}
                B.mjd_ctx_set_tuning(ctx, seg, r["workgroups"], 0)
                b = B.Batch(ctx, jobs, mode)
                info = b.info()
                b.close()
                if (seg, info["workgroups"]) in seen:
                    continue  # the same launch as a row already timed
                seen.add((seg, info["workgroups"]))
                r["workgroups_per_cu"] = round(info["workgroups"] / cu_count, 3)
                r["ms"] = time_of(r, reps)
                table.append(r)
        best = _refine(table, time_of, reps_top, top)
    finally:
        B.mjd_ctx_set_tuning(ctx, saved["seg_subtiles"], saved["workgroups"], saved["shape"])
    return best, table


def size_class(frame) -> str:
    """Sampling and the power-of-two buckets of width and height."""
    w, h = int(frame["width"]), int(frame["height"])
    return f"h{frame['h'][0]}v{frame['v'][0]}_w2^{int(math.log2(max(w, 1)))}_h2^{int(math.log2(max(h, 1)))}"


class TuneCache:
    """JSON file of tuned launch shapes.  Keys name the device, the kernel
    sources' hash and the workload class; an entry holds the tuning fields
    and the evidence (search ranges, interior flags, timing)."""

    def __init__(self, path: str = None):
        self.path = path or os.environ.get("MJD_TUNE_CACHE", DEFAULT_CACHE)
        self.entries = {}
        if os.path.exists(self.path):
            with open(self.path) as f:
                self.entries = json.load(f)

    @staticmethod
    def key(device: str, workload: str) -> str:
        return f"{device}|{kernel_hash()[:16]}|{workload}"

    @staticmethod
    def image_workload(frame, mode: int) -> str:
        return f"image|{size_class(frame)}|mode{mode}"

    def get(self, key: str):
        return self.entries.get(key)

    def put(self, key: str, entry: dict):
        self.entries[key] = entry
        d = os.path.dirname(os.path.abspath(self.path))
        os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.entries, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def _entry(best, table, axes):
    return {"seg_subtiles": best["seg_subtiles"], "workgroups": best["workgroups"], "shape": best.get("shape", 0),
            "best": best, "interior": {a: interior(best, table, a) for a in axes},
            "ranges": {a: sorted({r[a] for r in table}) for a in axes}, "candidates": len(table)}


def tuned_image(ctx, frame, mode: int, coef_sets, qt, out_sets, cache: TuneCache = None, device: int = 0,
                retune: bool = False):
    """Set ctx's tuning for this image class from the cache, or tune and
    store it.  Returns (entry, source) with source "cache" or "tuned"."""
    cache = cache or TuneCache()
    key = TuneCache.key(device_name(device), TuneCache.image_workload(frame, mode))
    e = None if retune else cache.get(key)
    source = "cache"
    if e is None:
        best, table = tune(ctx, frame, coef_sets, qt, mode, out_sets)
        e = _entry(best, table, ("seg_subtiles", "workgroups_per_cu"))
        e["table"] = table
        cache.put(key, e)
        source = "tuned"
    e = dict(e, key=key)
    B.mjd_ctx_set_tuning(ctx, e["seg_subtiles"], e["workgroups"], e["shape"])
    return e, source


def apply_cached(ctx, frame, mode: int, cache: TuneCache = None, device: int = 0) -> bool:
    """Set ctx's tuning from a cached entry for this image class, if any."""
    cache = cache or TuneCache()
    e = cache.get(TuneCache.key(device_name(device), TuneCache.image_workload(frame, mode)))
    if e is None:
        return False
    B.mjd_ctx_set_tuning(ctx, e["seg_subtiles"], e["workgroups"], e["shape"])
    return True


def tuned_batch(ctx, jobs, mode: int, workload: str, cache: TuneCache = None, device: int = 0,
                retune: bool = False):
    """Cached tuning of a batch workload (named by the caller: the batch
    mix it stands for).  Sets ctx's tuning; returns (entry, source)."""
    cache = cache or TuneCache()
    key = TuneCache.key(device_name(device), f"batch|{workload}|mode{mode}")
    e = None if retune else cache.get(key)
    source = "cache"
    if e is None:
        import torch
        best, table = tune_batch(ctx, jobs, mode, cu_count=torch.cuda.get_device_properties(device).multi_processor_count)
        e = _entry(best, table, ("seg_subtiles", "workgroups_per_cu"))
        e["table"] = table
        cache.put(key, e)
        source = "tuned"
    e = dict(e, key=key)
    B.mjd_ctx_set_tuning(ctx, e["seg_subtiles"], e["workgroups"], 0)
    return e, source
