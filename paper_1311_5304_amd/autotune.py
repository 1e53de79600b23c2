"""Launch-shape autotuner for the decode kernels.

The paper picks its work-group size per platform by profiling (Sec. 4.1 and
Sec. 5.1).  Here the free choices are the segment length (sub-tile rows a
workgroup walks, prefetching the next while decoding the current) and the
number of resident workgroups; both change only speed, never the output.
`tune()` times every candidate with HIP events on the caller's buffers and
returns the fastest; `TuneCache` keeps the choice per (device, sampling,
mode, size class) in a JSON file.
"""
from __future__ import annotations

import json
import math
import os

from . import _binding as B

SEG_CANDIDATES = (0, 1, 2, 3, 4, 6, 8, 12, 16, 24, 32)
WG_CANDIDATES = (0,)


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


def tune(ctx, frame, coef_sets, qt, mode: int, out_sets, reps: int = 20,
         seg_candidates=SEG_CANDIDATES, wg_candidates=WG_CANDIDATES):
    """Time each (seg_subtiles, max_workgroups) on rotating buffer sets.

    coef_sets / out_sets: lists of device tensors (rotated so caches do not
    hold the working set).  Returns (best, table) where table rows are
    dicts {seg_subtiles, max_workgroups, ms}."""
    g = B.mjd_geometry_of(frame)
    w = int(frame["width"])
    saved = B.mjd_ctx_get_tuning(ctx)
    table = []
    try:
        for seg in seg_candidates:
            for wgs in wg_candidates:
                B.mjd_ctx_set_tuning(ctx, seg, wgs)
                it = [0]

                def run():
                    k = it[0] % len(coef_sets)
                    it[0] += 1
                    B.mjd_decode(ctx, frame, coef_sets[k], qt, mode, out_sets[k], 3 * w, 0, g["mcus_y"])
                table.append({"seg_subtiles": seg, "max_workgroups": wgs, "ms": _time_ms(run, reps)})
    finally:
        B.mjd_ctx_set_tuning(ctx, saved["seg_subtiles"], saved["max_workgroups"])
    best = min(table, key=lambda r: r["ms"])
    return best, table


BATCH_SEG_CANDIDATES = (0, 1, 2, 3, 4, 6, 8, 12)


def tune_batch(ctx, jobs, mode: int, reps: int = 5, seg_candidates=BATCH_SEG_CANDIDATES,
               wg_candidates=WG_CANDIDATES, use_graph: bool = True):
    """Plan the batch once per (seg_subtiles, max_workgroups) candidate and
    time its persistent launch.  seg_subtiles 0 is the planner's own choice
    (about four segments per resident workgroup).  Returns (best, table);
    the planned Batch objects are released."""
    saved = B.mjd_ctx_get_tuning(ctx)
    table = []
    try:
        for seg in seg_candidates:
            for wgs in wg_candidates:
                B.mjd_ctx_set_tuning(ctx, seg, wgs)
                b = B.Batch(ctx, jobs, mode)
                try:
                    info = b.info()
                    ms = _time_ms(lambda: b.launch(use_graph=use_graph), reps, warmup=2)
                finally:
                    b.close()
                table.append({"seg_subtiles": seg, "max_workgroups": wgs, "segments": info["segments"],
                              "workgroups": info["workgroups"], "ms": ms})
    finally:
        B.mjd_ctx_set_tuning(ctx, saved["seg_subtiles"], saved["max_workgroups"])
    best = min(table, key=lambda r: r["ms"])
    return best, table


def size_class(frame) -> str:
    """Power-of-two bucket of the pixel count, with the sampling."""
    px = int(frame["width"]) * int(frame["height"])
    return f"h{frame['h'][0]}v{frame['v'][0]}_2^{int(math.log2(max(px, 1)))}"


class TuneCache:
    """JSON file of tuned launch shapes keyed by device / sampling / mode / size."""

    def __init__(self, path: str):
        self.path = path
        self.entries = {}
        if os.path.exists(path):
            with open(path) as f:
                self.entries = json.load(f)

    @staticmethod
    def key(device_name: str, frame, mode: int) -> str:
        return f"{device_name}|{size_class(frame)}|mode{mode}"

    def get(self, key: str):
        return self.entries.get(key)

    def put(self, key: str, best: dict):
        self.entries[key] = {"seg_subtiles": best["seg_subtiles"], "max_workgroups": best["max_workgroups"],
                             "ms": best["ms"]}
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.entries, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)
