#!/usr/bin/env python3
"""Benchmark of the fused JPEG back half on one MI355X.

A step is one pass of the whole path (dequantise -> IDCT -> upsample ->
colour -> RGB8 store) over one 4096x3072 4:2:0 image (quality 90 tables,
texture content, fancy upsampling), with the coefficients already resident in
device memory.  Five coefficient/RGB buffer sets (~377 MB) rotate between
steps so the 256 MB Infinity Cache cannot hold the working set.

Prints one JSON line: throughput in MPix/s, the roofline entry of the decode
kernel (algorithmic bytes / kernel time against 8 TB/s), the oracle's CPU rate
on a bounded sample, and side measurements (copy bandwidth, small-image
latency percentiles).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MPix/s IDCT+upsample+colour, % HBM roofline; batched vs per-image; p99 lat"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--sets", type=int, default=5, help="rotating buffer sets")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget for the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-latency", action="store_true", help="skip the small-image latency loop")
    ap.add_argument("--tune", action="store_true", help="autotune the launch shape before timing")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the decode path has no "
                                   "multi-GPU mode (images or MCU-row bands shard with no communication)"}))
        sys.exit(2)
    import torch

    import paper_1311_5304_amd as M
    from synth import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = M.Context(0)

    t0 = time.time()
    frame, coef, qt = workloads.large_420_fancy()
    gen_s = time.time() - t0
    W, H = frame["width"], frame["height"]
    g = M.mjd_geometry_of(frame)
    coef_bytes = coef.nbytes
    rgb_bytes = W * H * 3
    q_dev = torch.from_numpy(qt.view(np.int16)).to(dev)
    c_sets = [torch.from_numpy(coef).to(dev) for _ in range(args.sets)]
    o_sets = [torch.empty((H, W, 3), dtype=torch.uint8, device=dev) for _ in range(args.sets)]
    stream = torch.cuda.current_stream()

    if args.tune:
        from paper_1311_5304_amd import autotune
        best, table = autotune.tune(ctx, frame, c_sets, q_dev, M.MJD_UPSAMPLE_FANCY, o_sets,
                                    wg_candidates=(0, 256, 512, 768, 1024))
        M.mjd_ctx_set_tuning(ctx, best["seg_subtiles"], best["max_workgroups"])
        tuned = {"best": best, "table": table}
    else:
        tuned = None

    def step(i):
        k = i % args.sets
        M.mjd_decode(ctx, frame, c_sets[k], q_dev, M.MJD_UPSAMPLE_FANCY, o_sets[k], 3 * W, 0, g["mcus_y"],
                     stream)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for i in range(args.steps):
        step(i)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_total = ev0.elapsed_time(ev1)
    ms_per_step = ms_total / args.steps
    mpix_s = W * H * args.steps / (ms_total * 1e-3) / 1e6
    algo_bytes = coef_bytes + rgb_bytes
    achieved_gbs = algo_bytes / (ms_per_step * 1e-3) / 1e9

    # parity spot check of the timed output against the oracle (full image)
    out = {}
    extras = {"generation_s": round(gen_s, 2), "tuning": M.mjd_ctx_get_tuning(ctx)}
    if tuned:
        extras["autotune"] = tuned
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        reps = 0
        t_cpu = 0.0
        ref = None
        while t_cpu < args.cpu_seconds or reps == 0:
            t = time.perf_counter()
            ref = oracle.decode(frame, coef, qt, "fancy")
            t_cpu += time.perf_counter() - t
            reps += 1
        cpu = {"value": round(W * H * reps / t_cpu / 1e6, 3), "unit": "MPix/s", "cores": 1, "kind": "oracle",
               "sample": f"{reps} full decodes of the same 4096x3072 4:2:0 fancy image (numpy, one thread)"}
        gpu_out = o_sets[(args.steps - 1) % args.sets].cpu().numpy()
        extras["bit_exact_vs_oracle"] = bool(np.array_equal(gpu_out, ref))

    if True:
        # copy-kernel bandwidth over the same byte count (read coef-size, write coef-size)
        n = (algo_bytes // 2) // 16 * 16
        src = [torch.empty(n, dtype=torch.uint8, device=dev) for _ in range(args.sets)]
        dst = [torch.empty(n, dtype=torch.uint8, device=dev) for _ in range(args.sets)]
        for i in range(10):
            M.mjd_copy(ctx, dst[i % args.sets], src[i % args.sets], n, stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(100):
            M.mjd_copy(ctx, dst[i % args.sets], src[i % args.sets], n, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        copy_ms = e0.elapsed_time(e1) / 100
        extras["copy_GBps"] = round(2 * n / (copy_ms * 1e-3) / 1e9, 1)
        extras["copy_bytes_per_launch"] = 2 * n
        del src, dst
    if not args.no_latency:
        # small-image latency: 256x256 4:2:0 simple, kernel-only, per call
        f1, c1, q1 = workloads.small_420_simple()
        c1d = torch.from_numpy(c1).to(dev)
        q1d = torch.from_numpy(q1.view(np.int16)).to(dev)
        o1 = torch.empty((256, 256, 3), dtype=torch.uint8, device=dev)
        g1 = M.mjd_geometry_of(f1)
        lat = []
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(1000)]
        for a, b in evs:
            a.record(stream)
            M.mjd_decode(ctx, f1, c1d, q1d, M.MJD_UPSAMPLE_SIMPLE, o1, 768, 0, g1["mcus_y"], stream)
            b.record(stream)
        torch.cuda.synchronize()
        lat = np.array([a.elapsed_time(b) * 1e3 for a, b in evs])
        extras["small_256x256_420_simple_us"] = {"p50": round(float(np.percentile(lat, 50)), 2),
                                                 "p99": round(float(np.percentile(lat, 99)), 2)}

    out = {
        "metric": METRIC,
        "value": round(mpix_s, 1),
        "unit": "MPix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "one 4096x3072 image, 4:2:0, quality-90 tables, texture content, "
                               "fancy upsampling, int16 coefficients resident in HBM -> RGB8",
                   "width": W, "height": H, "sampling": "4:2:0", "upsample": "fancy",
                   "rotating_sets": args.sets},
        "roofline": {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved_gbs / HBM_PEAK_GBS, 4), "traffic": None},
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
