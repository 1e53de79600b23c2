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
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="budget of each oracle baseline leg (one core, then all cores)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-latency", action="store_true", help="skip the small-image latency loop")
    ap.add_argument("--no-tune", action="store_true",
                    help="launch with the library's default shape instead of the tuned one")
    ap.add_argument("--retune", action="store_true",
                    help="time every launch shape again even when the tuning cache holds this workload")
    ap.add_argument("--no-batch", action="store_true", help="skip the mixed 256-image batch measurement")
    ap.add_argument("--batch-images", type=int, default=256)
    ap.add_argument("--batch-reps", type=int, default=10)
    ap.add_argument("--no-pipeline", action="store_true", help="skip the end-to-end bitstream corpus measurement")
    ap.add_argument("--corpus-images", type=int, default=1000)
    ap.add_argument("--pipeline-threads", type=int, default=15, help="entropy worker threads (plus the caller)")
    ap.add_argument("--no-gpu-entropy", action="store_true",
                    help="skip the device-resident corpus decode (GPU entropy kernel + batched back half)")
    ap.add_argument("--gpu-entropy-reps", type=int, default=5)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-loop measurement")
    ap.add_argument("--no-model", action="store_true", help="skip fitting and checking the performance model")
    ap.add_argument("--no-variants", action="store_true", help="skip the decoder-variant measurements")
    ap.add_argument("--serve-requests", type=int, default=2200, help="requests per trace (the first 200 warm up)")
    return ap.parse_args()


PROFILE = os.path.join(ROOT, "profiles", "decode_segments_420_fancy_4096x3072.md")
KERNEL_SOURCES = ("segment.h", "decode_kernel.h", "aan.h", "decode.hip")


def profiled_traffic():
    """HBM bytes per launch of the headline kernel from the committed counter
    summary, or None when the kernel sources changed since it was taken."""
    import hashlib
    import re
    if not os.path.exists(PROFILE):
        return None
    text = open(PROFILE).read()
    m_hash = re.search(r"kernel_sources_sha256: ([0-9a-f]{64})", text)
    m_bytes = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    if not m_hash or not m_bytes:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1311_5304_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return int(m_bytes.group(1)) if h.hexdigest() == m_hash.group(1) else None


def tuning_report(entry, source):
    """The launch shape a measurement ran with: where it came from (the
    tuning cache or a fresh search), the ranges searched and whether the
    winner lies inside them on each ordered axis."""
    best = entry["best"]
    keep = ("shape", "sx", "sy", "threads", "resident_per_cu", "workgroups_per_cu", "workgroups", "seg_subtiles",
            "ms", "ms_refined", "segments", "launched")
    return {"source": source, "cache_key": entry.get("key"), "choice": {k: best[k] for k in keep if k in best},
            "interior": entry["interior"], "ranges": entry["ranges"], "candidates": entry["candidates"]}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _events_ms(torch, stream, fn, reps):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def batch_workload(args, M, ctx, dev, stream):
    """Mixed batch: N images, W and H uniform in 320..4096 (never multiples
    of 16), thirds of 4:4:4 / 4:2:2 / 4:2:0, quality 50..95 with per-image
    tables, gradient content with sigma 8 noise, generated on the GPU.

    Reports the batched persistent launch (hipGraph replay and direct) against
    per-image launches (back-to-back on one stream, and synchronised after each
    image), all on the same resident buffers, plus the tuned launch shape and a
    sampled bit-exactness check against the oracle."""
    import torch

    from paper_1311_5304_amd import autotune
    from synth import gpu_encode, workloads

    log(f"generating the {args.batch_images}-image batch on the GPU")
    t0 = time.time()
    specs = workloads.batch_specs(n=args.batch_images)
    imgs = []
    for spec in specs:
        frame, coef, qt = gpu_encode.batch_image_gpu(torch, spec, dev)
        qd = torch.from_numpy(qt.view(np.int16)).to(dev)
        out = torch.empty((frame["height"], frame["width"], 3), dtype=torch.uint8, device=dev)
        imgs.append((frame, coef, qd, out, 3 * frame["width"], qt))
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    jobs = [im[:5] for im in imgs]
    px = sum(f["width"] * f["height"] for f, *_ in imgs)
    nbytes = sum(c.numel() * 2 + o.numel() for _, c, _, o, _, _ in imgs)
    res = {"images": len(imgs), "megapixels": round(px / 1e6, 1), "algorithmic_bytes": nbytes,
           "generation_s": round(gen_s, 1)}

    def rate(ms):
        return {"ms": round(ms, 3), "MPix_s": round(px / (ms * 1e-3) / 1e6, 1),
                "GB_s": round(nbytes / (ms * 1e-3) / 1e9, 1),
                "frac_hbm": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    saved = M.mjd_ctx_get_tuning(ctx)
    if not args.no_tune:
        log("batch launch shape (tuning cache, else the autotuner)")
        entry, source = autotune.tuned_batch(ctx, jobs, M.MJD_UPSAMPLE_FANCY,
                                             f"{len(jobs)} images 320..4096 px mixed samplings", retune=args.retune)
        res["tuning"] = tuning_report(entry, source)
    batch = M.Batch(ctx, jobs, M.MJD_UPSAMPLE_FANCY)
    M.mjd_ctx_set_tuning(ctx, saved["seg_subtiles"], saved["workgroups"], saved["shape"])
    log("timing batched and per-image launches")
    res["plan"] = batch.info()
    batch.launch(use_graph=True)
    torch.cuda.synchronize()
    res["fancy_batched_graph"] = rate(_events_ms(torch, stream, lambda: batch.launch(use_graph=True),
                                                 args.batch_reps))
    res["fancy_batched_direct"] = rate(_events_ms(torch, stream, lambda: batch.launch(use_graph=False),
                                                  args.batch_reps))

    # the per-image launches run with the library's default launch shape
    M.mjd_ctx_set_tuning(ctx, 0, 0, 0)

    def per_image():
        for frame, c, q, o, pitch, _ in imgs:
            M.mjd_decode(ctx, frame, c, q, M.MJD_UPSAMPLE_FANCY, o, pitch, 0,
                         M.mjd_geometry_of(frame)["mcus_y"], stream)
    per_image()
    torch.cuda.synchronize()
    res["fancy_per_image_back_to_back"] = rate(_events_ms(torch, stream, per_image, max(1, args.batch_reps // 2)))
    t = time.perf_counter()
    for frame, c, q, o, pitch, _ in imgs:
        M.mjd_decode(ctx, frame, c, q, M.MJD_UPSAMPLE_FANCY, o, pitch, 0, M.mjd_geometry_of(frame)["mcus_y"],
                     stream)
        torch.cuda.synchronize()
    res["fancy_per_image_synced"] = rate((time.perf_counter() - t) * 1e3)
    res["speedup_batched_vs_per_image_synced"] = round(
        res["fancy_per_image_synced"]["ms"] / res["fancy_batched_graph"]["ms"], 2)

    # bit-exactness on samples: the last launch wrote every output (per image);
    # replay the batch so the checked bytes are the batched kernel's
    for *_, o, _, _ in imgs:
        o.fill_(0)
    batch.launch(use_graph=True)
    torch.cuda.synchronize()
    log("oracle check of batch samples")
    res["bit_exact_samples"] = batch_samples_match(imgs, "fancy")

    simple = M.Batch(ctx, jobs, M.MJD_UPSAMPLE_SIMPLE)
    simple.launch(use_graph=True)
    torch.cuda.synchronize()
    res["simple_batched_graph"] = rate(_events_ms(torch, stream, lambda: simple.launch(use_graph=True),
                                                  args.batch_reps))
    simple.close()
    batch.close()
    M.mjd_ctx_set_tuning(ctx, saved["seg_subtiles"], saved["workgroups"], saved["shape"])
    return res


def pipeline_workload(args, M, ctx, dev):
    """End-to-end decode of a corpus of baseline JPEG bitstreams (our encoder;
    1..24 MP, 4:3 / 3:2 / 16:9 either way up, 4:2:0, quality 85, a restart
    marker every 32 MCUs, texture content): host worker threads Huffman-decode
    restart intervals of MCU-row bands into pinned buffers, pipelined with
    host->device copies, the fused kernel and device->host copies of RGB8 on
    three streams.  The entropy-only run (same threads, nothing sent to the
    GPU) is the entropy-bound limit."""
    from concurrent.futures import ThreadPoolExecutor

    import torch

    import oracle
    from synth import fast_bitstream, gpu_encode, workloads

    log(f"generating the {args.corpus_images}-bitstream corpus")
    t0 = time.time()
    specs = workloads.corpus_specs(n=args.corpus_images)
    jpgs = [None] * len(specs)
    sample = None
    smallest = min(range(len(specs)), key=lambda i: specs[i][0] * specs[i][1])

    def encode_one(i, frame, coef, qt):
        jpgs[i] = fast_bitstream.write_jpeg(frame, coef, qt, restart_interval=32)

    with ThreadPoolExecutor(max_workers=16) as ex:
        futs = []
        for i, spec in enumerate(specs):
            frame, c, qt = gpu_encode.batch_image_gpu(torch, spec, dev, sigma=12.0, content="texture")
            coef = c.cpu().numpy()
            if i == smallest:
                sample = (frame, coef, qt)
            futs.append(ex.submit(encode_one, i, frame, coef, qt))
            if len(futs) > 32:
                futs.pop(0).result()
        for f in futs:
            f.result()
    gen_s = time.time() - t0
    px = sum(w * h for w, h, *_ in specs)
    nbytes = sum(len(j) for j in jpgs)
    frames = [workloads.make_frame(w, h, s) for w, h, s, _, _ in specs]
    max_blocks = max(oracle.geometry(f)["n_blocks"] for f in frames)
    max_px = max(w * h for w, h, *_ in specs)
    ring = [torch.empty(max_px * 3, dtype=torch.uint8).pin_memory() for _ in range(4)]
    outs = [ring[i % len(ring)] for i in range(len(jpgs))]
    pitches = [3 * w for w, *_ in specs]
    pipe = M.Pipeline(ctx, args.pipeline_threads, max_blocks, max_px, M.MJD_UPSAMPLE_FANCY, n_slots=3)
    try:
        log("pipeline: entropy-only run")
        ent = pipe.run(jpgs, outs, pitches, entropy_only=True)
        log("pipeline: end-to-end run")
        full = pipe.run(jpgs, outs, pitches)
        # bit-exactness: the smallest image through the pipeline against the
        # oracle's back half on the coefficients it was encoded from
        frame, coef, qt = sample
        o = torch.empty(frame["width"] * frame["height"] * 3, dtype=torch.uint8).pin_memory()
        pipe.run([jpgs[smallest]], [o], [3 * frame["width"]])
        exact = bool(np.array_equal(o.numpy().reshape(frame["height"], frame["width"], 3),
                                    oracle.decode(frame, coef.reshape(-1, 64), qt, "fancy")))
    finally:
        pipe.close()
    gpu_ms = full["h2d_ms"] + full["kernel_ms"] + full["d2h_ms"]
    dev_e2e = None
    if not args.no_gpu_entropy:
        dev_e2e = gpu_entropy_workload(args, M, ctx, dev, jpgs, frames, smallest, sample)
    return {
        "images": len(jpgs), "megapixels": round(px / 1e6, 1), "bitstream_MB": round(nbytes / 1e6, 1),
        "bits_per_pixel": round(8 * nbytes / px, 3), "generation_s": round(gen_s, 1),
        "threads": args.pipeline_threads + 1, "slots": 3,
        "MPix_s": round(px / (full["wall_ms"] * 1e-3) / 1e6, 1),
        "wall_ms": round(full["wall_ms"], 1),
        "entropy_only_wall_ms": round(ent["wall_ms"], 1),
        "entropy_only_MPix_s": round(px / (ent["wall_ms"] * 1e-3) / 1e6, 1),
        "fraction_of_entropy_bound": round(ent["wall_ms"] / full["wall_ms"], 4),
        "stage_overlap": round(1 - (full["wall_ms"] - ent["wall_ms"]) / gpu_ms, 4) if gpu_ms > 0 else None,
        "h2d_ms": round(full["h2d_ms"], 1), "kernel_ms": round(full["kernel_ms"], 1),
        "d2h_ms": round(full["d2h_ms"], 1), "worker_entropy_ms": round(full["entropy_ms"], 1),
        "parse_ms": round(full["parse_ms"], 1), "bands": full["bands"],
        "bit_exact_sample": {"image": smallest, "size": [frame["width"], frame["height"]], "equal": exact},
        "device_resident": dev_e2e,
    }


def model_workload(args, M, ctx, dev):
    """The paper's performance model (Sec. 5.1) fitted on this machine: a
    training set of synthetic 4:2:0 bitstreams on a grid of sizes from 0.75
    to 25 MP (qualities 50-95, texture and gradient content, like the paper's
    crops of a few photographs to many sizes), each timed in its four phases;
    then a held-out set of 16 other images (1-24 MP, inside the training
    grid), predicted and measured, the host parts of the partitioning
    (p_cpu, t_dispatch) at each one's quarter splits too."""
    import torch

    from paper_1311_5304_amd import perfmodel
    from synth import fast_bitstream, gpu_encode, workloads

    log("performance model: profiling the training set")
    t0 = time.time()
    rng = np.random.default_rng(workloads.seed_of(7, 0xFFFFF))

    def bitstream(w, h, q, seed, content):
        frame, c, qt = gpu_encode.batch_image_gpu(torch, (w, h, "420", q, seed), dev, sigma=12.0, content=content)
        return fast_bitstream.write_jpeg(frame, c.cpu().numpy(), qt, restart_interval=32)

    n_threads = args.pipeline_threads + 1
    hetero = M.Hetero(ctx, max_blocks=25_000_000 * 3 // 128 + 65536, max_pixels=25_000_000 + 65536,
                      n_threads=n_threads)

    # A grid over the whole prediction domain (polynomials extrapolate
    # badly, as the paper notes): widths 1024..6656, heights 768..4224, from
    # 0.75 to 25 MP; below that the per-call costs of the host decoder, which
    # the per-pixel rate of Eq. 4 does not model, dominate.
    train = []
    k = 0
    for w in range(1024, 6657, 512):
        for h in range(768, 4225, 384):
            if w * h > 25_000_000:
                continue
            q = (50, 60, 70, 80, 90, 95)[k % 6]
            content = "texture" if k % 2 == 0 else "gradient"
            train.append(perfmodel.measure(ctx, bitstream(w, h, q, workloads.seed_of(7, k), content), reps=3,
                                           hetero=hetero))
            k += 1
    model, info = perfmodel.fit(train)
    log("performance model: held-out images")
    errs = {"t_huff": [], "p_gpu": [], "total": []}
    held_out = []
    for i in range(16):
        while True:  # inside the training domain
            mp = rng.uniform(1.0, 24.0)
            aspect = rng.choice([4 / 3, 3 / 2, 16 / 9])
            w = int(round((mp * 1e6 * aspect) ** 0.5))
            h = int(round(mp * 1e6 / w))
            if 1024 <= w <= 6656 and 768 <= h <= 4224:
                break
        q = int(rng.integers(50, 96))
        content = "texture" if i % 2 == 0 else "gradient"
        s = perfmodel.measure(ctx, bitstream(w, h, q, workloads.seed_of(8, i), content), reps=3, hetero=hetero)
        held_out.append(s)
        p = perfmodel.predict(model, s["width"], s["height"], s["bytes"])
        meas = {"t_huff": s["t_huff"], "p_gpu": s["o_w"] + s["t_kernel"] + s["o_r"]}
        meas["total"] = meas["t_huff"] + meas["p_gpu"]
        for key in errs:
            errs[key].append(abs(p[key] - meas[key]) / meas[key])
    # the host parts of the partitioning at the held-out images' quarter splits
    errs.update(perfmodel.host_errors(model, held_out))
    abs_us = {k: round(float(np.mean(v)) * 1e6, 2) for k, v in perfmodel.host_errors(model, held_out, True).items()}

    def pct(v):
        return {q: round(float(np.percentile(v, q)) * 1e6, 2) for q in (10, 50, 90, 100)}
    host_spread = {"training_us": {k: pct(v) for k, v in perfmodel.host_times(train).items()},
                   "held_out_us": {k: pct(v) for k, v in perfmodel.host_times(held_out).items()},
                   "held_out_mean_abs_error_us": abs_us}
    part = partition_experiment(M, model, hetero, n_threads, bitstream, workloads)
    hetero.close()
    return {
        "training_images": len(train), "held_out_images": 16,
        "degrees_and_aic": {k: {"degree": v[0], "aic": round(v[1], 1)} for k, v in info.items()},
        "host_parts": {**host_spread, "max_degree": perfmodel.HOST_MAX_DEGREE, "monotone_in_rows": {
            k: perfmodel.rows_monotone(getattr(model, k), 1.0, 6656 / 1024.0, 4224 / 1024.0)
            for k in perfmodel.HOST_PARTS}},
        "held_out_abs_rel_error": {k: {"mean": round(float(np.mean(v)), 4), "max": round(float(np.max(v)), 4)}
                                   for k, v in errs.items()},
        "profiling_s": round(time.time() - t0, 1),
        "partition": part,
        "model": perfmodel.to_dict(model),
    }, model


def partition_experiment(M, model, hetero, n_threads, bitstream, workloads):
    """The CPU-GPU partitioning (Sec. 5.2) on a 12.6 MP and a 24 MP 4:2:0
    image (RGB back to pinned host memory, Huffman on the host's threads):
    GPU alone, host alone, and the SPS, overlapped and PPS splits the fitted
    model's Newton solve gives, with the model's predicted sides beside the
    measured ones; for SPS also half and twice the chosen host share; for PPS
    chunks of 4 to 32 MCU rows (the paper picks the chunk by profiling), then
    the best chunk with re-partitioning before the last chunk.  Every run's
    RGB must equal the GPU-only run's bytes.  Times are the best of 5."""
    import torch

    log("CPU-GPU partitioning")
    out = []
    for (w, h, q), seed in zip(((4096, 3072, 85), (6000, 4000, 85)), (11, 12)):
        jpg = bitstream(w, h, q, workloads.seed_of(9, seed), "texture")
        mcu_h = 16
        ref = torch.empty(h * w * 3, dtype=torch.uint8).pin_memory()
        rgb = torch.empty(h * w * 3, dtype=torch.uint8).pin_memory()
        same = [True]

        def run(cpu_rows, scheme, dst=rgb, **kw):
            best = None
            for _ in range(5):
                t = hetero.decode(jpg, dst, 3 * w, cpu_rows, scheme, M.MJD_UPSAMPLE_FANCY, **kw)
                if best is None or t["total_s"] < best["total_s"]:
                    best = t
            if dst is not ref:
                # numpy, one thread: torch's CPU ops would leave its OpenMP
                # threads spinning on the cores the next runs' host side uses
                same[0] &= bool(np.array_equal(dst.numpy(), ref.numpy()))
            return best

        # warm the host pool and the caches on this image before timing it
        for _ in range(3):
            hetero.decode(jpg, rgb, 3 * w, h // 2 // mcu_h * mcu_h, M.MJD_PART_SPS, M.MJD_UPSAMPLE_FANCY)

        def ms(t):
            return {(k[:-2] + "_ms" if k.endswith("_s") else k): (round(v * 1e3, 3) if k.endswith("_s") else v)
                    for k, v in t.items()}

        gpu_only = run(0, M.MJD_PART_SPS, ref)

        def summary(p, t, sides=True):
            d = {"planned_cpu_rows": p["cpu_rows"], "newton_iterations": p["iterations"],
                 "predicted_cpu_side_ms": round(p["t_cpu"] * 1e3, 3),
                 "predicted_gpu_side_ms": round(p["t_gpu"] * 1e3, 3)}
            if sides:
                cpu_side = t["dispatch_s"] + t["huff_cpu_s"] + t["cpu_s"]
                d["measured_cpu_side_ms"] = round(cpu_side * 1e3, 3)
                d["measured_gpu_side_ms"] = round(t["gpu_s"] * 1e3, 3)
                d["cpu_side_rel_error"] = round((cpu_side - p["t_cpu"]) / p["t_cpu"], 4) if p["t_cpu"] else None
                d["gpu_side_rel_error"] = round((t["gpu_s"] - p["t_gpu"]) / p["t_gpu"], 4) if p["t_gpu"] else None
            d.update(ms(t))
            d["speedup_vs_gpu_only"] = round(gpu_only["total_s"] / t["total_s"], 3)
            return d

        row = {"image": f"{w}x{h}", "bytes": len(jpg), "huff_threads": n_threads, "gpu_only": ms(gpu_only),
               "cpu_only": ms(run(h, M.MJD_PART_SPS))}
        for name, scheme in (("sps", M.MJD_PART_SPS), ("overlap", M.MJD_PART_OVERLAP)):
            p = M.mjd_partition_rows(model, scheme, w, h, mcu_h, len(jpg), n_threads)
            row[name] = summary(p, run(p["cpu_rows"], scheme))
            if name == "sps":
                sweep = []
                for f in (0.5, 2.0):
                    r = h - min(h, int(round((h - p["cpu_rows"] * f) / mcu_h)) * mcu_h)
                    r = min(max(r, 0), h)
                    sweep.append({"cpu_rows": r, "total_ms": round(run(r, scheme)["total_s"] * 1e3, 3)})
                row["sps_sweep"] = sweep
        chunks = []
        for c in (4, 8, 16, 32):
            p = M.mjd_partition_rows(model, M.MJD_PART_PPS, w, h, mcu_h, len(jpg), n_threads, c * mcu_h)
            chunks.append((c, p, run(p["cpu_rows"], M.MJD_PART_PPS, chunk_mcu_rows=c)))
        row["pps_chunks"] = [{"chunk_mcu_rows": c, "cpu_rows": t["cpu_rows"], "total_ms": round(t["total_s"] * 1e3, 3)}
                             for c, p, t in chunks]
        c, p, t = min(chunks, key=lambda e: e[2]["total_s"])
        row["pps"] = {"chunk_mcu_rows": c, **summary(p, t, sides=False)}
        t = run(p["cpu_rows"], M.MJD_PART_PPS, chunk_mcu_rows=c, model=model, huff_threads=n_threads)
        row["pps_repartition"] = {"chunk_mcu_rows": c, **summary(p, t, sides=False)}
        # Amdahl (Eqs. 18-19): against the host-only decoder, whose Huffman
        # part cannot be shared, the attainable speed-up is T_total / T_huff
        cpu_only = row["cpu_only"]
        bound = cpu_only["total_ms"] / cpu_only["huff_gpu_ms"]
        best_pps = min(row["pps"]["total_ms"], row["pps_repartition"]["total_ms"])
        row["amdahl"] = {"attainable_speedup_vs_cpu_only": round(bound, 3),
                         "pps_speedup_vs_cpu_only": round(cpu_only["total_ms"] / best_pps, 3),
                         "fraction_of_attainable": round(cpu_only["total_ms"] / best_pps / bound, 3)}
        row["all_runs_equal_gpu_only"] = same[0]
        out.append(row)
    return out


def variants_workload(args, M, ctx, dev):
    """The decoder variants at 4096x3072: the three IDCT methods on the
    headline 4:2:0 fancy coefficients and on h1v2 and 4:1:1 coefficient sets
    (seeded decaying random blocks on the documented domain), all through
    the fused segment kernel; grayscale (one launch); and the headline image
    decoded at 1/2, 1/4 and 1/8 (two launches with sample planes between
    them; MPix/s counts the source image's pixels).  Four buffer sets rotate
    so the working set exceeds the 256 MB Infinity Cache.  Algorithmic bytes
    are the coefficients read and the output written."""
    import torch

    from synth import workloads

    log("decoder variants")
    stream = torch.cuda.current_stream()
    frame, coef, qt = workloads.large_420_fancy()
    W, H = frame["width"], frame["height"]
    rng = np.random.default_rng(workloads.seed_of(10, 0))

    def synthetic(fr):
        n = M.mjd_variant_geometry(M.make_variant(fr, fr.get("ncomp", 3)))[0]["n_blocks"]
        lim = (1155 // qt.max(axis=0)).astype(np.int64)
        c = (rng.standard_normal((n, 64)) * lim / (4 + np.arange(64))).astype(np.int64)
        c[:, 0] = rng.integers(-lim[0] // 2, lim[0] // 2 + 1, n)
        return np.clip(c, -lim, lim).astype(np.int16)

    cases = [("420_fancy_" + m, frame, coef, m, "fancy", 3) for m in ("islow", "ifast", "float")]
    for name, hv in (("h1v2_fancy", ((1, 1, 1), (2, 1, 1))), ("411_fancy", ((4, 1, 1), (1, 1, 1)))):
        fr = {"width": W, "height": H, "h": hv[0], "v": hv[1], "qsel": (0, 1, 1)}
        c = synthetic(fr)
        for m in ("islow", "ifast", "float"):
            cases.append((f"{name}_{m}", fr, c, m, "fancy", 3))
    gray = {"width": W, "height": H, "h": (1, 1, 1), "v": (1, 1, 1), "qsel": (0, 0, 0), "ncomp": 1}
    cases.append(("gray_islow", gray, synthetic(gray), "islow", "fancy", 1))
    for sc in (2, 4, 8):
        cases.append((f"420_fancy_scale_1_{sc}", frame, coef, "islow", "fancy", 3, sc))
    q_dev = torch.from_numpy(qt.view(np.int16)).to(dev)
    out = {}
    for case in cases:
        name, fr, c, method, mode, nc = case[:6]
        sc = case[6] if len(case) > 6 else 1
        v = M.make_variant(fr, nc, method, mode, sc)
        g, wb = M.mjd_variant_geometry(v)
        wo, ho = -(-W // sc), -(-H // sc)
        sets = [(torch.from_numpy(c.reshape(-1)).to(dev),
                 torch.empty((ho, wo, 3) if nc == 3 else (ho, wo), dtype=torch.uint8, device=dev),
                 torch.empty(max(wb, 16), dtype=torch.uint8, device=dev)) for _ in range(4)]

        def call(k):
            cd, o, wk = sets[k % 4]
            M.mjd_decode_variant(ctx, v, cd, q_dev, o, nc * wo, wk, wb, stream)
        for k in range(8):
            call(k)
        torch.cuda.synchronize()
        # the median of five timed runs of 40 launches each
        reps, runs = 40, []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for k in range(reps):
                call(k)
            e1.record(stream)
            torch.cuda.synchronize()
            runs.append(e0.elapsed_time(e1) / reps)
        ms = sorted(runs)[len(runs) // 2]
        # a scaled decode needs each block's n x n corner only, but every
        # block is one 128-byte line, so the whole array is the HBM floor
        algo = c.nbytes + nc * wo * ho
        out[name] = {"us": round(ms * 1e3, 2), "MPix_s": round(W * H / (ms * 1e-3) / 1e6, 1),
                     "algorithmic_GB_s": round(algo / (ms * 1e-3) / 1e9, 1),
                     "frac_hbm": round(algo / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "plane_bytes": wb}
        del sets
        torch.cuda.empty_cache()
    return out


def gpu_entropy_workload(args, M, ctx, dev, jpgs, frames, sample_idx, sample):
    """The same corpus decoded on the device end to end: the bitstreams
    resident in HBM, Huffman decoding by the entropy kernel (one lane per
    restart interval, all images in one persistent launch), then the batched
    back half (one persistent launch) into RGB8 buffers in HBM.  Planning
    (headers, restart index, tables) happens before the timed region; the
    host->device copy of the bitstreams is timed on its own."""
    import torch

    import oracle

    log("device-resident corpus decode: planning")
    stream = torch.cuda.current_stream()
    offs, total = [], 0
    for j in jpgs:  # each stream 16-byte aligned and padded to 16
        offs.append(total)
        total += -(-len(j) // 16) * 16
    host = torch.zeros(total, dtype=torch.uint8).pin_memory()
    hv = host.numpy()
    for o, j in zip(offs, jpgs):
        hv[o:o + len(j)] = np.frombuffer(j, dtype=np.uint8)
    d_all = torch.empty(total, dtype=torch.uint8, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    d_all.copy_(host, non_blocking=True)
    e1.record(stream)
    torch.cuda.synchronize()
    h2d_ms = e0.elapsed_time(e1)
    jobs_e, jobs_d = [], []
    px = 0
    for i, (j, f) in enumerate(zip(jpgs, frames)):
        scan, qt = M.mjd_parse(j)
        off = M.mjd_restart_index(j, scan)
        g = M.mjd_geometry_of(f)
        c = torch.empty(g["n_blocks"] * 64, dtype=torch.int16, device=dev)
        o = torch.empty((f["height"], f["width"], 3), dtype=torch.uint8, device=dev)
        q = torch.from_numpy(qt.view(np.int16)).to(dev)
        jobs_e.append((scan, off, d_all[offs[i]:offs[i] + len(j)], len(j), c))
        jobs_d.append((f, c, q, o, 3 * f["width"]))
        px += f["width"] * f["height"]
    eb = M.EntropyBatch(ctx, jobs_e)
    db = M.Batch(ctx, jobs_d, M.MJD_UPSAMPLE_FANCY)
    info = eb.info()
    log("device-resident corpus decode: timing")
    eb.launch(stream)
    db.launch(stream=stream)
    eb.status()
    reps = max(1, args.gpu_entropy_reps)

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    ent_ms = timed(lambda: eb.launch(stream))
    back_ms = timed(lambda: db.launch(stream=stream))
    e2e_ms = timed(lambda: (eb.launch(stream), db.launch(stream=stream)))
    eb.status()
    # bit-exactness of the smallest image: its coefficients equal the
    # encoder's, its RGB equals the oracle's back half on them
    frame, coef, qt = sample
    got_c = jobs_d[sample_idx][1].cpu().numpy().reshape(-1, 64)
    got_rgb = jobs_d[sample_idx][3].cpu().numpy()
    exact = bool(np.array_equal(got_c, coef.reshape(-1, 64)) and
                 np.array_equal(got_rgb, oracle.decode(frame, coef.reshape(-1, 64), qt, "fancy")))
    nbytes = sum(len(j) for j in jpgs)
    res = {
        "MPix_s": round(px / (e2e_ms * 1e-3) / 1e6, 1),
        "ms": round(e2e_ms, 3),
        "entropy_kernel_ms": round(ent_ms, 3),
        "entropy_MPix_s": round(px / (ent_ms * 1e-3) / 1e6, 1),
        "entropy_bitstream_GBps": round(nbytes / (ent_ms * 1e-3) / 1e9, 2),
        "back_half_ms": round(back_ms, 3),
        "bitstream_h2d_ms": round(h2d_ms, 2),
        "MPix_s_with_h2d": round(px / ((e2e_ms + h2d_ms) * 1e-3) / 1e6, 1),
        "restart_intervals": info["intervals"], "entropy_workgroups": info["workgroups"],
        "reps": reps,
        "bit_exact_sample": {"image": sample_idx, "equal": exact},
    }
    db.close()
    eb.close()
    del jobs_e, jobs_d, d_all
    torch.cuda.empty_cache()
    return res


def pcie_bandwidth(dev, nbytes: int = 256 << 20, reps: int = 5):
    """Pinned host<->device copy rates (GB/s): each direction alone, and both
    at once on two streams (the link is full duplex)."""
    import torch
    h_src = torch.empty(nbytes, dtype=torch.uint8).pin_memory()
    h_dst = torch.empty(nbytes, dtype=torch.uint8).pin_memory()
    d_a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    d_b = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()

    def timed(fn):
        best = float("inf")
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        return best

    def h2d():
        with torch.cuda.stream(s1):
            d_a.copy_(h_src, non_blocking=True)

    def d2h():
        with torch.cuda.stream(s2):
            h_dst.copy_(d_b, non_blocking=True)

    t_h2d, t_d2h = timed(h2d), timed(d2h)
    t_both = timed(lambda: (h2d(), d2h()))
    gbs = lambda t, n=nbytes: round(n / t / 1e9, 2)
    return {"h2d_GBps": gbs(t_h2d), "d2h_GBps": gbs(t_d2h), "both_directions_GBps": gbs(t_both, 2 * nbytes),
            "bytes_per_copy": nbytes}


def serve_workload(args, M, ctx, dev, model=None):
    """Serving loop: Poisson arrivals of requests log-uniform in 0.1..24 MP
    (mixed samplings, quality 50..95, gradient content), coefficients in
    pinned host memory, RGB8 back to pinned host memory (or left in device
    memory, the path without the device->host copy), a 16 GiB device
    budget.  Continuous batching, uncapped and with batches capped at 4 ms of
    the performance model's predicted GPU time, against the synchronous
    one-at-a-time server on the same trace.  The default policy is the one
    with the higher capacity on a saturating trace; the arrival rates are
    0.7x and 0.9x of its capacity.  Capacity is also stated against the
    measured pinned PCIe rates, which bound it: every request's coefficients
    cross host->device and its RGB device->host."""
    import torch

    import oracle
    from synth import gpu_encode, workloads

    log("serving: generating the request pool")
    specs = workloads.serving_pool()
    pool = []
    for spec in specs:
        frame, c, qt = gpu_encode.batch_image_gpu(torch, spec, dev, sigma=8.0)
        coef = c.cpu().pin_memory()
        q = torch.from_numpy(qt.view(np.int16).reshape(-1).copy()).pin_memory()
        out = torch.empty((frame["height"], frame["width"], 3), dtype=torch.uint8).pin_memory()
        d_out = torch.empty((frame["height"], frame["width"], 3), dtype=torch.uint8, device=dev)
        pool.append((frame, coef, q, out, qt, d_out))
    px_of = [f["width"] * f["height"] for f, *_ in pool]
    h2d_of = [c.numel() * 2 + 512 for _, c, *_ in pool]
    d2h_of = [3 * p for p in px_of]
    budget = 16 << 30
    warm = 200
    n = max(args.serve_requests, warm + 100)
    log("serving: pinned PCIe rates")
    link = pcie_bandwidth(dev)

    def run(mode, rate, cap_s=0.0, device_out=False):
        trace = workloads.serving_trace(n, len(pool), rate if rate else 1.0)
        srv = M.Server(ctx, budget, M.MJD_UPSAMPLE_FANCY, mode=mode, max_batch=256, max_inflight=2,
                       model=model if cap_s else None, max_batch_s=cap_s)
        try:
            t0 = srv.now_ns() + 2_000_000
            ids = []
            for (at, k) in trace:
                f, c, q, o, _, d = pool[k]
                ids.append(srv.submit(f, c, q, d if device_out else o, 3 * f["width"], t0 + (at if rate else 0)))
            times = [srv.wait(i) for i in ids]
        finally:
            srv.close()
        meas = times[warm:]
        ks = [k for _, k in trace[warm:]]
        px = sum(px_of[k] for k in ks)
        span = (max(t["done_ns"] for t in meas) - min(t["arrival_ns"] for t in meas)) * 1e-9
        lat = np.array([(t["done_ns"] - t["arrival_ns"]) * 1e-6 for t in meas])
        h2d = sum(h2d_of[k] for k in ks) / span / 1e9
        d2h = 0.0 if device_out else sum(d2h_of[k] for k in ks) / span / 1e9
        return {"MPix_s": round(px / span / 1e6, 1), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "mean_batch": round(float(np.mean([t["batch"] for t in meas])), 2),
                "h2d_GBps": round(h2d, 2), "d2h_GBps": round(d2h, 2)}

    log("serving: saturating traces (capacity)")
    cap = run(M.MJD_SERVE_CONTINUOUS, 0)
    cap_model = run(M.MJD_SERVE_CONTINUOUS, 0, 4e-3) if model is not None else None
    mean_px = float(np.mean(px_of))
    default_cap_s = 4e-3 if cap_model is not None and cap_model["MPix_s"] > cap["MPix_s"] else 0.0
    best = cap_model if default_cap_s else cap
    cap_dev = run(M.MJD_SERVE_CONTINUOUS, 0, default_cap_s, device_out=True)
    # the link bound: requests cross host->device (coefficients) and back
    # (RGB) on a full-duplex link, so the busier direction sets the rate
    h2d_bpp = sum(h2d_of) / sum(px_of)
    d2h_bpp = 3.0
    bound = min(link["h2d_GBps"] / h2d_bpp, link["d2h_GBps"] / d2h_bpp) * 1e3
    res = {"pool_images": len(pool), "requests": n, "warmup": warm, "budget_GiB": budget >> 30,
           "mean_request_MP": round(mean_px / 1e6, 3), "pcie": link,
           "default_policy": "continuous, model cap 4 ms" if default_cap_s else "continuous, uncapped",
           "capacity_continuous": cap,
           "capacity_default_rgb_in_device_memory": cap_dev,
           "capacity_vs_link": {
               "h2d_bytes_per_pixel": round(h2d_bpp, 3), "d2h_bytes_per_pixel": d2h_bpp,
               "link_bound_MPix_s": round(bound, 1),
               "default_fraction_of_link_bound": round(best["MPix_s"] / bound, 4),
               "default_h2d_fraction": round(best["h2d_GBps"] / link["h2d_GBps"], 4),
               "default_d2h_fraction": round(best["d2h_GBps"] / link["d2h_GBps"], 4)}}
    if cap_model is not None:
        res["capacity_continuous_model_cap_4ms"] = cap_model
    for frac in (0.7, 0.9):
        rate = frac * best["MPix_s"] * 1e6 / mean_px
        log(f"serving: Poisson trace at {frac} x capacity ({rate:.0f} requests/s)")
        res[f"default_{frac}x"] = dict(run(M.MJD_SERVE_CONTINUOUS, rate, default_cap_s), rate_per_s=round(rate, 1))
        res[f"default_rgb_in_device_memory_{frac}x"] = dict(
            run(M.MJD_SERVE_CONTINUOUS, rate, default_cap_s, device_out=True), rate_per_s=round(rate, 1))
        res[f"sync_{frac}x"] = dict(run(M.MJD_SERVE_SYNC, rate), rate_per_s=round(rate, 1))
        res[f"sync_rgb_in_device_memory_{frac}x"] = dict(run(M.MJD_SERVE_SYNC, rate, device_out=True),
                                                          rate_per_s=round(rate, 1))
        if model is not None:
            # the other batching policies on the same trace: uncapped, or
            # batches sized by the fitted performance model (paper Sec. 5.1),
            # each closing once its predicted GPU time would pass the cap
            if default_cap_s:
                res[f"continuous_uncapped_{frac}x"] = dict(run(M.MJD_SERVE_CONTINUOUS, rate), rate_per_s=round(rate, 1))
            for cap_ms in ((16.0,) if default_cap_s else (4.0, 16.0)):
                res[f"continuous_model_cap_{cap_ms:g}ms_{frac}x"] = dict(
                    run(M.MJD_SERVE_CONTINUOUS, rate, cap_ms * 1e-3), rate_per_s=round(rate, 1))
    # bit-exactness: the smallest pool image as served (host and device
    # outputs), against the oracle
    k = min(range(len(pool)), key=lambda i: px_of[i])
    f, c, q, o, qt, d = pool[k]
    ref = oracle.decode(f, c.numpy().reshape(-1, 64), qt, "fancy")
    res["bit_exact_sample"] = {"pool_image": k, "size": [f["width"], f["height"]],
                               "equal": bool(np.array_equal(o.numpy(), ref)),
                               "equal_device_output": bool(np.array_equal(d.cpu().numpy(), ref))}
    return res


def batch_samples_match(imgs, mode):
    """Oracle check of the batched outputs: the three smallest images whole,
    and one interior MCU row of the three largest (decoded by the oracle from
    that row and its neighbours, which is all the row depends on)."""
    import oracle
    order = sorted(range(len(imgs)), key=lambda i: imgs[i][0]["width"] * imgs[i][0]["height"])
    ok = True
    checked = []
    for i in order[:3]:
        frame, c, _, o, _, qt = imgs[i]
        ref = oracle.decode(frame, c.cpu().numpy().reshape(-1, 64), qt, mode)
        ok &= bool(np.array_equal(o.cpu().numpy(), ref))
        checked.append(f"image {i} whole")
    for i in order[-3:]:
        frame, c, _, o, _, qt = imgs[i]
        g = oracle.geometry(frame)
        mh = g["mcu_h"]
        r = g["mcus_y"] // 2
        per_row = c.numel() // g["mcus_y"]
        band = c[(r - 1) * per_row:(r + 2) * per_row].cpu().numpy().reshape(-1, 64)
        sub = dict(frame, height=3 * mh)
        ref = oracle.decode(sub, band, qt, mode)[mh:2 * mh]
        ok &= bool(np.array_equal(o[r * mh:(r + 1) * mh].cpu().numpy(), ref))
        checked.append(f"image {i} MCU row {r}")
    return {"all_equal": ok, "checked": checked}


# ---- CPU baseline: the oracle on the host cores ------------------------------------------------
# The pool is forked before this process touches the GPU; the workers inherit
# the workload and write their bands into one shared anonymous mapping.
_CPU_JOB = {}


def host_cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "os_cpu_count": os.cpu_count(), "usable_cpus": usable}


def _oracle_band(band):
    """Oracle decode of MCU rows [r0, r1): the sub-frame of those rows and
    one neighbour row on each side (all a fancy h2v2 band depends on), its
    middle rows written into the shared output."""
    import oracle
    r0, r1 = band
    frame, coef, qt, buf = _CPU_JOB["frame"], _CPU_JOB["coef"], _CPU_JOB["qt"], _CPU_JOB["buf"]
    g = oracle.geometry(frame)
    mh, W, H = g["mcu_h"], frame["width"], frame["height"]
    per_row = g["mcus_x"] * g["blocks_per_mcu"]
    a, b = max(r0 - 1, 0), min(r1 + 1, g["mcus_y"])
    sub = dict(frame, height=min(H, b * mh) - a * mh)
    rgb = oracle.decode(sub, coef[a * per_row:b * per_row], qt, "fancy")
    y0, y1 = r0 * mh, min(H, r1 * mh)
    out = np.frombuffer(buf, dtype=np.uint8).reshape(H, W, 3)
    out[y0:y1] = rgb[y0 - a * mh:y1 - a * mh]
    return y1 - y0


def cpu_baseline(frame, coef, qt, seconds):
    """The oracle, as it stands, timed on the host: one core (whole-image
    decodes) and all usable cores (a process pool over MCU-row bands of the
    same image).  Returns (baseline entry, the oracle's RGB)."""
    import mmap
    import multiprocessing as mp

    import oracle
    W, H = frame["width"], frame["height"]
    info = host_cpu_info()
    reps, t1 = 0, 0.0
    ref = None
    while t1 < seconds or reps == 0:
        t = time.perf_counter()
        ref = oracle.decode(frame, coef, qt, "fancy")
        t1 += time.perf_counter() - t
        reps += 1
    one = W * H * reps / t1 / 1e6
    n = max(1, min(16, info["usable_cpus"] or 1))
    g = oracle.geometry(frame)
    rows = g["mcus_y"]
    per_band = max(1, -(-rows // (2 * n)))      # about two bands per worker
    bands = [(r, min(rows, r + per_band)) for r in range(0, rows, per_band)]
    buf = mmap.mmap(-1, W * H * 3)
    _CPU_JOB.update(frame=frame, coef=coef, qt=qt, buf=buf)
    with mp.get_context("fork").Pool(n) as pool:
        pool.map(_oracle_band, bands)            # warm the workers
        reps_n, tn = 0, 0.0
        while tn < seconds or reps_n == 0:
            t = time.perf_counter()
            pool.map(_oracle_band, bands, chunksize=1)
            tn += time.perf_counter() - t
            reps_n += 1
    pooled = np.frombuffer(buf, dtype=np.uint8).reshape(H, W, 3).copy()
    _CPU_JOB.clear()
    buf.close()
    many = W * H * reps_n / tn / 1e6
    entry = {"value": round(many, 3), "unit": "MPix/s", "cores": n, "kind": "oracle",
             "sample": f"{reps_n} decodes of the {W}x{H} 4:2:0 fancy image, each as {len(bands)} bands of "
                       f"{per_band} MCU rows over a pool of {n} processes (a band decodes one neighbour MCU row "
                       f"on each side, {2 * len(bands) - 2} extra rows per image); numpy",
             "one_core": {"value": round(one, 3), "unit": "MPix/s", "cores": 1,
                          "sample": f"{reps} whole-image decodes, one process"},
             "pool_speedup": round(many / one, 2),
             "bands_equal_whole_image": bool(np.array_equal(pooled, ref)),
             "host": info}
    return entry, ref


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the decode path has no "
                                   "multi-GPU mode (images or MCU-row bands shard with no communication)"}))
        sys.exit(2)
    from synth import workloads

    log("generating the 4096x3072 workload")
    t0 = time.time()
    frame, coef, qt = workloads.large_420_fancy()
    gen_s = time.time() - t0
    cpu, ref = None, None
    if not args.no_cpu_baseline:
        # before this process initialises the GPU: the pool is forked
        log("timing the oracle on the host (one core, then a process pool)")
        cpu, ref = cpu_baseline(frame, coef, qt, args.cpu_seconds)

    import torch

    import paper_1311_5304_amd as M

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = M.Context(0)
    W, H = frame["width"], frame["height"]
    g = M.mjd_geometry_of(frame)
    coef_bytes = coef.nbytes
    rgb_bytes = W * H * 3
    q_dev = torch.from_numpy(qt.view(np.int16)).to(dev)
    c_sets = [torch.from_numpy(coef).to(dev) for _ in range(args.sets)]
    o_sets = [torch.empty((H, W, 3), dtype=torch.uint8, device=dev) for _ in range(args.sets)]
    stream = torch.cuda.current_stream()

    tuning = None
    if not args.no_tune:
        from paper_1311_5304_amd import autotune
        log("headline launch shape (tuning cache, else the autotuner)")
        entry, source = autotune.tuned_image(ctx, frame, M.MJD_UPSAMPLE_FANCY, c_sets, q_dev, o_sets,
                                             retune=args.retune)
        tuning = tuning_report(entry, source)

    # copy-kernel bandwidth over the same byte count (read half, write half),
    # measured first: it also brings the GPU to its working clocks before the
    # headline's warm-up steps (the setup before it is host work only)
    n = ((coef_bytes + rgb_bytes) // 2) // 16 * 16
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
    copy_report = {"copy_GBps": round(2 * n / (copy_ms * 1e-3) / 1e9, 1), "copy_bytes_per_launch": 2 * n}
    del src, dst

    # the call's arguments marshalled once (the frame struct, device
    # addresses, the stream handle), so a step costs the host one C call
    frame_c = M.make_frame(frame)
    addrs = [(c.data_ptr(), o.data_ptr()) for c, o in zip(c_sets, o_sets)]
    q_addr, stream_h = q_dev.data_ptr(), stream.cuda_stream

    def step(i):
        ca, oa = addrs[i % args.sets]
        M.mjd_decode(ctx, frame_c, ca, q_addr, M.MJD_UPSAMPLE_FANCY, oa, 3 * W, 0, g["mcus_y"], stream_h)

    log("timing the headline decode")
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
    extras = {"generation_s": round(gen_s, 2), "tuning": tuning or {"source": "library default",
                                                                     **M.mjd_ctx_get_tuning(ctx)}}
    extras.update(copy_report)
    if ref is not None:
        gpu_out = o_sets[(args.steps - 1) % args.sets].cpu().numpy()
        extras["bit_exact_vs_oracle"] = bool(np.array_equal(gpu_out, ref))

    # the workloads below decode other sizes: library default launch shape
    M.mjd_ctx_set_tuning(ctx, 0, 0, 0)

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
        # end to end on the host clock: pinned coefficients in, decode, RGB
        # back to pinned host memory, synchronised per image
        c1h = torch.from_numpy(c1).pin_memory()
        o1h = torch.empty((256, 256, 3), dtype=torch.uint8).pin_memory()
        e2e = []
        for i in range(1100):
            t = time.perf_counter()
            c1d.copy_(c1h, non_blocking=True)
            M.mjd_decode(ctx, f1, c1d, q1d, M.MJD_UPSAMPLE_SIMPLE, o1, 768, 0, g1["mcus_y"], stream)
            o1h.copy_(o1, non_blocking=True)
            stream.synchronize()
            if i >= 100:
                e2e.append((time.perf_counter() - t) * 1e6)
        e2e = np.array(e2e)
        import oracle
        extras["small_256x256_420_simple_end_to_end_us"] = {
            "p50": round(float(np.percentile(e2e, 50)), 2), "p99": round(float(np.percentile(e2e, 99)), 2),
            "reps": len(e2e), "path": "pinned H2D of the coefficients, decode, D2H of RGB, stream sync",
            "bit_exact": bool(np.array_equal(o1h.numpy(), oracle.decode(f1, c1, q1, "simple")))}

    if not args.no_batch:
        del c_sets, o_sets
        torch.cuda.empty_cache()
        extras["batch"] = batch_workload(args, M, ctx, dev, stream)
        torch.cuda.empty_cache()
    if not args.no_variants:
        extras["variants"] = variants_workload(args, M, ctx, dev)
    if not args.no_pipeline:
        extras["pipeline"] = pipeline_workload(args, M, ctx, dev)
    model = None
    if not args.no_model:
        extras["model"], model = model_workload(args, M, ctx, dev)
    if not args.no_serve:
        extras["serve"] = serve_workload(args, M, ctx, dev, model)

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
                     "unit": "GB/s", "frac": round(achieved_gbs / HBM_PEAK_GBS, 4), "traffic": profiled_traffic()},
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
