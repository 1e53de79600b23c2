"""Off-line profiling and fitting of the performance model (paper Sec. 5.1).

The paper times an instrumented decoder once per machine on a training set
of images and fits closed forms to the times:
- the Huffman rate per pixel, against the entropy density d = file bytes /
  (w * h) (Eqs. 3-4);
- the three parts of the GPU time against the image dimensions: the copy of
  the coefficients in, the kernel, and the copy of the RGB out (pinned
  buffers on both sides, as in the paper);
- for the CPU-GPU partitioning (Sec. 5.2), the host's back half of x rows
  (P_CPU) and the host's time to enqueue the GPU's rows (T_dispatch), each
  against the width and the rows of its side.
`measure` times one bitstream's phases on this machine; `fit` turns a list
of measurements into an `mjd_model`; `predict` evaluates it (Horner form, in
the library).  The fits and the evaluation are the library's (include/mjd.h);
this module only measures and marshals.
"""
from __future__ import annotations

import time

import numpy as np

from . import _binding as B

PARTS = ("o_w", "t_kernel", "o_r")
HOST_PARTS = ("p_cpu", "t_dispatch")
# The host parts are fitted at degree 3 at most and must not fall as their
# side's rows grow: a high-degree surface through times measured at only a
# few row counts per width swings between them, where the partition solve
# then looks.
HOST_MAX_DEGREE = 3


def measure(ctx, jpg: bytes, reps: int = 3, upsample: int = B.MJD_UPSAMPLE_FANCY, hetero=None) -> dict:
    """Times one bitstream: Huffman decoding on one host thread (the paper's
    sequential phase), then host->device copy of the coefficients, the decode
    kernel and device->host copy of the RGB (each the best of `reps`).  With
    a heterogeneous decoder (B.Hetero) also the back half on its host threads
    (p_cpu) and the host's time to enqueue the GPU part (t_dispatch)."""
    import torch

    scan, qt = B.mjd_parse(jpg)
    off = B.mjd_restart_index(jpg, scan)
    frame = B.scan_frame(scan)
    g = B.mjd_geometry_of(frame)
    w, h = frame["width"], frame["height"]
    coef_h = torch.empty(g["n_blocks"] * 64, dtype=torch.int16).pin_memory()
    rgb_h = torch.empty(h * w * 3, dtype=torch.uint8).pin_memory()
    t_huff = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        B.mjd_entropy_decode(jpg, scan, off, coef_h, 0, g["mcus_y"], 1)
        t_huff = min(t_huff, time.perf_counter() - t0)
    dev = torch.device("cuda", torch.cuda.current_device())
    coef_d = torch.empty_like(coef_h, device=dev)
    rgb_d = torch.empty((h, w, 3), dtype=torch.uint8, device=dev)
    q_d = torch.from_numpy(qt.view(np.int16)).to(dev)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    best = {k: float("inf") for k in PARTS}
    for _ in range(reps + 1):  # the first pass warms up
        ev[0].record(stream)
        coef_d.copy_(coef_h, non_blocking=True)
        ev[1].record(stream)
        B.mjd_decode(ctx, frame, coef_d, q_d, upsample, rgb_d, 3 * w, 0, g["mcus_y"], stream)
        ev[2].record(stream)
        rgb_h.copy_(rgb_d.view(-1), non_blocking=True)
        ev[3].record(stream)
        torch.cuda.synchronize()
        for k, (a, b) in zip(PARTS, ((0, 1), (1, 2), (2, 3))):
            best[k] = min(best[k], ev[a].elapsed_time(ev[b]) * 1e-3)
    out = {"width": w, "height": h, "bytes": len(jpg), "t_huff": t_huff, **best}
    if hetero is not None:
        # split the image at the quarters: the host's time for its x rows
        # (p_cpu at (w, x)) and the enqueueing of the GPU's h - x rows
        # (t_dispatch at (w, h - x)), each the best of `reps`
        host = []
        for r in sorted({0, g["mcus_y"] // 4, g["mcus_y"] // 2, 3 * g["mcus_y"] // 4, g["mcus_y"]}):
            cpu_rows = h - min(h, r * g["mcu_h"])
            cpu_s = dispatch_s = float("inf")
            for _ in range(reps):
                t = hetero.decode(jpg, rgb_h, 3 * w, cpu_rows, B.MJD_PART_SPS, upsample)
                cpu_s, dispatch_s = min(cpu_s, t["cpu_s"]), min(dispatch_s, t["dispatch_s"])
            if cpu_rows:
                host.append(("p_cpu", w, cpu_rows, cpu_s))
            if cpu_rows < h:
                host.append(("t_dispatch", w, h - cpu_rows, dispatch_s))
        out["host"] = host
    return out


def fit(samples, max_degree: int = B.MJD_POLY_MAX_DEGREE) -> tuple:
    """-> (mjd_model, {part: (degree, AIC)}) from `measure` results."""
    w = np.array([s["width"] for s in samples], np.float64)
    h = np.array([s["height"] for s in samples], np.float64)
    px = w * h
    d = np.array([s["bytes"] for s in samples], np.float64) / px
    model = B.mjd_model()
    info = {}
    p, aic = B.mjd_poly1_fit(d, np.array([s["t_huff"] for s in samples]) / px, max_degree)
    model.huff_per_pixel = p
    info["huff_per_pixel"] = (p.degree, aic)
    for part in PARTS:
        p2, aic = B.mjd_poly2_fit(w / 1024.0, h / 1024.0, np.array([s[part] for s in samples]), max_degree)
        setattr(model, part, p2)
        info[part] = (p2.degree, aic)
    for part in HOST_PARTS:  # against (width, rows) of the part's side
        pts = np.array([x[1:] for s in samples for x in s.get("host", ()) if x[0] == part], np.float64)
        if len(pts):
            a, b = pts[:, 0] / 1024.0, pts[:, 1] / 1024.0
            for deg in range(min(max_degree, HOST_MAX_DEGREE), -1, -1):
                p2, aic = B.mjd_poly2_fit(a, b, pts[:, 2], deg)
                if rows_monotone(p2, a.min(), a.max(), b.max()):
                    break
            setattr(model, part, p2)
            info[part] = (p2.degree, aic)
    return model, info


def rows_monotone(p2, a_lo: float, a_hi: float, b_hi: float, n: int = 48) -> bool:
    """True when the fitted surface does not fall as its second argument
    (rows / 1024) grows from 0 to b_hi, at every width of [a_lo, a_hi]
    (checked on an n x n grid)."""
    for a in np.linspace(a_lo, a_hi, n):
        v = [B.mjd_poly2_eval(p2, float(a), float(b)) for b in np.linspace(0.0, b_hi, n)]
        if any(y1 < y0 - 1e-9 for y0, y1 in zip(v, v[1:])):
            return False
    return True


def host_errors(model, samples, absolute: bool = False) -> dict:
    """Errors of the host parts' predictions against `measure` results taken
    with a heterogeneous decoder: {part: [|pred - meas| / meas]}, or in
    seconds with absolute=True."""
    out = {part: [] for part in HOST_PARTS}
    for s in samples:
        for part, w, rows, t in s.get("host", ()):
            pred = B.mjd_poly2_eval(getattr(model, part), w / 1024.0, rows / 1024.0)
            out[part].append(abs(pred - t) if absolute else abs(pred - t) / t)
    return out


def host_times(samples) -> dict:
    """{part: [measured seconds]} of the host parts in `measure` results."""
    out = {part: [] for part in HOST_PARTS}
    for s in samples:
        for part, _, _, t in s.get("host", ()):
            out[part].append(t)
    return out


def predict(model, width: int, height: int, file_bytes: int) -> dict:
    return B.mjd_model_predict(model, width, height, file_bytes)


def to_dict(model) -> dict:
    """A JSON-able copy of the model's coefficients."""
    out = {"huff_per_pixel": {"degree": model.huff_per_pixel.degree,
                              "c": list(model.huff_per_pixel.c)[:model.huff_per_pixel.degree + 1]}}
    for part in PARTS + HOST_PARTS:
        p = getattr(model, part)
        out[part] = {"degree": p.degree, "c": list(p.c)[:(p.degree + 1) * (p.degree + 2) // 2]}
    return out


def from_dict(d: dict):
    model = B.mjd_model()
    model.huff_per_pixel.degree = d["huff_per_pixel"]["degree"]
    for i, c in enumerate(d["huff_per_pixel"]["c"]):
        model.huff_per_pixel.c[i] = c
    for part in PARTS + HOST_PARTS:
        if part not in d:
            continue
        p = getattr(model, part)
        p.degree = d[part]["degree"]
        for i, c in enumerate(d[part]["c"]):
            p.c[i] = c
    return model
