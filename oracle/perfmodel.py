"""The paper's performance model, written out plainly (oracle; test
infrastructure only).

Sec. 5.1: each decoding phase's time is a polynomial fitted to measured
times, of degree at most seven, the degree chosen by comparing the Akaike
information criterion of the fits; the Huffman time is a per-pixel rate,
itself a polynomial in the entropy density d = file size / (w * h)
(Eqs. 3-4); the GPU time is the host->device transfer, the kernel and the
device->host transfer added up.

Readings (the paper names the tools, not their details):
  * least squares on the monomials x^i (one variable) or a^i b^j with
    i + j <= degree (two variables);
  * AIC = n ln(RSS / n) + 2k for n samples and k terms, over the degrees
    whose k is below n; a residual sum below 1e-24 of sum(y^2) counts as
    that floor, so that among exact fits the one with fewest terms wins;
  * the GPU parts are fitted against the scaled dimensions w / 1024 and
    h / 1024.

The fit is numpy's least-squares solver on a design matrix built term by
term; evaluation is the sum of the terms as defined (no Horner form), so a
reader can check it against the definition.
"""
from __future__ import annotations

import math

import numpy as np

MAX_DEGREE = 7
EXACT_FLOOR = 1e-24


def terms2(degree: int):
    """(i, j) exponent pairs of a, b with i + j <= degree, grouped by i."""
    return [(i, j) for i in range(degree + 1) for j in range(degree + 1 - i)]


def aic(rss: float, sumsq: float, n: int, k: int) -> float:
    floor = EXACT_FLOOR * (sumsq if sumsq > 0 else 1.0)
    return n * math.log(max(rss, floor) / n) + 2 * k


def _fit(columns, y):
    A = np.array(columns, dtype=np.float64).T
    coef, _, rank, _ = np.linalg.lstsq(A, y, rcond=None)
    if rank < A.shape[1]:
        return None, None
    r = y - A @ coef
    return coef, float(r @ r)


def fit1(x, y, max_degree: int = MAX_DEGREE):
    """-> (degree, coefficients c[i] of x^i, AIC) of the least-AIC fit."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    n = len(y)
    sumsq = float(y @ y)
    best = None
    for deg in range(max_degree + 1):
        k = deg + 1
        if k >= n:
            break
        coef, rss = _fit([x ** i for i in range(k)], y)
        if coef is None:
            continue
        a = aic(rss, sumsq, n, k)
        if best is None or a < best[2]:
            best = (deg, coef, a)
    return best


def fit2(a, b, y, max_degree: int = MAX_DEGREE):
    """-> (degree, coefficients in terms2(degree) order, AIC)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    y = np.asarray(y, np.float64)
    n = len(y)
    sumsq = float(y @ y)
    best = None
    for deg in range(max_degree + 1):
        t = terms2(deg)
        if len(t) >= n:
            break
        coef, rss = _fit([a ** i * b ** j for i, j in t], y)
        if coef is None:
            continue
        v = aic(rss, sumsq, n, len(t))
        if best is None or v < best[2]:
            best = (deg, coef, v)
    return best


def eval1(degree: int, coef, x: float) -> float:
    return float(sum(coef[i] * x ** i for i in range(degree + 1)))


def eval2(degree: int, coef, a: float, b: float) -> float:
    return float(sum(c * a ** i * b ** j for c, (i, j) in zip(coef, terms2(degree))))


def predict(model, width: int, height: int, file_bytes: int) -> dict:
    """model: {"huff_per_pixel": (deg, coef), "o_w"|"t_kernel"|"o_r": (deg, coef)}
    -> the Eq. 3-4 terms and their sums, in seconds."""
    px = width * height
    a, b = width / 1024.0, height / 1024.0
    d = file_bytes / px
    out = {"d": d, "t_huff": eval1(*model["huff_per_pixel"], d) * px}
    for part in ("o_w", "t_kernel", "o_r"):
        out[part] = eval2(*model[part], a, b)
    out["p_gpu"] = out["o_w"] + out["t_kernel"] + out["o_r"]
    out["total"] = out["t_huff"] + out["p_gpu"]
    return out


# ---- CPU-GPU partitioning (Sec. 5.2) --------------------------------------------------------
# The GPU decodes the first rows, the CPU the last x (reading of the paper's
# equations, which name x the CPU's rows).  Huffman time of r rows is
# huff_per_pixel(d) * w * r / n for n host threads.  After the Huffman
# decoding that precedes the split both sides take:
#   SPS (Eqs. 8-10):      CPU = T_dispatch(w, h - x) + P_cpu(w, x)
#   overlap (Eqs. 12-13): CPU = T_dispatch(w, h - x) + T_huff(w, x, d) + P_cpu(w, x)
#   PPS (Eqs. 14-15):     CPU = T_huff(w, h - c, d) + P_cpu(w, x) + T_dispatch(w, h - x),
#                         c = min(chunk, h - x) the GPU's first chunk
#   and in each            GPU = P_gpu(w, h - x).
# Readings: the overlap scheme's CPU Huffman term covers the CPU's x rows
# (the text: the CPU decodes its own part's entropy data while the GPU
# runs); the first chunk cannot be taller than the GPU's share.

def _huff(model, w, h, file_bytes, rows, n):
    return eval1(*model["huff_per_pixel"], file_bytes / (w * h)) * w * rows / n


def sides(model, scheme: str, w: int, h: int, file_bytes: int, huff_threads: float, x: float, chunk: float = 0.0):
    a = w / 1024.0
    gpu = sum(eval2(*model[p], a, (h - x) / 1024.0) for p in ("o_w", "t_kernel", "o_r"))
    cpu = eval2(*model["t_dispatch"], a, (h - x) / 1024.0) + eval2(*model["p_cpu"], a, x / 1024.0)
    if scheme == "overlap":
        cpu += _huff(model, w, h, file_bytes, x, huff_threads)
    elif scheme == "pps":
        cpu += _huff(model, w, h, file_bytes, h - min(chunk, h - x), huff_threads)
    return cpu, gpu


def best_split(rows: int, mcu_h: int, side_fn):
    """Brute force over every split of `rows` on an MCU-row boundary (the GPU
    takes whole MCU rows from the top) -> (later finish, CPU rows)."""
    best = None
    for r in range(-(-rows // mcu_h) + 1):
        g = min(rows, r * mcu_h)
        x = rows - g
        cpu, gpu = side_fn(x)
        t = max(cpu if x else 0.0, gpu if g else 0.0)
        if best is None or t < best[0]:
            best = (t, x)
    return best


def best_partition(model, scheme: str, w: int, h: int, mcu_h: int, file_bytes: int, huff_threads: float = 1.0,
                   chunk: float = 0.0):
    return best_split(h, mcu_h, lambda x: sides(model, scheme, w, h, file_bytes, huff_threads, x, chunk))


# Re-partitioning before the GPU's last chunk (Eqs. 16-17).  r rows remain to
# be shared (the last chunk's and the CPU's); the Huffman data of u rows is
# still undecoded, after t_done seconds of decoding; the earlier chunks still
# owe the GPU `busy` seconds.  Readings: the undecoded rows' density is
# d' = (max(0, E - t_done) / E) / (u / h) * d with E the model's estimate for
# the whole image (the share of Huffman time left over the share of height
# left); the split of the r rows gives the GPU r - x' (the equation's P_GPU
# argument h - x read as the remainder's r - x'), and the paper's
# P_prevGPU/T_prevGPU is `busy`.
#   CPU = T_dispatch(w, r - x') + T_huff(w, u, d') + P_cpu(w, x')
#   GPU = P_gpu(w, r - x') + busy

def repartition_sides(model, w, h, r, file_bytes, huff_threads, u, t_done, busy, x):
    d = file_bytes / (w * h)
    est = eval1(*model["huff_per_pixel"], d) * w * h / huff_threads
    d_new = (max(0.0, est - t_done) / est) / (u / h) * d if u and est > 0 else 0.0
    a = w / 1024.0
    gpu = sum(eval2(*model[p], a, (r - x) / 1024.0) for p in ("o_w", "t_kernel", "o_r")) + busy
    cpu = (eval2(*model["t_dispatch"], a, (r - x) / 1024.0) + eval1(*model["huff_per_pixel"], d_new) * w * u
           / huff_threads + eval2(*model["p_cpu"], a, x / 1024.0))
    return cpu, gpu


def best_repartition(model, w, h, r, mcu_h, file_bytes, huff_threads, u, t_done, busy):
    return best_split(r, mcu_h, lambda x: repartition_sides(model, w, h, r, file_bytes, huff_threads, u, t_done,
                                                            busy, x))
