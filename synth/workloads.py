"""Seeded workload recipes (coefficient-domain inputs for the decoder).

Seeds are (workload_id << 20) | image_index.  Each recipe returns the frame
description, the quantised int16 blocks in MCU order and the uint16[4][64]
quant tables; the pixel content and quality follow the workload's stated
distribution.
"""
from __future__ import annotations

import numpy as np

from .encode import encode_rgb, make_frame, mcu_grid
from .images import gradient_rgb, texture_rgb


def seed_of(workload_id: int, index: int) -> int:
    return (workload_id << 20) | index


def small_420_simple():
    """256x256, 4:2:0, quality 75, gradient content with sigma 8 noise."""
    rgb = gradient_rgb(256, 256, seed_of(1, 0), sigma=8.0)
    frame, coef, qt = encode_rgb(rgb, "420", 75)
    return frame, coef, qt


def large_420_fancy(width: int = 4096, height: int = 3072):
    """4096x3072 (12.6 MP), 4:2:0, quality 90, texture content with sigma 12 noise."""
    rgb = texture_rgb(width, height, seed_of(2, 0), sigma=12.0)
    frame, coef, qt = encode_rgb(rgb, "420", 90)
    return frame, coef, qt


def batch_specs(n: int = 256, lo: int = 320, hi: int = 4096, workload_id: int = 3):
    """Per-image (width, height, sampling, quality, seed) for the mixed batch.

    Width and height are uniform in lo..hi and redrawn while divisible by 16;
    the samplings are split into thirds (4:4:4, 4:2:2, 4:2:0) and shuffled;
    quality is uniform in 50..95."""
    rng = np.random.default_rng(seed_of(workload_id, 0xFFFFF))
    thirds = [n // 3, n // 3, n - 2 * (n // 3)]
    samplings = ["444"] * thirds[0] + ["422"] * thirds[1] + ["420"] * thirds[2]
    rng.shuffle(samplings)
    specs = []
    for i in range(n):
        def draw():
            while True:
                v = int(rng.integers(lo, hi + 1))
                if v % 16:
                    return v
        w, h = draw(), draw()
        q = int(rng.integers(50, 96))
        specs.append((w, h, samplings[i], q, seed_of(workload_id, i)))
    return specs


def corpus_specs(n: int = 1000, mp_lo: float = 1.0, mp_hi: float = 24.0, workload_id: int = 4):
    """Per-image (width, height, sampling, quality, seed) of the bitstream corpus.

    Megapixels uniform in [mp_lo, mp_hi]; aspect ratio 4:3, 3:2 or 16:9 with
    a random orientation; 4:2:0; quality 85."""
    rng = np.random.default_rng(seed_of(workload_id, 0xFFFFF))
    specs = []
    for i in range(n):
        mp = float(rng.uniform(mp_lo, mp_hi))
        a = (4 / 3, 3 / 2, 16 / 9)[int(rng.integers(0, 3))]
        w = int(round((mp * 1e6 * a) ** 0.5))
        h = max(1, int(round(mp * 1e6 / w)))
        if rng.integers(0, 2):
            w, h = h, w
        specs.append((w, h, "420", 85, seed_of(workload_id, i)))
    return specs


def serving_pool(n: int = 96, mp_lo: float = 0.1, mp_hi: float = 24.0, workload_id: int = 5):
    """Distinct request images of the serving trace: megapixels log-uniform in
    [mp_lo, mp_hi], aspect ratio uniform in [3:4, 4:3], samplings in thirds,
    quality uniform in 50..95."""
    rng = np.random.default_rng(seed_of(workload_id, 0xFFFFF))
    thirds = [n // 3, n // 3, n - 2 * (n // 3)]
    samplings = ["444"] * thirds[0] + ["422"] * thirds[1] + ["420"] * thirds[2]
    rng.shuffle(samplings)
    specs = []
    for i in range(n):
        mp = float(np.exp(rng.uniform(np.log(mp_lo), np.log(mp_hi))))
        a = float(rng.uniform(0.75, 4 / 3))
        w = max(1, int(round((mp * 1e6 * a) ** 0.5)))
        h = max(1, int(round(mp * 1e6 / w)))
        specs.append((w, h, samplings[i], int(rng.integers(50, 96)), seed_of(workload_id, i)))
    return specs


def serving_trace(n_requests: int, pool_size: int, rate_per_s: float, workload_id: int = 5):
    """Poisson arrivals: (arrival time in ns from the trace start, pool index) per request."""
    rng = np.random.default_rng(seed_of(workload_id, 0xFFFFE))
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    return [(int(round(x * 1e9)), int(rng.integers(0, pool_size))) for x in t]


def batch_image(spec, sigma: float = 8.0):
    w, h, sampling, q, seed = spec
    rgb = gradient_rgb(w, h, seed, sigma=sigma)
    return encode_rgb(rgb, sampling, q)


def random_coefficients(frame: dict, seed: int, scale: float = 60.0, density: float = 0.3):
    """Random blocks for a frame with no pixel source behind them.

    AC coefficients are Laplacian with a magnitude that decays with frequency
    and are zeroed with probability 1 - density; DC is uniform in +-1016.
    Everything is clipped to +-1023, so with all-ones quant tables the
    dequantised values stay inside the range an 8-bit image can produce."""
    rng = np.random.default_rng(seed)
    mx, my = mcu_grid(frame)
    bpm = sum(h * v for h, v in zip(frame["h"], frame["v"]))
    n = mx * my * bpm
    k = np.arange(64)
    freq = (k // 8) + (k % 8)
    mag = scale / (1.0 + freq)
    c = rng.laplace(0.0, 1.0, size=(n, 64)) * mag
    keep = rng.random((n, 64)) < density
    keep[:, 0] = True
    c = np.where(keep, np.rint(c), 0)
    c[:, 0] = rng.integers(-1016, 1017, size=n)
    return np.clip(c, -1023, 1023).astype(np.int16)


__all__ = ["seed_of", "small_420_simple", "large_420_fancy", "batch_specs", "corpus_specs", "serving_pool",
           "serving_trace", "batch_image",
           "random_coefficients", "make_frame", "mcu_grid"]
