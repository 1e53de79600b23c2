"""Seeded synthetic RGB content standing in for the paper's photo test sets.

The paper's image corpora are not available, so the workloads use seeded
content with a controlled amount of high-frequency energy:

* gradient: per channel a + b*x/W + c*y/H + e*(x/W)*(y/H) with a ~ U[32,224],
  b, c, e ~ U[-96,96], plus N(0, sigma^2) noise, rounded and clamped to 0..255.
* texture: gradient (without its noise) + sum over k=1..8 of
  A_k * sin(2*pi*(x*cos(theta_k) + y*sin(theta_k))/P_k + phi_k) with P_k
  log-uniform in [4, 64] px, A_k ~ U[4, 24], a per-channel gain ~ U[0.7, 1.3],
  plus N(0, sigma^2) noise.

All draws come from numpy.random.default_rng(seed).
"""
from __future__ import annotations

import numpy as np


def _grid(width: int, height: int):
    x = np.arange(width, dtype=np.float64)[None, :] / max(width, 1)
    y = np.arange(height, dtype=np.float64)[:, None] / max(height, 1)
    return x, y


def _to_u8(img: np.ndarray) -> np.ndarray:
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def gradient_rgb(width: int, height: int, seed: int, sigma: float = 8.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x, y = _grid(width, height)
    out = np.empty((height, width, 3), dtype=np.float64)
    for ch in range(3):
        a = rng.uniform(32, 224)
        b, c, e = rng.uniform(-96, 96, size=3)
        out[:, :, ch] = a + b * x + c * y + e * x * y
    out += rng.normal(0.0, sigma, size=out.shape)
    return _to_u8(out)


def texture_rgb(width: int, height: int, seed: int, sigma: float = 12.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x, y = _grid(width, height)
    xs = np.arange(width, dtype=np.float64)[None, :]
    ys = np.arange(height, dtype=np.float64)[:, None]
    base = np.empty((height, width, 3), dtype=np.float64)
    for ch in range(3):
        a = rng.uniform(32, 224)
        b, c, e = rng.uniform(-96, 96, size=3)
        base[:, :, ch] = a + b * x + c * y + e * x * y
    tex = np.zeros((height, width), dtype=np.float64)
    for _ in range(8):
        period = float(np.exp(rng.uniform(np.log(4.0), np.log(64.0))))
        amp = rng.uniform(4, 24)
        theta = rng.uniform(0, np.pi)
        phi = rng.uniform(0, 2 * np.pi)
        tex += amp * np.sin(2 * np.pi * (xs * np.cos(theta) + ys * np.sin(theta)) / period + phi)
    gains = rng.uniform(0.7, 1.3, size=3)
    out = base + tex[:, :, None] * gains[None, None, :]
    out += rng.normal(0.0, sigma, size=out.shape)
    return _to_u8(out)


def flat_rgb(width: int, height: int, rgb=(128, 128, 128)) -> np.ndarray:
    out = np.empty((height, width, 3), dtype=np.uint8)
    out[:, :] = np.asarray(rgb, dtype=np.uint8)
    return out
