"""Encoder side of the synthetic workloads on the GPU (torch), for the
workloads too large to generate with numpy in a benchmark run.

Same recipe as synth.encode / synth.images.gradient_rgb (JFIF colour
transform, edge padding, rounded-mean chroma downsampling, FP64 forward DCT,
rounding quantiser, MCU-order interleave), with the random draws taken from a
seeded torch CUDA generator.  Floating-point rounding may differ from the
numpy path in rare ties, so the coefficients are not promised identical to
synth.encode's; every parity check compares the decoder and the oracle on
the same coefficient array.
"""
from __future__ import annotations

import math

import numpy as np

from .encode import SAMPLINGS, make_frame, mcu_grid
from .tables import quant_tables


def _dct_matrix(torch, device):
    m = np.empty((8, 8), dtype=np.float64)
    for k in range(8):
        ck = math.sqrt(0.5) if k == 0 else 1.0
        for n in range(8):
            m[k, n] = 0.5 * ck * math.cos((2 * n + 1) * k * math.pi / 16.0)
    return torch.from_numpy(m).to(device)


def gradient_ycc(torch, width: int, height: int, seed: int, sigma: float, device):
    """Seeded gradient + noise RGB content, converted to rounded YCbCr int planes [3, H, W]."""
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    x = torch.arange(width, device=device, dtype=torch.float64)[None, :] / width
    y = torch.arange(height, device=device, dtype=torch.float64)[:, None] / height
    chans = []
    for _ in range(3):
        p = torch.rand(4, generator=g, device=device, dtype=torch.float64)
        a = 32 + 192 * p[0]
        b, c, e = (p[1:] * 192 - 96)
        chans.append(a + b * x + c * y + e * x * y)
    rgb = torch.stack(chans)
    rgb = rgb + sigma * torch.randn(rgb.shape, generator=g, device=device, dtype=torch.float64)
    rgb = torch.clamp(torch.floor(rgb + 0.5), 0, 255)
    r, gg, b = rgb[0], rgb[1], rgb[2]
    ycc = torch.stack([0.299 * r + 0.587 * gg + 0.114 * b,
                       -0.168736 * r - 0.331264 * gg + 0.5 * b + 128.0,
                       0.5 * r - 0.418688 * gg - 0.081312 * b + 128.0])
    return torch.clamp(torch.floor(ycc + 0.5), 0, 255)


def texture_ycc(torch, width: int, height: int, seed: int, sigma: float, device):
    """Seeded texture content (gradient + 8 sinusoids, periods log-uniform in
    4..64 px, amplitudes U[4, 24], per-channel gains U[0.7, 1.3], plus noise)
    -> rounded YCbCr planes [3, H, W].  Each plane wave
    sin(u*x + v*y + phi) is formed as sin(u x) cos(v y + phi) + cos(u x) sin(v y + phi)
    from row and column vectors."""
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    f64 = torch.float64
    xs = torch.arange(width, device=device, dtype=f64)
    ys = torch.arange(height, device=device, dtype=f64)
    x = xs[None, :] / width
    y = ys[:, None] / height
    chans = []
    for _ in range(3):
        p = torch.rand(4, generator=g, device=device, dtype=f64)
        a = 32 + 192 * p[0]
        b, c, e = (p[1:] * 192 - 96)
        chans.append(a + b * x + c * y + e * x * y)
    tex = torch.zeros((height, width), device=device, dtype=f64)
    for _ in range(8):
        p = torch.rand(4, generator=g, device=device, dtype=f64)
        period = torch.exp(math.log(4.0) + p[0] * (math.log(64.0) - math.log(4.0)))
        amp = 4 + 20 * p[1]
        theta = math.pi * p[2]
        phi = 2 * math.pi * p[3]
        u = 2 * math.pi * torch.cos(theta) / period
        v = 2 * math.pi * torch.sin(theta) / period
        sx, cx = torch.sin(u * xs), torch.cos(u * xs)
        sy, cy = torch.sin(v * ys + phi), torch.cos(v * ys + phi)
        tex += amp * (cy[:, None] * sx[None, :] + sy[:, None] * cx[None, :])
    gains = 0.7 + 0.6 * torch.rand(3, generator=g, device=device, dtype=f64)
    rgb = torch.stack([chans[k] + gains[k] * tex for k in range(3)])
    rgb = rgb + sigma * torch.randn(rgb.shape, generator=g, device=device, dtype=f64)
    rgb = torch.clamp(torch.floor(rgb + 0.5), 0, 255)
    r, gg, b = rgb[0], rgb[1], rgb[2]
    ycc = torch.stack([0.299 * r + 0.587 * gg + 0.114 * b,
                       -0.168736 * r - 0.331264 * gg + 0.5 * b + 128.0,
                       0.5 * r - 0.418688 * gg - 0.081312 * b + 128.0])
    return torch.clamp(torch.floor(ycc + 0.5), 0, 255)


def encode_ycc(torch, frame: dict, ycc, qt: np.ndarray, device):
    """YCbCr planes [3, H, W] (float64 integers) -> int16 coefficients [n_blocks, 64] on device."""
    mx, my = mcu_grid(frame)
    hmax, vmax = max(frame["h"]), max(frame["v"])
    pw, ph = mx * 8 * hmax, my * 8 * vmax
    d = _dct_matrix(torch, device)
    grids = []
    for c in range(3):
        plane = ycc[c]
        h, w = plane.shape
        plane = torch.nn.functional.pad(plane[None, None], (0, pw - w, 0, ph - h), mode="replicate")[0, 0]
        fh, fv = hmax // frame["h"][c], vmax // frame["v"][c]
        if fh > 1 or fv > 1:
            n = fh * fv
            s = plane.reshape(ph // fv, fv, pw // fh, fh).sum(dim=(1, 3))
            plane = torch.floor((s + n // 2) / n)
        gh, gw = plane.shape[0] // 8, plane.shape[1] // 8
        blocks = (plane.reshape(gh, 8, gw, 8).permute(0, 2, 1, 3) - 128.0).contiguous()
        coefs = torch.matmul(torch.matmul(d, blocks), d.t().contiguous())  # D X D^T per block
        q = torch.from_numpy(qt[frame["qsel"][c]].astype(np.float64)).to(device).reshape(8, 8)
        qc = torch.sign(coefs) * torch.floor(torch.abs(coefs) / q + 0.5)
        hc, vc = frame["h"][c], frame["v"][c]
        qc = qc.reshape(my, vc, mx, hc, 64).permute(0, 2, 1, 3, 4).reshape(my, mx, vc * hc, 64)
        grids.append(qc)
    return torch.cat(grids, dim=2).reshape(-1, 64).to(torch.int16).contiguous()


def batch_image_gpu(torch, spec, device, sigma: float = 8.0, content: str = "gradient"):
    """One image of synth.workloads.batch_specs / corpus_specs, generated on the GPU.

    -> (frame, coef int16 [n_blocks*64] on device, qt uint16[4][64] numpy)."""
    w, h, sampling, q, seed = spec
    assert sampling in SAMPLINGS
    frame = make_frame(w, h, sampling)
    qt = quant_tables(q)
    make = gradient_ycc if content == "gradient" else texture_ycc
    ycc = make(torch, w, h, seed, sigma, device)
    coef = encode_ycc(torch, frame, ycc, qt, device)
    return frame, coef.reshape(-1), qt
