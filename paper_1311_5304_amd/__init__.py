"""MI355X (gfx950) JPEG back-half decoder: dequantise -> islow IDCT ->
chroma upsampling -> YCbCr->RGB as one fused HIP kernel behind a C ABI
(include/mjd.h).  PyTorch supplies device memory and streams only.
"""
from __future__ import annotations

from ._binding import (MJD_IDCT_FLOAT, MJD_IDCT_IFAST, MJD_IDCT_ISLOW, MJD_PART_OVERLAP, MJD_PART_PPS, MJD_PART_SPS, MJD_SERVE_CONTINUOUS, MJD_SERVE_SYNC,  # noqa: F401
                       MJD_UPSAMPLE_FANCY, MJD_UPSAMPLE_SIMPLE,
                       Batch, Context, EntropyBatch, Hetero, MjdError, Pipeline, Server, make_variant, mjd_decode_variant, mjd_partition_rows,
                       mjd_repartition_rows, mjd_variant, mjd_variant_geometry,
                       mjd_batch_create, mjd_batch_destroy, mjd_batch_launch, mjd_decode_batch_noalloc,
                       mjd_copy, mjd_ctx_create, mjd_ctx_destroy, mjd_ctx_get_tuning, mjd_ctx_set_tuning, mjd_shape_count, mjd_shape_info,
                       mjd_decode, mjd_decode_host, mjd_entropy_batch_create, mjd_entropy_batch_destroy,
                       mjd_entropy_batch_info, mjd_entropy_batch_launch, mjd_entropy_batch_status,
                       mjd_entropy_decode, mjd_geometry_of, mjd_model, mjd_model_predict, mjd_poly1, mjd_poly2,
                       mjd_poly1_eval, mjd_poly1_fit, mjd_poly2_eval, mjd_poly2_fit, mjd_last_error, mjd_parse,
                       mjd_restart_index, make_frame, scan_frame)

UPSAMPLE = {"simple": MJD_UPSAMPLE_SIMPLE, "fancy": MJD_UPSAMPLE_FANCY}


def decode(ctx: Context, frame, coef, qt, mode: str = "fancy", out=None, rows=None, stream=None):
    """Decode one image (or MCU-row band `rows=(row0, row1)`) on the GPU.

    coef: torch.int16 CUDA tensor with n_blocks*64 elements in MCU order;
    qt: torch uint16/int16 CUDA tensor of 4*64 entries; out: optional
    torch.uint8 CUDA tensor [H, W, 3] (contiguous).  Returns `out`."""
    import torch

    if frame.get("ncomp", 3) != 3:
        raise ValueError("grayscale frames decode with decode_variant(..., ncomp=1)")
    g = mjd_geometry_of(frame)
    if coef.numel() != g["n_blocks"] * 64 or coef.element_size() != 2 or not coef.is_cuda:
        raise ValueError("coef must be a CUDA int16 tensor of n_blocks*64 elements")
    if qt.numel() != 256 or qt.element_size() != 2 or not qt.is_cuda:
        raise ValueError("qt must be a CUDA 16-bit tensor of 4*64 entries")
    if not coef.is_contiguous() or not qt.is_contiguous():
        raise ValueError("coef and qt must be contiguous")
    h, w = int(frame["height"]), int(frame["width"])
    if out is None:
        out = torch.empty((h, w, 3), dtype=torch.uint8, device=coef.device)
    if out.shape != (h, w, 3) or out.dtype != torch.uint8 or not out.is_contiguous():
        raise ValueError("out must be a contiguous uint8 tensor [H, W, 3]")
    r0, r1 = rows if rows is not None else (0, g["mcus_y"])
    mjd_decode(ctx, frame, coef, qt, UPSAMPLE[mode], out, 3 * w, r0, r1, stream)
    return out


def decode_variant(ctx: Context, frame, coef, qt, idct: str = "islow", mode: str = "fancy", ncomp: int = 3,
                   out=None, stream=None, scale: int = 1):
    """Decode one image through the variants path (IDCT method `idct`,
    samplings (1,1), (2,1), (1,2), (2,2), (4,1), or grayscale with ncomp=1;
    output 1/scale of the image for scale 2, 4, 8).  Allocates the plane
    workspace with torch.  Returns `out`: uint8 [H', W', 3], or [H', W'] for
    grayscale, H' = ceil(H / scale), W' = ceil(W / scale)."""
    import torch

    v = make_variant(frame, ncomp, idct, mode, scale)
    g, wb = mjd_variant_geometry(v)
    if coef.numel() != g["n_blocks"] * 64 or coef.element_size() != 2 or not coef.is_cuda:
        raise ValueError("coef must be a CUDA int16 tensor of n_blocks*64 elements")
    if qt.numel() != 256 or qt.element_size() != 2 or not qt.is_cuda:
        raise ValueError("qt must be a CUDA 16-bit tensor of 4*64 entries")
    h, w = -(-int(frame["height"]) // scale), -(-int(frame["width"]) // scale)
    shape = (h, w, 3) if ncomp == 3 else (h, w)
    if out is None:
        out = torch.empty(shape, dtype=torch.uint8, device=coef.device)
    if tuple(out.shape) != shape or out.dtype != torch.uint8 or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous uint8 tensor {shape}")
    work = torch.empty(max(wb, 16), dtype=torch.uint8, device=coef.device)
    mjd_decode_variant(ctx, v, coef, qt, out, ncomp * w, work, wb, stream)
    return out


def entropy_decode(jpg, n_threads: int = 1, out=None):
    """Parse a baseline JPEG and Huffman-decode it on host threads.

    -> (frame dict, coefficients int16 [n_blocks, 64] in MCU order, qt uint16 [4, 64]).
    `out` may be a host buffer (numpy array or pinned tensor) of n_blocks*64 int16."""
    import numpy as np

    scan, qt = mjd_parse(jpg)
    frame = scan_frame(scan)
    g, _ = mjd_variant_geometry(make_variant(frame, frame.get("ncomp", 3)))  # also h1v2, 4:1:1, grayscale
    off = mjd_restart_index(jpg, scan)
    coef = np.empty((g["n_blocks"], 64), dtype=np.int16) if out is None else out
    mjd_entropy_decode(jpg, scan, off, coef, 0, g["mcus_y"], n_threads)
    return frame, coef, qt
