"""The JPEG writer of synth.bitstream with its entropy coder in C++, for the
large corpora: the same headers (synth.bitstream.headers), the same
per-image optimal Huffman tables (synth.bitstream.build_tables over the
same symbol counts) and the same entropy-coded bytes, so the files are
byte-identical to synth.bitstream.write_jpeg."""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import bitstream
from .build_ext import LIB

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is missing: build it with `python -m synth.build_ext`")
        L = ctypes.CDLL(LIB)
        vp, u64, i32, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32
        L.se_symbol_counts.argtypes = [vp, u64, i32, vp, vp, u32, vp]
        L.se_symbol_counts.restype = i32
        L.se_encode.argtypes = [vp, u64, i32, vp, vp, u32, vp, vp, vp, u64]
        L.se_encode.restype = ctypes.c_int64
        _lib = L
    return _lib


def _layout(frame):
    hs, vs = frame["h"], frame["v"]
    hmax, vmax = max(hs), max(vs)
    mx = -(-frame["width"] // (8 * hmax))
    my = -(-frame["height"] // (8 * vmax))
    comp = [c for c in range(3) for _ in range(hs[c] * vs[c])]
    tbl = [bitstream.LUMA_CHROMA_TABLES[c] for c in comp]
    return mx * my, len(comp), np.array(tbl, np.uint8), np.array(comp, np.uint8)


def write_jpeg(frame: dict, coef: np.ndarray, qt: np.ndarray, restart_interval: int = 0) -> bytes:
    coef = np.ascontiguousarray(coef, dtype=np.int16)
    n_mcu, bpm, tbl, comp = _layout(frame)
    if coef.size != n_mcu * bpm * 64:
        raise ValueError("coefficient array does not match the frame")
    counts = np.zeros((4, 256), dtype=np.uint32)
    L = lib()
    if L.se_symbol_counts(coef.ctypes.data, n_mcu, bpm, tbl.ctypes.data, comp.ctypes.data,
                          int(restart_interval), counts.ctypes.data) != 0:
        raise ValueError("bad arguments")
    as_dict = [{int(s): int(c) for s, c in enumerate(row) if c} for row in counts]
    tables, codes = bitstream.build_tables([as_dict[0], as_dict[2]], [as_dict[1], as_dict[3]])
    code_arr = np.zeros((4, 256), dtype=np.uint16)
    len_arr = np.zeros((4, 256), dtype=np.uint8)
    for (cls, t), table in codes.items():
        for sym, (code, length) in table.items():
            code_arr[2 * t + cls, sym] = code
            len_arr[2 * t + cls, sym] = length
    head = bitstream.headers(frame, qt, tables, restart_interval)
    cap = coef.size * 4 + 1024  # a coefficient never needs more than 26 bits + stuffing
    out = np.empty(cap, dtype=np.uint8)
    n = L.se_encode(coef.ctypes.data, n_mcu, bpm, tbl.ctypes.data, comp.ctypes.data, int(restart_interval),
                    code_arr.ctypes.data, len_arr.ctypes.data, out.ctypes.data, cap)
    if n < 0:
        raise RuntimeError(f"entropy coder failed ({n})")
    return bytes(head) + out[:n].tobytes() + b"\xFF\xD9"
