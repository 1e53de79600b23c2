"""Baseline (SOF0) Huffman JPEG writer used to produce test and workload bitstreams.

It takes quantised blocks in MCU order (natural coefficient order) and writes
a sequential-mode interchange file (T.81 Annex B): SOI, DQT, SOF0, DHT, an
optional DRI, one interleaved SOS scan, RSTn markers every `restart_interval`
MCUs, EOI.  Entropy coding follows T.81 F.1.2: the DC difference against the
per-component predictor as (size category, extra bits), the AC coefficients in
zig-zag order as (zero run, size) symbols with ZRL and EOB; 0xFF bytes are
stuffed with 0x00; the bit buffer is padded with 1-bits before every marker;
predictors restart at zero after every RSTn.

Huffman tables are built per image from the symbol counts (T.81 Annex K.2:
code sizes of a Huffman tree over the counts plus one reserved symbol, limited
to 16 bits, reserved code removed, canonical codes assigned in order of size).
"""
from __future__ import annotations

import heapq
import struct

import numpy as np

from .tables import zigzag_order

_ZZ = zigzag_order()


def _category(v: int) -> int:
    return abs(int(v)).bit_length()


def _extra_bits(v: int, s: int) -> int:
    return v if v >= 0 else v + (1 << s) - 1


def _tokens_for_block(block_nat: np.ndarray, pred: int):
    """-> (dc_token, ac_tokens, new_pred); a token is (symbol, nbits, bits)."""
    zz = block_nat[_ZZ]
    dc = int(zz[0])
    diff = dc - pred
    s = _category(diff)
    dc_tok = (s, s, _extra_bits(diff, s))
    ac = []
    nz = np.nonzero(zz[1:])[0] + 1
    last = 0
    for k in nz:
        k = int(k)
        run = k - last - 1
        while run > 15:
            ac.append((0xF0, 0, 0))
            run -= 16
        v = int(zz[k])
        s = _category(v)
        ac.append(((run << 4) | s, s, _extra_bits(v, s)))
        last = k
    if last != 63:
        ac.append((0x00, 0, 0))
    return dc_tok, ac, dc


def _code_lengths(counts: dict) -> tuple[list[int], list[int]]:
    """Huffman code sizes limited to 16 bits -> (BITS[1..16], HUFFVAL)."""
    syms = sorted(counts)
    if not syms:
        syms = [0]
        counts = {0: 1}
    # reserved pseudo-symbol 256 guarantees no code word is all ones
    items = [(counts[s], i, [s]) for i, s in enumerate(syms)] + [(1, len(syms), [256])]
    size = {s: 0 for s in syms}
    size[256] = 0
    heapq.heapify(items)
    tie = len(items)
    while len(items) > 1:
        f1, _, a = heapq.heappop(items)
        f2, _, b = heapq.heappop(items)
        for s in a + b:
            size[s] += 1
        heapq.heappush(items, (f1 + f2, tie, a + b))
        tie += 1
    bits = [0] * 33
    for s, l in size.items():
        bits[l] += 1
    # limit code lengths to 16 (T.81 K.2, Figure K.3)
    for i in range(32, 16, -1):
        while bits[i] > 0:
            j = i - 2
            while bits[j] == 0:
                j -= 1
            bits[i] -= 2
            bits[i - 1] += 1
            bits[j + 1] += 2
            bits[j] -= 1
    i = 16
    while bits[i] == 0:
        i -= 1
    bits[i] -= 1  # drop the reserved code
    order = sorted(syms, key=lambda s: (size[s], s))
    return bits[1:17], order


def _canonical(bits: list[int], vals: list[int]) -> dict:
    codes = {}
    code = 0
    k = 0
    for length in range(1, 17):
        for _ in range(bits[length - 1]):
            codes[vals[k]] = (code, length)
            code += 1
            k += 1
        code <<= 1
    return codes


class _BitWriter:
    def __init__(self):
        self.out = bytearray()
        self.acc = 0
        self.n = 0

    def put(self, value: int, nbits: int):
        if nbits == 0:
            return
        self.acc = (self.acc << nbits) | (value & ((1 << nbits) - 1))
        self.n += nbits
        while self.n >= 8:
            self.n -= 8
            byte = (self.acc >> self.n) & 0xFF
            self.out.append(byte)
            if byte == 0xFF:
                self.out.append(0x00)
        self.acc &= (1 << self.n) - 1

    def flush_ones(self):
        if self.n:
            self.put((1 << (8 - self.n)) - 1, 8 - self.n)


def _segment(marker: int, payload: bytes) -> bytes:
    return struct.pack(">HH", 0xFF00 | marker, len(payload) + 2) + payload


LUMA_CHROMA_TABLES = (0, 1, 1)  # Huffman table set per component: luma 0, chroma 1


def build_tables(dc_counts, ac_counts):
    """Per-table symbol counts -> ([(class, id, BITS, HUFFVAL)], {(class, id): {symbol: (code, length)}})."""
    tables = []
    codes = {}
    for t in range(2):
        for cls, counts in ((0, dc_counts[t]), (1, ac_counts[t])):
            bits, vals = _code_lengths(counts)
            tables.append((cls, t, bits, vals))
            codes[(cls, t)] = _canonical(bits, vals)
    return tables, codes


def headers(frame: dict, qt: np.ndarray, tables, restart_interval: int) -> bytearray:
    """SOI, DQT, SOF0, DHT, optional DRI and SOS: everything before the
    entropy-coded data.  frame["ncomp"] == 1 writes a grayscale frame (one
    component, sampling 1x1, one non-interleaved scan)."""
    nc = frame.get("ncomp", 3)
    hs, vs, qsel = (frame["h"], frame["v"], frame["qsel"]) if nc == 3 else ((1,), (1,), tuple(frame["qsel"][:1]))
    tbl = LUMA_CHROMA_TABLES
    out = bytearray(b"\xFF\xD8")
    for slot in sorted(set(qsel)):
        zz = np.asarray(qt[slot], dtype=np.int64)[_ZZ]
        if zz.max() > 255 or zz.min() < 1:
            raise ValueError("baseline quant tables need entries in 1..255")
        out += _segment(0xDB, bytes([slot]) + bytes(int(v) for v in zz))
    sof = struct.pack(">BHHB", 8, frame["height"], frame["width"], nc)
    for c in range(nc):
        sof += bytes([c + 1, (hs[c] << 4) | vs[c], qsel[c]])
    out += _segment(0xC0, sof)
    for cls, t, bits, vals in tables:
        out += _segment(0xC4, bytes([(cls << 4) | t]) + bytes(bits) + bytes(vals))
    if restart_interval:
        out += _segment(0xDD, struct.pack(">H", restart_interval))
    sos = bytes([nc])
    for c in range(nc):
        sos += bytes([c + 1, (tbl[c] << 4) | tbl[c]])
    sos += bytes([0, 63, 0])
    out += _segment(0xDA, sos)
    return out


def write_jpeg(frame: dict, coef: np.ndarray, qt: np.ndarray, restart_interval: int = 0) -> bytes:
    nc = frame.get("ncomp", 3)
    hs, vs = (frame["h"], frame["v"]) if nc == 3 else ((1,), (1,))
    hmax, vmax = max(hs), max(vs)
    mx = -(-frame["width"] // (8 * hmax))
    my = -(-frame["height"] // (8 * vmax))
    bpm = sum(h * v for h, v in zip(hs, vs))
    n_mcu = mx * my
    coef = np.asarray(coef, dtype=np.int16).reshape(n_mcu, bpm, 64)
    comp_of = [c for c in range(nc) for _ in range(hs[c] * vs[c])]
    tbl = LUMA_CHROMA_TABLES

    # pass 1: tokens and symbol statistics
    tokens = []
    dc_counts = [{}, {}]
    ac_counts = [{}, {}]
    pred = [0, 0, 0]
    for m in range(n_mcu):
        if restart_interval and m % restart_interval == 0:
            pred = [0, 0, 0]
        mt = []
        for b in range(bpm):
            c = comp_of[b]
            dc_tok, ac_toks, pred[c] = _tokens_for_block(coef[m, b], pred[c])
            t = tbl[c]
            dc_counts[t][dc_tok[0]] = dc_counts[t].get(dc_tok[0], 0) + 1
            for a in ac_toks:
                ac_counts[t][a[0]] = ac_counts[t].get(a[0], 0) + 1
            mt.append((t, dc_tok, ac_toks))
        tokens.append(mt)

    tables, codes = build_tables(dc_counts, ac_counts)
    out = headers(frame, qt, tables, restart_interval)
    w = _BitWriter()
    for m, mt in enumerate(tokens):
        if restart_interval and m and m % restart_interval == 0:
            w.flush_ones()
            w.out += bytes([0xFF, 0xD0 + ((m // restart_interval - 1) & 7)])
        for t, dc_tok, ac_toks in mt:
            code, length = codes[(0, t)][dc_tok[0]]
            w.put(code, length)
            w.put(dc_tok[2], dc_tok[1])
            for sym, nb, val in ac_toks:
                code, length = codes[(1, t)][sym]
                w.put(code, length)
                w.put(val, nb)
    w.flush_ones()
    out += w.out
    out += b"\xFF\xD9"
    return bytes(out)
