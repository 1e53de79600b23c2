"""Baseline JPEG interchange-format reader and Huffman decoder (oracle; test
infrastructure only).

The paper's decoder front end (Sec. 2: the file is a sequence of segments
carrying the dimensions, the sampling factors, the Huffman and quantisation
tables and the entropy-coded data; Sec. 1 and Sec. 4.5: Huffman decoding is
sequential and runs on the CPU).  The segment syntax, the DECODE / RECEIVE /
EXTEND procedures, DC prediction, zig-zag order and restart markers follow
T.81 (Annex B, F.2.2), written out plainly: one bit at a time, one symbol at
a time.

Output: the frame description, the quantised blocks in MCU order in natural
coefficient order (index 8*row + col), and uint16[4][64] quant tables in
natural order.
"""
from __future__ import annotations

import numpy as np


class JpegError(ValueError):
    pass


def _zigzag():
    """Natural index of each zig-zag position, by stepping along the
    anti-diagonals of the 8x8 grid and turning at its borders."""
    order = []
    r = c = 0
    up = True
    for _ in range(64):
        order.append(8 * r + c)
        if up:
            if c == 7:
                r += 1
                up = False
            elif r == 0:
                c += 1
                up = False
            else:
                r -= 1
                c += 1
        else:
            if r == 7:
                c += 1
                up = True
            elif c == 0:
                r += 1
                up = True
            else:
                r += 1
                c -= 1
    return order


ZIGZAG = _zigzag()


class _Huffman:
    """Canonical code from BITS/HUFFVAL (T.81 C.2, F.2.2.3)."""

    def __init__(self, bits, vals):
        self.vals = list(vals)
        self.mincode = [0] * 17
        self.maxcode = [-1] * 18
        self.valptr = [0] * 17
        code = 0
        k = 0
        for length in range(1, 17):
            n = bits[length - 1]
            if n:
                self.valptr[length] = k
                self.mincode[length] = code
                code += n
                k += n
                self.maxcode[length] = code - 1
            code <<= 1
        self.maxcode[17] = 1 << 20
        if k != len(self.vals):
            raise JpegError("DHT counts do not match its values")


class _BitReader:
    def __init__(self, data: bytes, pos: int):
        self.data = data
        self.pos = pos
        self.byte = 0
        self.left = 0
        self.marker = None

    def bit(self) -> int:
        if self.left == 0:
            if self.marker is not None:
                raise JpegError("entropy data ran into a marker")
            if self.pos >= len(self.data):
                raise JpegError("entropy data truncated")
            b = self.data[self.pos]
            self.pos += 1
            if b == 0xFF:
                nxt = self.data[self.pos] if self.pos < len(self.data) else None
                if nxt == 0x00:
                    self.pos += 1
                else:
                    self.marker = nxt
                    self.pos -= 1
                    raise JpegError("entropy data ran into a marker")
            self.byte = b
            self.left = 8
        self.left -= 1
        return (self.byte >> self.left) & 1

    def receive(self, s: int) -> int:
        v = 0
        for _ in range(s):
            v = (v << 1) | self.bit()
        return v

    def decode(self, t: _Huffman) -> int:
        code = self.bit()
        length = 1
        while code > t.maxcode[length]:
            code = (code << 1) | self.bit()
            length += 1
            if length > 16:
                raise JpegError("bad Huffman code")
        return t.vals[t.valptr[length] + code - t.mincode[length]]

    def align_and_expect_rst(self, n: int):
        self.left = 0
        d = self.data
        if self.pos + 1 >= len(d) or d[self.pos] != 0xFF or d[self.pos + 1] != 0xD0 + n:
            raise JpegError(f"expected RST{n}")
        self.pos += 2


def _extend(v: int, s: int) -> int:
    return v - (1 << s) + 1 if s and v < (1 << (s - 1)) else v


def parse_and_decode(data: bytes):
    """-> (frame, coef int16[n_blocks, 64] MCU order natural, qt uint16[4, 64]).

    Any malformed or truncated input raises JpegError."""
    try:
        return _parse(bytes(data))
    except (IndexError, KeyError, ValueError) as e:
        if isinstance(e, JpegError):
            raise
        raise JpegError(f"malformed stream: {e!r}") from e


def _parse(data: bytes):
    if data[:2] != b"\xFF\xD8":
        raise JpegError("missing SOI")
    pos = 2
    qt = np.ones((4, 64), dtype=np.uint16)
    dc_tabs, ac_tabs = {}, {}
    comps = None
    width = height = 0
    restart = 0
    coef = None
    frame = None
    while True:
        while pos < len(data) and data[pos] != 0xFF:
            pos += 1
        while pos < len(data) and data[pos] == 0xFF:
            pos += 1
        if pos >= len(data):
            raise JpegError("missing EOI")
        marker = data[pos]
        pos += 1
        if marker == 0xD9:
            break
        if 0xD0 <= marker <= 0xD7 or marker == 0x01:
            continue
        seglen = (data[pos] << 8) | data[pos + 1]
        seg = data[pos + 2:pos + seglen]
        pos += seglen
        if marker == 0xDB:
            i = 0
            while i < len(seg):
                pq, tq = seg[i] >> 4, seg[i] & 15
                i += 1
                vals = []
                for k in range(64):
                    if pq:
                        vals.append((seg[i] << 8) | seg[i + 1])
                        i += 2
                    else:
                        vals.append(seg[i])
                        i += 1
                for k in range(64):
                    qt[tq, ZIGZAG[k]] = vals[k]
        elif marker in (0xC0, 0xC1):
            if seg[0] != 8:
                raise JpegError("only 8-bit precision")
            height = (seg[1] << 8) | seg[2]
            width = (seg[3] << 8) | seg[4]
            n = seg[5]
            comps = []
            for c in range(n):
                cid, hv, tq = seg[6 + 3 * c:9 + 3 * c]
                comps.append({"id": cid, "h": hv >> 4, "v": hv & 15, "tq": tq})
        elif 0xC2 <= marker <= 0xCF and marker not in (0xC4, 0xC8, 0xCC):
            raise JpegError("only baseline sequential Huffman JPEG is read")
        elif marker == 0xC4:
            i = 0
            while i < len(seg):
                tc, th = seg[i] >> 4, seg[i] & 15
                bits = list(seg[i + 1:i + 17])
                vals = list(seg[i + 17:i + 17 + sum(bits)])
                (ac_tabs if tc else dc_tabs)[th] = _Huffman(bits, vals)
                i += 17 + sum(bits)
        elif marker == 0xDD:
            restart = (seg[0] << 8) | seg[1]
        elif marker == 0xDA:
            if comps is None:
                raise JpegError("SOS before SOF")
            ns = seg[0]
            by_id = {c["id"]: k for k, c in enumerate(comps)}
            order = []
            for j in range(ns):
                cid, tt = seg[1 + 2 * j], seg[2 + 2 * j]
                order.append((by_id[cid], dc_tabs[tt >> 4], ac_tabs[tt & 15]))
            if ns != len(comps) or [o[0] for o in order] != list(range(ns)):
                raise JpegError("only one interleaved scan in frame component order is read")
            frame, coef, pos = _decode_scan(data, pos, width, height, comps, order, restart)
        # APPn, COM and anything else: skipped
    if coef is None:
        raise JpegError("no scan")
    for c, comp in enumerate(comps):
        if comp["tq"] > 3:
            raise JpegError("bad table selector")
    return frame, coef, qt


def _decode_scan(data, pos, width, height, comps, order, restart):
    ncomp = len(comps)
    if ncomp == 1:
        # non-interleaved: one block per MCU, over the component's own block grid
        comps = [dict(comps[0], h=1, v=1)]
    hs = [c["h"] for c in comps]
    vs = [c["v"] for c in comps]
    hmax, vmax = max(hs), max(vs)
    mx = -(-width // (8 * hmax))
    my = -(-height // (8 * vmax))
    bpm = sum(h * v for h, v in zip(hs, vs))
    coef = np.zeros((mx * my, bpm, 64), dtype=np.int16)
    rd = _BitReader(data, pos)
    pred = [0] * ncomp
    restarts = 0
    for m in range(mx * my):
        if restart and m and m % restart == 0:
            rd.align_and_expect_rst(restarts & 7)
            restarts += 1
            pred = [0] * ncomp
        b = 0
        for ci, dct, act in order:
            for _ in range(comps[ci]["h"] * comps[ci]["v"]):
                zz = [0] * 64
                s = rd.decode(dct)
                diff = _extend(rd.receive(s), s)
                pred[ci] += diff
                zz[0] = pred[ci]
                k = 1
                while k < 64:
                    rs = rd.decode(act)
                    r, s = rs >> 4, rs & 15
                    if s == 0:
                        if r == 15:
                            k += 16
                            continue
                        break
                    k += r
                    if k > 63:
                        raise JpegError("AC run past the end of the block")
                    zz[k] = _extend(rd.receive(s), s)
                    k += 1
                for k in range(64):
                    coef[m, b, ZIGZAG[k]] = zz[k]
                b += 1
    frame = {"width": width, "height": height,
             "h": tuple(hs), "v": tuple(vs), "qsel": tuple(c["tq"] for c in comps)}
    return frame, coef.reshape(-1, 64), rd.pos
