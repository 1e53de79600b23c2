"""MCU geometry of a frame (oracle; test infrastructure only).

Paper Sec. 2: an image is split into 8x8 blocks and decoded in minimum coded
units; an MCU holds the blocks of every component that cover one region, so
4:4:4 gives an 8x8-pixel MCU and 4:2:2 a 16x8-pixel MCU.  The 4:2:0 case
(16x16) and the component sizes follow the usual T.81 convention (reading):
hmax = max h_i, vmax = max v_i; the MCU is 8*hmax x 8*vmax pixels; component
i has a padded grid of (mcus_y*v_i) x (mcus_x*h_i) blocks and a true size of
ceil(W*h_i/hmax) x ceil(H*v_i/vmax) samples.
"""
from __future__ import annotations


def ceil_div(a: int, b: int) -> int:
    return -(-a // b)


def geometry(frame: dict) -> dict:
    w, h = int(frame["width"]), int(frame["height"])
    hs, vs = tuple(frame["h"]), tuple(frame["v"])
    hmax, vmax = max(hs), max(vs)
    mcus_x = ceil_div(w, 8 * hmax)
    mcus_y = ceil_div(h, 8 * vmax)
    bpm = sum(a * b for a, b in zip(hs, vs))
    return {
        "hmax": hmax, "vmax": vmax,
        "mcu_w": 8 * hmax, "mcu_h": 8 * vmax,
        "mcus_x": mcus_x, "mcus_y": mcus_y,
        "blocks_per_mcu": bpm,
        "n_blocks": mcus_x * mcus_y * bpm,
        "comp_w": [ceil_div(w * hs[i], hmax) for i in range(3)],
        "comp_h": [ceil_div(h * vs[i], vmax) for i in range(3)],
        "grid_w": [mcus_x * hs[i] for i in range(3)],
        "grid_h": [mcus_y * vs[i] for i in range(3)],
    }
