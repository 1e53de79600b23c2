"""Host side of the decoder variants (no GPU): the library's variant
geometry equals the oracle's for every sampling and grayscale, and bad
variants are refused before any launch."""
import pytest

import oracle.variants as V


@pytest.fixture(scope="module")
def M():
    import paper_1311_5304_amd as mod
    return mod


CASES = [(37, 21, 1, 1), (37, 21, 2, 1), (37, 21, 1, 2), (37, 21, 2, 2), (37, 21, 4, 1), (1, 1, 4, 1),
         (4096, 3072, 2, 2), (65535, 9, 4, 1)]


@pytest.mark.parametrize("w,h,hy,vy", CASES)
def test_geometry_matches_oracle(M, w, h, hy, vy):
    fr = {"width": w, "height": h, "h": (hy, 1, 1), "v": (vy, 1, 1), "qsel": (0, 1, 1)}
    g, wb = M.mjd_variant_geometry(M.make_variant(fr, 3, "ifast", "fancy"))
    o = V.variant_geometry(fr)
    for k in ("mcu_w", "mcu_h", "mcus_x", "mcus_y", "blocks_per_mcu", "n_blocks"):
        assert g[k] == o[k], k
    assert g["comp_w"] == o["comp_w"] and g["comp_h"] == o["comp_h"]
    # the three sample planes, each a whole block grid with rows padded to 16
    # bytes, 256-byte aligned; at 1/s scale blocks of 8/s samples
    for s in (1, 2, 4, 8):
        g, wb = M.mjd_variant_geometry(M.make_variant(fr, 3, "islow", "fancy", s))
        n = 8 // s
        need = sum(-(-((o["grid_w"][c] * n + 15) // 16 * 16 * o["grid_h"][c] * n) // 256) * 256 for c in range(3))
        # full size decodes in one fused pass: no planes
        assert wb == (need if s > 1 else 0)
        assert g["comp_w"] == [-(-x // s) for x in o["comp_w"]] and g["comp_h"] == [-(-x // s) for x in o["comp_h"]]
    with pytest.raises(M.MjdError) as e:  # the reduced transforms are islow-style only
        M.mjd_variant_geometry(M.make_variant(fr, 3, "float", "fancy", 2))
    assert e.value.code == -2


@pytest.mark.parametrize("w,h", [(29, 19), (8, 8), (1, 1), (65535, 3)])
def test_grayscale_geometry(M, w, h):
    fr = {"width": w, "height": h, "qsel": (2,)}
    g, wb = M.mjd_variant_geometry(M.make_variant(fr, 1, "float"))
    o = V.variant_geometry(dict(fr, ncomp=1))
    assert (g["mcus_x"], g["mcus_y"], g["n_blocks"], g["blocks_per_mcu"]) == (o["mcus_x"], o["mcus_y"],
                                                                              o["n_blocks"], 1)
    assert g["comp_w"] == [w, 0, 0] and g["comp_h"] == [h, 0, 0] and wb == 0


def test_bad_variants_are_refused(M):
    fr = {"width": 64, "height": 64, "h": (2, 1, 1), "v": (2, 1, 1), "qsel": (0, 1, 1)}
    ok = M.make_variant(fr)
    M.mjd_variant_geometry(ok)
    for field, value in (("ncomp", 2), ("idct", 3), ("upsample", 9), ("scale", 3)):
        bad = M.make_variant(fr)
        setattr(bad, field, value)
        with pytest.raises(M.MjdError):
            M.mjd_variant_geometry(bad)
    for hv in (((4, 1, 1), (2, 1, 1)), ((2, 2, 1), (2, 1, 1)), ((3, 1, 1), (1, 1, 1))):
        with pytest.raises(M.MjdError) as e:
            M.mjd_variant_geometry(M.make_variant(dict(fr, h=hv[0], v=hv[1])))
        assert e.value.code == -2  # MJD_EUNSUPPORTED
    with pytest.raises(M.MjdError):
        M.mjd_variant_geometry(M.make_variant(dict(fr, width=0)))
    with pytest.raises(M.MjdError):
        M.mjd_variant_geometry(M.make_variant(dict(fr, qsel=(4, 0, 0))))
