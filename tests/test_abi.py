"""Host-side checks of the C ABI: the library loads, exports everything the
header declares, and its host-only geometry/validation agrees with the
oracle's geometry.  No GPU needed."""
import ctypes
import os
import re

import pytest

import oracle
from paper_1311_5304_amd import _binding as B
from synth.encode import make_frame

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w\s\*]*?\b(mjd_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert {"mjd_decode", "mjd_geometry_of", "mjd_ctx_create", "mjd_last_error", "mjd_ctx_set_tuning"} <= names
    lib = ctypes.CDLL(B.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_geometry_matches_oracle():
    for samp in ("444", "422", "420"):
        for w in list(range(1, 41)) + [65535]:
            for h in (1, 2, 7, 8, 9, 15, 16, 17, 40, 65535):
                f = make_frame(w, h, samp)
                g = B.mjd_geometry_of(f)
                o = oracle.geometry(f)
                for k in ("mcu_w", "mcu_h", "mcus_x", "mcus_y", "blocks_per_mcu", "n_blocks"):
                    assert g[k] == o[k], (samp, w, h, k)
                assert g["comp_w"] == o["comp_w"] and g["comp_h"] == o["comp_h"]


@pytest.mark.parametrize("bad, code", [
    (dict(width=0), B.MJD_EINVAL),
    (dict(height=0), B.MJD_EINVAL),
    (dict(width=65536), B.MJD_EINVAL),
    (dict(qsel=(0, 1, 4)), B.MJD_EINVAL),
    (dict(h=(1, 2, 1), v=(1, 1, 1)), B.MJD_EUNSUPPORTED),
    (dict(h=(1, 1, 1), v=(2, 1, 1)), B.MJD_EUNSUPPORTED),
    (dict(h=(4, 1, 1), v=(1, 1, 1)), B.MJD_EUNSUPPORTED),
    (dict(h=(0, 1, 1), v=(1, 1, 1)), B.MJD_EINVAL),
])
def test_geometry_rejects_bad_frames(bad, code):
    f = dict(make_frame(64, 32, "420"))
    f.update(bad)
    with pytest.raises(B.MjdError) as ei:
        B.mjd_geometry_of(f)
    assert ei.value.code == code
    assert B.mjd_last_error()


def test_tuning_rejects_null_context():
    t = B.mjd_tuning(2, 8, 1)
    assert B.lib().mjd_ctx_set_tuning(None, ctypes.byref(t)) == B.MJD_EINVAL
    assert B.lib().mjd_ctx_get_tuning(None, ctypes.byref(t)) == B.MJD_EINVAL
    s = B.mjd_shape()
    assert B.lib().mjd_shape_info(None, 2, 2, B.MJD_UPSAMPLE_FANCY, 0, ctypes.byref(s)) == B.MJD_EINVAL


def test_shape_lists_per_sampling_class():
    """Every fused sampling class offers several sub-tile shapes to the
    autotuner; other samplings and modes are refused without a GPU."""
    for h, v in ((1, 1), (2, 1), (2, 2)):
        for mode in (B.MJD_UPSAMPLE_SIMPLE, B.MJD_UPSAMPLE_FANCY):
            assert B.mjd_shape_count(h, v, mode) >= 3
    with pytest.raises(B.MjdError) as ei:
        B.mjd_shape_count(1, 2, B.MJD_UPSAMPLE_FANCY)
    assert ei.value.code == B.MJD_EUNSUPPORTED
    with pytest.raises(B.MjdError) as ei:
        B.mjd_shape_count(2, 2, 7)
    assert ei.value.code == B.MJD_EINVAL


STRUCTS = [B.mjd_frame, B.mjd_geometry, B.mjd_tuning, B.mjd_shape, B.mjd_job, B.mjd_huffman, B.mjd_scan,
           B.mjd_pipeline_config, B.mjd_pipeline_stats, B.mjd_server_config, B.mjd_request,
           B.mjd_request_times, B.mjd_entropy_job, B.mjd_poly1, B.mjd_poly2, B.mjd_model, B.mjd_prediction, B.mjd_partition, B.mjd_hetero_times,
           B.mjd_hetero_plan, B.mjd_variant]


def test_frame_struct_layout():
    assert ctypes.sizeof(B.mjd_frame) == 20
    assert ctypes.sizeof(B.mjd_geometry) == 56


def test_binding_structs_match_the_c_header(tmp_path):
    """sizeof/offsetof of every struct of include/mjd.h, as a C compiler
    lays them out, equal the ctypes declarations of the binding."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc:
        pytest.skip("no C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mjd.h"', "int main(void) {"]
    for st in STRUCTS:
        name = st.__name__
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for field, _ in st._fields_:
            lines.append(f'printf("{name}.{field} %zu\\n", offsetof({name}, {field}));')
    lines += ["return 0; }"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                                check=True).stdout.split("\n") if line)
    for st in STRUCTS:
        name = st.__name__
        assert int(out[name]) == ctypes.sizeof(st), name
        for field, _ in st._fields_:
            assert int(out[f"{name}.{field}"]) == getattr(st, field).offset, (name, field)
