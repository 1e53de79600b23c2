"""Host robustness on the CPU: the library's host-only C++ (parser, restart
index, threaded Huffman decoder, host back half, worker pool, model fits)
built with AddressSanitizer + UndefinedBehaviorSanitizer and, separately,
with ThreadSanitizer, and driven by tests/host_sanitize_driver.cpp on the
project's bitstreams (several decoded concurrently, 1 and 8 threads each, a
band, a damaged restart interval).  Any sanitizer report or failed check
fails the test; the driver's RGB must equal the oracle's."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from synth import bitstream, encode, images

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1311_5304_amd", "csrc")
HOST_SOURCES = ["host_common.cpp", "host_jpeg.cpp", "model.cpp", "cpu_decode.cpp"]

SANITIZERS = {
    "address_undefined": (["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
                          {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0",
                           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}),
    "thread": (["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1"}),
}


def _build(tmp, flags):
    cxx = shutil.which("g++")
    if not cxx:
        pytest.skip("no g++")
    exe = os.path.join(tmp, "driver")
    cmd = [cxx, "-O1", "-g", "-std=c++17", "-pthread", "-fno-omit-frame-pointer", *flags,
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(ROOT, "tests", "host_sanitize_driver.cpp"),
           *[os.path.join(CSRC, s) for s in HOST_SOURCES], "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise AssertionError(f"sanitizer build failed:\n{r.stderr[-4000:]}")
    return exe


@pytest.fixture(scope="module")
def streams(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    cases = [(203, 77, "420", 85, 3), (130, 67, "422", 60, 1), (95, 120, "444", 90, 5), (64, 48, "420", 75, 0)]
    frames = []
    for i, (w, h, samp, q, ri) in enumerate(cases):
        rgb = images.texture_rgb(w, h, 40 + i, sigma=12)
        frame, coef, qt = encode.encode_rgb(rgb, samp, q)
        (d / f"s{i}.jpg").write_bytes(bitstream.write_jpeg(frame, coef, qt, restart_interval=ri))
        frames.append((frame, coef, qt))
    return str(d), frames


@pytest.mark.parametrize("kind", sorted(SANITIZERS))
def test_host_code_under_sanitizer(tmp_path, streams, kind):
    d, frames = streams
    flags, env_extra = SANITIZERS[kind]
    exe = _build(str(tmp_path), flags)
    env = dict(os.environ, **env_extra)
    env.pop("LD_PRELOAD", None) if kind == "thread" else None
    r = subprocess.run([exe, d, str(len(frames))], capture_output=True, text=True, env=env, timeout=600)
    report = r.stderr
    for marker in ("ERROR: AddressSanitizer", "ERROR: LeakSanitizer", "runtime error:", "WARNING: ThreadSanitizer"):
        assert marker not in report, f"{kind}: sanitizer report\n{report[-6000:]}"
    assert r.returncode == 0, f"{kind}: driver failed ({r.returncode})\n{report[-4000:]}"
    for i, (frame, coef, qt) in enumerate(frames):
        got = np.fromfile(os.path.join(d, f"s{i}.rgb"), dtype=np.uint8).reshape(frame["height"], frame["width"], 3)
        assert np.array_equal(got, oracle.decode(frame, coef, qt, "fancy")), f"stream {i} RGB differs"
