"""The per-lane restart-interval decoder of the GPU entropy kernel, run on
the CPU (CPU only): the same template the kernel instantiates, compiled with
g++ over an environment that bounds-checks every table, stream and block
access.  Its coefficients must equal the oracle's reader (T.81 Annex F.2.2
written out bit by bit) and the encoder's input; on corrupted entropy-coded
data it must flag exactly the streams the host decoder rejects, and never
read outside its interval."""
import os
import random
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from synth import bitstream, encode, images

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_1311_5304_amd", "_lib")


@pytest.fixture(scope="module")
def M():
    import paper_1311_5304_amd as mod
    return mod


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    cxx = shutil.which("g++")
    if not cxx:
        pytest.skip("no C++ compiler")
    if not os.path.exists(os.path.join(LIBDIR, "libmjd.so")):
        pytest.skip("libmjd.so is not built")
    exe = str(tmp_path_factory.mktemp("lane") / "entropy_lane_host")
    subprocess.run([cxx, "-O1", "-std=c++17", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_1311_5304_amd", "csrc"),
                    os.path.join(ROOT, "tests", "entropy_lane_host.cpp"), "-o", exe, "-L", LIBDIR, "-lmjd",
                    "-Wl,-rpath," + LIBDIR], check=True)
    return exe


def run_lane(harness, data, tmp_path, name="s"):
    src, dst = tmp_path / f"{name}.jpg", tmp_path / f"{name}.bin"
    src.write_bytes(bytes(data))
    r = subprocess.run([harness, str(src), str(dst)], capture_output=True, text=True)
    assert r.returncode == 0, (r.returncode, r.stderr)
    n_intervals, bad = map(int, r.stdout.split())
    return n_intervals, bad, np.fromfile(dst, dtype=np.int16).reshape(-1, 64)


def _stream(w, h, samp, q, ri, seed):
    rgb = images.texture_rgb(w, h, seed, sigma=12)
    frame, coef, qt = encode.encode_rgb(rgb, samp, q)
    return frame, coef, qt, bitstream.write_jpeg(frame, coef, qt, restart_interval=ri)


@pytest.mark.parametrize("samp", ["444", "422", "420"])
@pytest.mark.parametrize("ri", [0, 1, 3, 32])
def test_lane_matches_oracle_reader(harness, tmp_path, samp, ri):
    for (w, h, seed) in ((1, 1, 1), (17, 9, 2), (45, 38, 3), (130, 67, 4)):
        frame, coef, qt, data = _stream(w, h, samp, 85, ri, seed)
        _, c_or, _ = oracle.parse_and_decode(data)
        n, bad, c = run_lane(harness, data, tmp_path)
        assert bad == 0
        assert np.array_equal(c, c_or)
        assert np.array_equal(c, coef)


def test_lane_extreme_values_and_long_codes(M, harness, tmp_path):
    """Largest baseline magnitudes, ZRL runs, coefficient 63, and random
    blocks whose optimal codes exceed the 9-bit look-ahead (the canonical
    code walk) with many stuffed 0xFF bytes."""
    frame = encode.make_frame(16, 8, "444")
    coef = np.zeros((6, 64), dtype=np.int16)
    coef[0, 0], coef[1, 0], coef[2, 0] = 1023, -1024, 0
    coef[3, 0], coef[4, 0], coef[5, 0] = -1024, 1023, 1
    coef[0, 63] = -1023
    coef[1, 17] = 1023
    coef[2, 1:64] = np.arange(1, 64)
    coef[5, 1:64:17] = -700
    qt = np.ones((4, 64), dtype=np.uint16)
    rng = np.random.default_rng(5)
    cases = [(frame, coef)]
    for samp, w, h in (("420", 80, 64), ("422", 30, 10), ("444", 24, 16)):
        fr = encode.make_frame(w, h, samp)
        nb = oracle.geometry(fr)["n_blocks"]
        # magnitude categories 1..10 with probability halving per category:
        # the rare ones get codes longer than the look-ahead
        size = np.minimum(rng.geometric(0.5, size=(nb, 64)), 10)
        mag = (1 << (size - 1)) + (rng.random((nb, 64)) * (1 << (size - 1))).astype(np.int64)
        c = np.where(rng.random((nb, 64)) < 0.5, -mag, mag).astype(np.int16)
        c[:, 0] = rng.integers(-1023, 1024, size=nb)
        c[rng.random((nb, 64)) < 0.4] = 0
        cases.append((fr, c))
    stuffed = long_codes = 0
    for fr, c in cases:
        for ri in (0, 1, 2):
            data = bitstream.write_jpeg(fr, c, qt, restart_interval=ri)
            scan, _ = M.mjd_parse(data)
            stuffed += data.count(b"\xFF\x00")
            long_codes += sum(sum(t.bits[9:]) for t in scan.ac)
            _, bad, got = run_lane(harness, data, tmp_path)
            assert bad == 0
            assert np.array_equal(got, c)
    assert stuffed > 0 and long_codes > 0


def test_lane_flags_corruption_like_the_host_decoder(M, harness, tmp_path):
    """Random bytes of the entropy-coded data replaced (markers and stuffing
    left alone so the restart index stays valid): the lane decoder rejects
    an interval exactly when the host decoder rejects the stream, decodes
    the same coefficients when both accept it, and stays inside its interval
    (the harness exits 3 on any access outside it)."""
    rnd = random.Random(11)
    streams = [_stream(130, 67, "420", 85, 3, 4), _stream(64, 48, "444", 60, 1, 5), _stream(90, 40, "422", 95, 0, 6)]
    seen = {True: 0, False: 0}
    for frame, coef, qt, data in streams:
        scan, _ = M.mjd_parse(data)
        off = M.mjd_restart_index(data, scan)
        g = M.mjd_geometry_of(frame)
        s0, s1 = scan.data_offset, scan.data_end
        for k in range(25):
            b = bytearray(data)
            for _ in range(rnd.choice((1, 1, 2, 6))):
                p = rnd.randrange(s0, s1)
                if b[p] == 0xFF or b[p - 1] == 0xFF:
                    continue
                b[p] = rnd.choice([v for v in range(255)])
            host = np.zeros((g["n_blocks"], 64), dtype=np.int16)
            try:
                M.mjd_entropy_decode(bytes(b), scan, off, host, 0, g["mcus_y"], 1)
                host_ok = True
            except M.MjdError as e:
                assert e.code == -5
                host_ok = False
            _, bad, got = run_lane(harness, b, tmp_path)
            assert (bad == 0) == host_ok
            if host_ok:
                assert np.array_equal(got, host)
            seen[host_ok] += 1
    assert seen[True] > 5 and seen[False] > 5
