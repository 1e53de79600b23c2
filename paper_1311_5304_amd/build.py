"""Builds the HIP library (libmjd.so) in-tree for gfx950 with hipcc."""
from __future__ import annotations

import json
import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "_lib")
LIB = os.path.join(LIBDIR, "libmjd.so")
BUILD = os.path.join(PKG, "_build")

SOURCES = ["api.hip", "decode.hip", "batch.hip", "copy.hip", "server.hip", "entropy.hip", "variants.hip"]
# host-only C++ (no device code): built with the host compiler
HOST_SOURCES = ["host_common.cpp", "host_jpeg.cpp", "pipeline.cpp", "model.cpp", "cpu_decode.cpp", "hetero.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # integer arithmetic wraps (two's complement); only the descaled results
    # of the transform need to fit in 32 bits
    "-fwrapv",
    # no packed-FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I" + os.path.join(ROOT, "include"),
]


# the float IDCT variant rounds once per operation (no fused multiply-adds)
HIPCC_FILE_FLAGS = {"variants.hip": ["-ffp-contract=off"]}

CXX_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-pthread", "-Wall", "-Wextra", "-Wno-unused-parameter",
             "-I" + os.path.join(ROOT, "include"), "-I" + "/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"]


def cxx() -> str:
    for cand in (os.environ.get("CXX"), shutil.which("g++"), shutil.which("c++")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("no host C++ compiler found")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"command failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r


# per-kernel register, scratch and spill figures of the last build, from the
# compiler's resource-usage remarks (tests check that no kernel spills)
RESOURCES = os.path.join(BUILD, "kernel_resources.json")
_REMARK = re.compile(r"remark:\s+(Function Name|VGPRs|AGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]|"
                     r"VGPRs Spill|SGPRs Spill|LDS Size \[bytes/block\]):\s+(\S+)")


def parse_resource_remarks(text: str) -> dict:
    """{kernel symbol: {figure: value}} from -Rpass-analysis=kernel-resource-usage output."""
    out, cur = {}, None
    for m in _REMARK.finditer(text):
        key, val = m.group(1), m.group(2)
        if key == "Function Name":
            cur = out.setdefault(val, {})
        elif cur is not None:
            cur[key.split(" [")[0]] = int(val) if val.lstrip("-").isdigit() else val
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    objs = []
    cmds = []
    for src in SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmds.append([cc, *HIPCC_FLAGS, *HIPCC_FILE_FLAGS.get(src, []), "-Rpass-analysis=kernel-resource-usage",
                     "-c", os.path.join(CSRC, src), "-o", obj])
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".host.o")
        objs.append(obj)
        cmds.append([cxx(), *CXX_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
    resources = {}
    with ThreadPoolExecutor(max_workers=min(4, len(cmds))) as ex:
        for r in ex.map(_run, cmds):
            resources.update(parse_resource_remarks(r.stderr))
            if verbose and (r.stdout or r.stderr):
                print(r.stdout, r.stderr, file=sys.stderr)
    with open(RESOURCES, "w") as f:
        json.dump(resources, f, indent=1, sort_keys=True)
    tmp = LIB + ".tmp"
    _run([cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
