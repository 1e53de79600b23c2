"""Register and scratch use of every kernel in the last build, from the
compiler's resource-usage remarks that build() records: no kernel may spill
registers to scratch memory (a spill in the segment decoder once made the
batched launch 60% slower while every output stayed bit-exact).  No GPU
needed."""
import json
import os

import pytest

from paper_1311_5304_amd import build as B


def resources():
    if not os.path.exists(B.RESOURCES):
        pytest.fail(f"{B.RESOURCES} is missing: run `python -m paper_1311_5304_amd.build` first")
    with open(B.RESOURCES) as f:
        return json.load(f)


def test_every_kernel_listed():
    r = resources()
    names = " ".join(r)
    for k in ("decode_segments", "decode_segments_aan", "decode_batch", "copy16", "entropy"):
        assert k in names, k


def test_no_kernel_uses_scratch():
    bad = {k: v for k, v in resources().items() if v.get("ScratchSize", 0) or v.get("VGPRs Spill", 0)}
    assert not bad, json.dumps(bad, indent=1)


def test_segment_decoders_fit_two_waves_per_simd():
    # 2 waves per SIMD (256 registers) is what the launch shapes assume
    for k, v in resources().items():
        if "decode_segments" in k or "decode_batch" in k:
            assert v["VGPRs"] <= 256 and v["Occupancy"] >= 2, (k, v)


def test_parse_resource_remarks():
    text = ("a.hip:1:1: remark: Function Name: _Zk1 [-Rpass-analysis=kernel-resource-usage]\n"
            "a.hip:1:1: remark:     VGPRs: 173 [-Rpass-analysis=kernel-resource-usage]\n"
            "a.hip:1:1: remark:     ScratchSize [bytes/lane]: 8 [-Rpass-analysis=kernel-resource-usage]\n"
            "a.hip:1:1: remark:     Occupancy [waves/SIMD]: 2 [-Rpass-analysis=kernel-resource-usage]\n"
            "a.hip:9:1: remark: Function Name: _Zk2 [-Rpass-analysis=kernel-resource-usage]\n"
            "a.hip:9:1: remark:     VGPRs Spill: 3 [-Rpass-analysis=kernel-resource-usage]\n")
    r = B.parse_resource_remarks(text)
    assert r == {"_Zk1": {"VGPRs": 173, "ScratchSize": 8, "Occupancy": 2}, "_Zk2": {"VGPRs Spill": 3}}
