"""Kernel resources checked on the CPU from the gfx950 assembly: no kernel
spills to scratch memory, and the raster kernels keep to at most 128 VGPRs
at the sorter depths the tuner uses for light frames (4 waves per SIMD),
with LDS to match."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    import sys
    sys.path.insert(0, os.path.join(ROOT, "paper_2405_13364_amd"))
    import build as B
    out = tmp_path_factory.mktemp("isa") / "k.s"
    cmd = [B.HIPCC, "-x", "hip", "--cuda-device-only", "-S", os.path.join(B.CSRC, "lr_kernels.hip"), "-o", str(out)]
    cmd += [f for f in B.FLAGS if f != "-fPIC"]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    s = out.read_text()
    res = {}
    for m in re.finditer(r"\.amdhsa_kernel (\S+)\n(.*?)\.end_amdhsa_kernel", s, re.S):
        body = m.group(2)
        res[m.group(1)] = {
            "scratch": int(re.search(r"private_segment_fixed_size (\d+)", body).group(1)),
            "vgpr": int(re.search(r"next_free_vgpr (\d+)", body).group(1)),
            "lds": int(re.search(r"group_segment_fixed_size (\d+)", body).group(1)),
        }
    assert len(res) > 20
    return res


def test_no_kernel_uses_scratch(kernels):
    assert {k: v["scratch"] for k, v in kernels.items() if v["scratch"]} == {}


def test_raster_register_budget(kernels):
    # release variants: depth 4..16 exact (flat colours), depth 4 and 8 with
    # the transmittance cutoff or vertex colours
    seen = 0
    for name, v in kernels.items():
        if "k_raster" in name and (re.search(r"ILi(4|8|12|16)ELb0E.*ELb0ELb0EEEvT", name) or
                                   re.search(r"ILi(4|8)ELb0E.*ELb(1ELb0|0ELb1)EEEvT", name)):
            assert v["vgpr"] <= 128, (name, v["vgpr"])
            seen += 1
    assert seen >= 20


def test_raster_lds_allows_sixteen_waves_per_cu(kernels):
    """A raster workgroup of NW waves must leave room for 16 / NW of them per
    CU (160 KiB of LDS), so LDS does not cut occupancy below 4 waves/SIMD."""
    seen = 0
    for name, v in kernels.items():
        m = re.search(r"k_raster.*Li(\d+)ELb[01]ELb[01]EEEvT", name)
        if m:
            nw = int(m.group(1))
            assert (16 // nw) * v["lds"] <= 160 * 1024, (name, nw, v["lds"])
            seen += 1
    assert seen > 0
