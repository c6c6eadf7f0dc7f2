"""Register budget of the sweep instantiations that carry the benchmark
(host-side check of the compiled gfx950 code; no GPU needed).

VGPRs are allocated in granules of 8 out of 512 per SIMD lane.
  - sweep_kernel<8, 4, 10> runs about 99% of the benchmark's vectors and is
    compiled for 7 waves per SIMD: at most 72 VGPRs.  The spills that costs
    must stay out of the hot loops: none inside the per-step and recorded-step
    loops (loop depth >= 3 in the compiled code), at most a handful at the
    block boundary (depth 2).  5, 6, 7 and 8 waves measured 205.8, 191.1,
    180.4 and 187.3 ms on the benchmark's dominant launch.
  - sweep_kernel<8, 4, 16> keeps 5 waves: at most 96 VGPRs, no spills (97
    would round to 104 and drop to 4 waves, measured 15% slower).
"""
import os
import re
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "..", "paper_2301_00806_amd", "csrc", "sweep_g8.hip")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not installed")
    out = tmp_path_factory.mktemp("asm") / "g8.s"
    cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "--cuda-device-only", "-S", SRC, "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out.read_text()


def meta(txt, tag):
    for blk in txt.split("  - .agpr_count")[1:]:
        name = re.search(r"\.name:\s+(\S+)", blk).group(1)
        if tag in name:
            get = lambda key: int(re.search(r"\." + key + r":\s+(\d+)", blk).group(1))
            return get("vgpr_count"), get("vgpr_spill_count")
    raise AssertionError(tag)


def scratch_by_depth(txt, tag):
    """Scratch accesses of one kernel, by the loop depth of their block."""
    start = next(i for i, l in enumerate(txt.split("\n")) if re.match(r"^_ZN3wpm12sweep_kernel" + tag + r"\S*:", l))
    lines = txt.split("\n")[start:]
    end = next(i for i, l in enumerate(lines) if "s_endpgm" in l)
    depth, hits = 0, {}
    for l in lines[:end]:
        if l.startswith(".LBB"):
            d = re.search(r"Depth=(\d+)", l)
            depth = int(d.group(1)) if d else 0
        if re.search(r"scratch_(load|store)", l):
            hits[depth] = hits.get(depth, 0) + 1
    return hits


def test_dominant_template_fits_seven_waves(asm):
    vgpr, _ = meta(asm, "sweep_kernelILi8ELi4ELi10E")
    assert vgpr <= 72, f"sweep_kernel<8, 4, 10> uses {vgpr} VGPRs: fewer than 7 waves per SIMD"
    hits = scratch_by_depth(asm, "ILi8ELi4ELi10E")
    assert sum(v for d, v in hits.items() if d >= 3) == 0, hits
    assert hits.get(2, 0) <= 4, hits


def test_wide_template_fits_five_waves(asm):
    vgpr, spill = meta(asm, "sweep_kernelILi8ELi4ELi16E")
    assert spill == 0
    assert vgpr <= 96, f"sweep_kernel<8, 4, 16> uses {vgpr} VGPRs: 4 waves per SIMD"
