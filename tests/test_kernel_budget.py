"""Register budget of the sweep instantiations (host-side check of the
compiled gfx950 code; no GPU needed).

VGPRs are allocated in granules of 8 out of 512 per SIMD lane, so 7 waves per
SIMD allow at most 72.  Every instantiation is compiled for 7 waves.  The
words of the state P that do not fit are spilled, which is cheap only if no
scratch access lands on the path every 64-step block takes.  That path is
found in the compiled code itself: the basic blocks of the loop holding the
phase-1 steps (the loop with the 3-input logic ops 0x5c) that dominate all of
its back edges, i.e. run on every iteration.  Blocks that run only when a lane
passed the fast filter, or once per 4096 steps, are not on it.

sweep_kernel<8, 4, 10> holds about 99% of the benchmark's vectors: no scratch
access on its per-block path.  The wider templates are allowed one reload per
block (a 64-bit value; about 0.2% of the block's VALU work).
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


def basic_blocks(txt, tag):
    """Basic blocks of one kernel: name, loop comments, instructions."""
    lines = txt.split("\n")
    start = next(i for i, l in enumerate(lines) if re.match(r"^_ZN3wpm12sweep_kernel" + tag + r"\S*:", l))
    end = next(i for i in range(start, len(lines)) if lines[i].startswith(".Lfunc_end"))
    blocks, cur = [], None
    for l in lines[start + 1:end]:
        m = re.match(r"^(\.LBB\d+_\d+):(.*)$", l) or re.match(r"^; (%bb\.\d+):(.*)$", l)
        if m:
            cur = {"name": m.group(1), "comment": [m.group(2)], "ins": []}
            blocks.append(cur)
            continue
        if cur is None:
            cur = {"name": "entry", "comment": [""], "ins": []}
            blocks.append(cur)
        s = l.strip()
        if s.startswith(";"):
            if not cur["ins"]:
                cur["comment"].append(s)
        elif s and not s.startswith("."):
            cur["ins"].append(s)
    for b in blocks:
        c = " ".join(b["comment"])
        m = re.search(r"Header=BB(\d+_\d+)", c)
        b["header"] = b["name"] if "Loop Header" in c else (".LBB" + m.group(1) if m else None)
        b["parents"] = [".LBB" + x for x in re.findall(r"Parent Loop BB(\d+_\d+)", c)]
    return blocks


def successors(blocks):
    idx = {b["name"]: i for i, b in enumerate(blocks)}
    out = []
    for i, b in enumerate(blocks):
        last = b["ins"][-1] if b["ins"] else ""
        op = last.split()[0] if last else ""
        s = []
        if (op.startswith("s_cbranch") or op == "s_branch") and last.split()[-1] in idx:
            s.append(idx[last.split()[-1]])
        if op not in ("s_branch", "s_endpgm") and i + 1 < len(blocks):
            s.append(i + 1)
        out.append(s)
    return out


def per_block_path(txt, tag):
    """(scratch accesses, phase-1 logic ops) on the blocks that every
    iteration of the phase-1 loop executes."""
    blocks = basic_blocks(txt, tag)
    weight = {}
    for b in blocks:
        n = sum("bitop3:0x5c" in x for x in b["ins"])
        if n and b["header"]:
            weight[b["header"]] = weight.get(b["header"], 0) + n
    loop = max(weight, key=weight.get)
    parents = {b["name"]: b["parents"] for b in blocks if b["header"] == b["name"]}
    members = [i for i, b in enumerate(blocks)
               if b["header"] == loop or loop in parents.get(b["header"], [])]
    succ = successors(blocks)
    head = next(i for i in members if blocks[i]["name"] == loop)
    latches = [i for i in members if head in succ[i]]
    preds = {i: [j for j in members if i in succ[j]] for i in members}
    dom = {i: set(members) for i in members}
    dom[head] = {head}
    changed = True
    while changed:
        changed = False
        for i in members:
            if i == head:
                continue
            ps = [dom[p] for p in preds[i]]
            nd = (set.intersection(*ps) if ps else set()) | {i}
            if nd != dom[i]:
                dom[i], changed = nd, True
    hot = set.intersection(*[dom[l] for l in latches])
    scratch = [x for i in hot for x in blocks[i]["ins"] if re.match(r"scratch_(load|store)", x)]
    steps = sum(sum("bitop3:0x5c" in x for x in blocks[i]["ins"]) for i in hot)
    return scratch, steps


@pytest.mark.parametrize("qs,wm,allowed", [(4, 10, 0), (4, 4, 0), (4, 16, 1), (4, 32, 2), (8, 10, 1),
                                           (8, 32, 1)])
def test_seven_waves_and_no_spills_per_block(asm, qs, wm, allowed):
    tag = f"ILi8ELi{qs}ELi{wm}E"
    vgpr, _ = meta(asm, "sweep_kernel" + tag)
    assert vgpr <= 72, f"sweep_kernel<8, {qs}, {wm}> uses {vgpr} VGPRs: fewer than 7 waves per SIMD"
    scratch, steps = per_block_path(asm, tag)
    # the path found is the real one: both chains' two logic ops for 32 steps
    assert steps == 64, steps
    assert len(scratch) <= allowed, scratch
