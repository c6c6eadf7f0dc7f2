"""Register budget of the sweep kernel (host-side check of the compiled
gfx950 code; no GPU needed).

One kernel serves every instance shape, compiled for 7 and for 8 waves per
SIMD (at most 72 and 64 VGPRs: VGPRs are allocated in granules of 8 out of
512 per SIMD lane).  Its only per-lane state is the fast filter's four chains;
a check rebuilds any other word from LDS tables.  So the whole kernel, not
just its hot loop, must compile without any scratch access: no spill traffic
reaches memory.  The per-block path -- the basic blocks of the loop holding
the phase-1 steps that dominate all of its back edges, i.e. run on every
64-step block -- is checked for its instruction mix: the 64 steps' logic ops,
no more than 440 VALU instructions, no scalar register reloads from VGPR
lanes, and XORs whose two operands are VGPRs (a scalar operand measured
about 14% slower on the whole sweep).
"""
import os
import re
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, ".."))
from paper_2301_00806_amd import build as BLD  # noqa: E402

SRC = os.path.join(BLD.CSRC, "sweep.hip")


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not os.path.exists(BLD.HIPCC):
        pytest.skip("hipcc not installed")
    out = tmp_path_factory.mktemp("asm") / "sweep.s"
    cmd = ([BLD.HIPCC, "-O3", "-std=c++17"] + BLD.DEVICE + BLD.EXTRA.get("sweep.hip", []) +
           ["--cuda-device-only", "-S", SRC, "-o", str(out)])
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out.read_text()


def meta(txt, tag):
    for blk in txt.split("  - .agpr_count")[1:]:
        name = re.search(r"\.name:\s+(\S+)", blk).group(1)
        if tag in name:
            get = lambda key: int(re.search(r"\." + key + r":\s+(\d+)", blk).group(1))
            return {k: get(k) for k in ("vgpr_count", "vgpr_spill_count", "private_segment_fixed_size")}
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
    """Instructions on the blocks that every iteration of the phase-1 loop
    executes."""
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
    return [x for i in sorted(hot) for x in blocks[i]["ins"]]


def kernel_text(txt, tag):
    lines = txt.split("\n")
    start = next(i for i, l in enumerate(lines) if re.match(r"^_ZN3wpm12sweep_kernel" + tag + r"\S*:", l))
    end = next(i for i in range(start, len(lines)) if lines[i].startswith(".Lfunc_end"))
    return lines[start:end]


@pytest.mark.parametrize("waves,vgprs", [(7, 72), (8, 64)])
def test_no_scratch_and_lean_per_block_path(asm, waves, vgprs):
    tag = f"ILi{waves}E"
    m = meta(asm, "sweep_kernel" + tag)
    assert m["vgpr_count"] <= vgprs, m
    assert m["vgpr_spill_count"] == 0 and m["private_segment_fixed_size"] == 0, m
    assert not [l for l in kernel_text(asm, tag) if re.match(r"\s*(scratch_|buffer_store|buffer_load)", l)]
    path = per_block_path(asm, tag)
    # the path found is the real one: both chains' two logic ops for 32 steps
    assert sum("bitop3:0x5c" in x for x in path) == 64
    valu = [x for x in path if x.startswith("v_")]
    assert len(valu) <= 440, len(valu)
    assert not [x for x in valu if x.startswith("v_readlane")]
    xors = [x for x in valu if x.startswith("v_xor_b32")]
    assert len(xors) >= 4 * 60
    assert not [x for x in xors if re.search(r"\bs\d+\b", x)], "XOR with a scalar operand on the per-block path"
