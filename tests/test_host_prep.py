"""Host-side engine logic against the oracle (no GPU needed).

The packed table is interpreted on the CPU (tests/tablesim.py) and its
accepted set compared with the oracle's enumeration; candidates, ridges and
kernel dimensions are compared with the oracle's own routines.
"""
import ctypes
import itertools
import random

import numpy as np
import pytest

import oracle as O
import wpm_inputs as W
from paper_2301_00806_amd import _lib as L
from paper_2301_00806_amd import engine as E
import tablesim as TS


def test_library_exports_every_declared_symbol():
    import re, os
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "wpm.h")).read()
    declared = set(re.findall(r"\b(wpm_[a-z_]+)\s*\(", hdr))
    lib = L.lib()
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(L.EXPORTED)


def test_strerror_codes():
    lib = L.lib()
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.wpm_strerror(code)
    assert lib.wpm_strerror(-99) == b"unknown status"


@pytest.mark.parametrize("seed", range(6))
def test_candidates_ridges_k_match_oracle(seed):
    rng = random.Random(seed)
    n = rng.randint(2, 7)
    m = n + rng.randint(1, 5)
    lam = [rng.randrange(1 << n) for _ in range(m)]
    F = E.candidates(n, m, lam)
    assert list(F) == O.candidates(n, m, lam)
    if len(F) == 0 or n < 2:
        return
    ridges, B, k = E.kernel_basis(n, m, F)
    assert list(ridges) == O.ridges(n, list(F))
    assert k == O.kernel_dim(n, list(F))
    # every basis vector is in the kernel: each ridge meets it evenly
    for t in range(k):
        chosen = [int(F[j]) for j in range(len(F)) if (int(B[t, j // 32]) >> (j % 32)) & 1]
        for r in ridges:
            assert sum(1 for f in chosen if f & int(r) == int(r)) % 2 == 0


def test_ubt_bound_matches_oracle():
    for n in range(2, 12):
        assert E.ubt_bound(n) == O.ubt_bound(n)


def _instances_small():
    out = [("fano", 3, 7, W.fano().lam, None)]
    out.append(("octa", 2, 6, [1, 2, 1, 2, 3, 3], None))
    k5 = [(1 << a) | (1 << b) for a, b in itertools.combinations(range(6), 2)]
    out.append(("K6", 2, 6, None, k5))
    for i, inst in enumerate(W.batch(O.kdim_of, count=8)):
        if inst.meta["k"] <= 14:
            out.append((f"batch{i}", inst.n, inst.m, inst.lam, None))
    return out


@pytest.mark.parametrize("case", _instances_small(), ids=lambda c: c[0])
def test_packed_table_semantics_match_oracle(case):
    name, n, m, lam, facets = case
    p = E.prepare(n, m, lam=lam, facets=facets)
    mf = p.max_facets
    want = O.enumerate_wpm(n, [int(f) for f in p.facets], mf)
    got_x = TS.survivors_direct(p.table)
    got = sorted(TS.facets_of_x(p.basis, p.facets, x) for x in got_x)
    assert got == want
    assert TS.survivors_walk(p.table, cbits=7) == got_x


def test_walk_with_larger_chunks():
    inst = [i for i in W.batch(O.kdim_of, count=16) if 12 <= i.meta["k"] <= 13][0]
    p = E.prepare(inst.n, inst.m, lam=inst.lam)
    assert TS.survivors_walk(p.table, cbits=9) == TS.survivors_direct(p.table)


def test_walk_across_4096_step_segments():
    # chunks of 2^13 steps: the segment row takes row 12 once inside each
    # chunk, and the second segment's candidates use Gray bit 11 toggled by
    # its parity
    inst = [i for i in W.batch(O.kdim_of, count=64) if 14 <= i.meta["k"] <= 15][0]
    p = E.prepare(inst.n, inst.m, lam=inst.lam)
    assert p.k >= 14
    assert TS.survivors_walk(p.table, cbits=13) == TS.survivors_direct(p.table)


def test_walk_with_unaligned_items_and_coset():
    # items whose first chunk is not a multiple of their lane count (the lane
    # offset from the item's aligned reference is then nonzero), in a coset
    # (the offset row is part of the reference state)
    inst = [i for i in W.batch(O.kdim_of, count=64) if 14 <= i.meta["k"] <= 16][0]
    p = E.prepare(inst.n, inst.m, lam=inst.lam)
    assert TS.survivors_walk(p.table, cbits=7, lanes=48, offset_first=5) == TS.survivors_direct(p.table)
    K = TS.facets_of_x(p.basis, p.facets, TS.survivors_direct(p.table)[0])
    q = E.prepare(inst.n, inst.m, lam=inst.lam, forced_in=[K[0]])
    assert q.offset is not None and q.k >= 8
    assert TS.survivors_walk(q.table, cbits=7, lanes=64, offset_first=3) == TS.survivors_direct(q.table)


def test_pack_rejects_large_k_and_bad_input():
    lib = L.lib()
    info = L.InstanceInfo()
    F = np.array([0b011, 0b101, 0b110], dtype=np.uint32)
    B = np.zeros(70 * 1, dtype=np.uint32)
    st = lib.wpm_pack_instance(2, 3, E._ptr(F), 3, E._ptr(B), 70, None, None, 0, 0, None, 0, ctypes.byref(info))
    assert st == L.WPM_EKMAX
    bad = np.array([0b011, 0b011], dtype=np.uint32)  # duplicate facet
    st = lib.wpm_pack_instance(2, 3, E._ptr(bad), 2, E._ptr(B), 0, None, None, 0, 0, None, 0, ctypes.byref(info))
    assert st == L.WPM_EINVAL
    wrong = np.array([0b111], dtype=np.uint32)  # size 3, n = 2
    No, ko = ctypes.c_int32(), ctypes.c_int32()
    st = lib.wpm_kernel_basis(2, 3, E._ptr(wrong), 1, None, 0, ctypes.byref(No), None, 0, ctypes.byref(ko))
    assert st == L.WPM_EINVAL
    lam = np.array([1, 2, 9], dtype=np.uint32)  # column 9 has bits above n = 2
    Mo = ctypes.c_int32()
    out = np.zeros(8, np.uint32)
    assert lib.wpm_build_candidates(2, 3, E._ptr(lam), E._ptr(out), 8, ctypes.byref(Mo)) == L.WPM_EINVAL


def test_build_queue_skips_k0():
    items = E.build_queue(np.array([0, 8, 0], dtype=np.int32), 7, 64)
    assert set(items["instance"].tolist()) == {1}


def test_build_queue_covers_every_chunk_once():
    k = np.array([7, 12, 20, 9], dtype=np.int32)
    for cb, lanes, mx, order in [(7, 64, 0, 0), (10, 256, 0, 1), (7, 128, 4, 1)]:
        items = E.build_queue(k, cb, lanes, cost=np.array([1, 2, 3, 4], np.float32),
                              max_items_per_instance=mx, order=order)
        for i, kk in enumerate(k):
            mine = items[items["instance"] == i]
            covered = sum(int(it["lanes"]) << int(it["cbits"]) for it in mine)
            assert covered == 1 << max(int(kk), 7)
            spans = sorted((int(it["first"]) << int(it["cbits"]),
                            (int(it["first"]) + int(it["lanes"])) << int(it["cbits"])) for it in mine)
            for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
                assert a1 == b0
            if mx:
                assert len(mine) <= mx
        if order == 1:
            cost = [float([1, 2, 3, 4][it["instance"]]) * (int(it["lanes"]) << int(it["cbits"])) for it in items]
            assert cost == sorted(cost, reverse=True)


def test_pack_bins_assigns_every_item_once_lpt():
    k = np.array([7, 12, 16, 9, 20], dtype=np.int32)
    items = E.build_queue(k, 9, 64, min_items_per_instance=2)
    cost = np.array([1.0, 0.5, 2.0, 1.0, 0.25], np.float32)
    out, offs, mx = E.pack_bins(items, 7, cost)
    assert offs[0] == 0 and offs[-1] == len(items)
    key = lambda a: sorted((int(i["instance"]), int(i["first"]), int(i["cbits"])) for i in a)
    assert key(out) == key(items)
    c = lambda it: float(cost[it["instance"]]) * int(it["lanes"]) * (1 << int(it["cbits"]))
    loads = [sum(c(out[j]) for j in range(offs[b], offs[b + 1])) for b in range(7)]
    assert abs(max(loads) - mx) < 1e-6 * mx
    # LPT bound: makespan <= 4/3 * OPT, and OPT >= max(mean load, largest item)
    lower = max(sum(loads) / 7, max(c(it) for it in items))
    assert max(loads) <= 4.0 / 3.0 * lower + 1e-9 * lower


def test_single_hip_runtime_in_process():
    # libwpm.so must bind to the HIP runtime torch already loaded (one runtime
    # per process: shared streams and device memory)
    import os
    L.lib()
    maps = open(f"/proc/{os.getpid()}/maps").read()
    hips = {l.split()[-1] for l in maps.splitlines() if "libamdhip64" in l}
    assert len(hips) == 1, hips


def test_launch_class_split_keeps_every_item():
    k = np.array([7, 12, 16, 9, 20], dtype=np.int32)
    items = E.build_queue(k, 9, 64)

    class FakeBatch:
        cls = np.array([40416, 20416, 40416, 80416, 20416])
    out, segs = E.split_by_class(FakeBatch, items)
    assert len(out) == len(items) and segs[0].start == 0 and segs[-1].end == len(items)
    assert [s.cls for s in segs] == [80416, 40416, 20416]
    for s in segs:
        assert set(FakeBatch.cls[out[s.start:s.end]["instance"]]) == {s.cls}


def test_build_queue_count_only_and_caller_array():
    # the per-class plans count each class's items first and then fill
    # slices of one (pinned) array: both paths give the plain queue
    k = np.array([12, 0, 9, 15, 7], dtype=np.int32)
    cost = np.array([1, 2, 3, 0.5, 1], np.float32)
    ref = E.build_queue(k, 9, 64, cost=cost, order=1)
    assert E.build_queue(k, 9, 64, cost=cost, order=1, count_only=True) == len(ref)
    buf = np.zeros(len(ref) + 5, dtype=E.ITEM_DTYPE)
    got = E.build_queue(k, 9, 64, cost=cost, order=1, out=lambda n: buf[3:3 + n])
    assert np.array_equal(got, ref) and np.array_equal(buf[3:3 + len(ref)], ref)
    raw = buf.view(np.uint64)
    assert not raw[:6].any() and not raw[2 * (3 + len(ref)):].any()   # untouched outside the slice
    assert E.build_queue(np.zeros(3, np.int32), 9, 64, count_only=True) == 0
    assert len(E.build_queue(np.zeros(3, np.int32), 9, 64, out=lambda n: buf[:n])) == 0


def test_build_queue_groups_and_counts():
    k = np.array([9, 12, 16, 8, 0, 20], dtype=np.int32)
    grp = np.array([1, 3, 1, 2, 3, 3], dtype=np.int32)
    items, per = E.build_queue(k, 9, 64, cost=np.arange(1, 7, dtype=np.float32), order=1,
                               group=grp, return_counts=True)
    g = grp[items["instance"].astype(np.int64)]
    assert list(g) == sorted(g, reverse=True)          # groups in decreasing key
    assert per[4] == 0 and per.sum() == len(items)
    for i in range(len(k)):
        assert (items["instance"] == i).sum() == per[i]


@pytest.mark.parametrize("case", _instances_small(), ids=lambda c: c[0])
def test_deferred_ridges_keep_table_semantics(case):
    # only the filter group (or two groups) resident: the other critical
    # ridges are listed as deferred ridges, checked after the resident groups
    name, n, m, lam, facets = case
    for mg in (1, 2):
        p = E.prepare(n, m, lam=lam, facets=facets, max_groups=mg)
        assert p.info.groups <= mg
        assert p.info.n_deferred >= max(0, p.info.n_crit - 32 * mg)
        want = O.enumerate_wpm(n, [int(f) for f in p.facets], p.max_facets)
        got_x = TS.survivors_direct(p.table)
        assert sorted(TS.facets_of_x(p.basis, p.facets, x) for x in got_x) == want


def test_many_parents_are_deferred_not_rejected():
    # K_11: every vertex (ridge) has 10 parents, more than the slot words hold
    F = [(1 << a) | (1 << b) for a, b in itertools.combinations(range(11), 2)]
    p = E.prepare(2, 11, facets=F, max_facets=0, pack=False)
    E.pack_prepared(p)
    assert p.info.n_deferred == 11 and p.info.groups == 1 and p.info.n_filter == 0
