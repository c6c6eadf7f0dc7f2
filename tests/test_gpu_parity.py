"""GPU sweep vs the CPU oracle, through the C ABI (needs an MI355X).

Bit-exact comparison of result sets in vertex-mask space (facet masks of every
weak pseudo-manifold), per instance, plus schedule invariance of the counts.
"""
import itertools
import os
import sys

import numpy as np
import pytest

import oracle as O
import wpm_inputs as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def E():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_00806_amd import engine
    engine.device_query()
    return engine


def run(E, preps, **kw):
    _say(f"[gpu] sweep {len(preps)} instance(s) k={[p.k for p in preps][:8]} {kw}")
    return E.sweep(preps, **kw)


def oracle_sets(preps, node_limit=0):
    return [O.enumerate_wpm(p.n, [int(f) for f in p.facets], p.max_facets, node_limit=node_limit)
            for p in preps]


def test_fano(E):
    f = W.fano()
    for mf in (None, 0):
        p = E.prepare(3, 7, lam=f.lam, max_facets=mf)
        res, sets = run(E, [p])
        want = oracle_sets([p])[0]
        assert sets[0] == want
        assert int(res.counts[0]) == len(want) == res.total


def test_single_n6_m10(E):
    inst = W.single(E.kdim)
    p = E.prepare(inst.n, inst.m, lam=inst.lam)
    assert p.k == inst.meta["k"] == O.kdim_of(inst)
    res, sets = run(E, [p], cbits=12)
    want = oracle_sets([p])[0]
    assert len(sets[0]) == len(want)
    assert sets[0] == want


def test_single_chunks_across_segments(E):
    # 2^14-step chunks: each wave's segment row changes at the 4096-step
    # segment boundaries inside its chunks, and candidates of odd segments use
    # Gray bit 11 toggled by the segment parity
    inst = W.single(E.kdim)
    p = E.prepare(inst.n, inst.m, lam=inst.lam)
    res, sets = run(E, [p], cbits=14, wg_size=64)
    want = oracle_sets([p])[0]
    assert sets[0] == want
    assert int(res.counts[0]) == len(want) == res.total


def test_graphs_many_parents(E):
    # n = 2: ridges are vertices; K_7 and K_8 have 6 and 7 parents per ridge
    preps = []
    for v in (5, 6, 7, 8):
        F = [(1 << a) | (1 << b) for a, b in itertools.combinations(range(v), 2)]
        preps.append(E.prepare(2, v, facets=F, max_facets=0))
    res, sets = run(E, preps)
    assert sets == oracle_sets(preps)
    # dense candidates: blocks overflow the wave's candidate list, so the
    # overflow steps are rechecked from the scalar mask (stats[4])
    assert int(res.stats[4]) > 0


def test_batch_mixed(E):
    insts = [i for i in W.batch(E.kdim, count=96) if i.meta["k"] <= 22][:48]
    preps = E.prepare_many(insts)
    res, sets = run(E, preps, cbits=9)
    want = oracle_sets(preps)
    for i, (g, w) in enumerate(zip(sets, want)):
        assert g == w, f"instance {i} k={preps[i].k}"
    assert res.total == sum(len(w) for w in want)


@pytest.mark.parametrize("waves", [7, 8])
def test_512_thread_workgroups_match_oracle(E, waves):
    # eight waves share one workgroup's staged tables (an autotuner option)
    insts = [i for i in W.batch(E.kdim, count=64) if i.meta["k"] <= 20][:24]
    preps = E.prepare_many(insts)
    batch = E.DeviceBatch(preps)
    sw = E.Sweeper(batch, cap=1 << 20)
    items = E.build_queue(batch.k, 10, 512, cost=np.ones(len(preps), np.float32), order=1)
    assert items["lanes"].max() == 512
    sw.set_items(items)
    _say(f"[gpu] 512-thread workgroups, {waves} waves per SIMD, {len(items)} items")
    sw.launch(2, wg_size=512, waves=waves)
    res = sw.result()
    want = oracle_sets(preps)
    assert sw.collect() == want
    assert list(res.counts) == [len(w) for w in want]


def test_schedule_invariance(E):
    insts = W.batch(E.kdim, count=40)
    preps = E.prepare_many(insts)
    ref = None
    for mode in (0, 1, 2):
        for cbits, wg in ((7, 64), (10, 256), (14, 128)):
            res, _ = run(E, preps, mode=mode, cbits=cbits, wg_size=wg, want_sets=False)
            if ref is None:
                ref = res.counts.copy()
            assert np.array_equal(res.counts, ref), (mode, cbits, wg)
    # LPT order and coarse items give the same counts
    res, _ = run(E, preps, mode=2, cbits=8, order=1, max_items_per_instance=2,
                 cost=np.arange(len(preps), dtype=np.float32), want_sets=False)
    assert np.array_equal(res.counts, ref)


def test_overlapped_record_copies_match_plain_launch(E):
    # Sweeper.launch_fetch splits the largest class into launches and copies
    # each finished slot range while the next launch runs: the same counts
    # and the same multiset of records as one launch and one copy
    from paper_2301_00806_amd import scheduler as S
    insts = [i for i in W.batch(E.kdim, count=96) if i.meta["k"] <= 24][:48]
    preps = E.prepare_many(insts)
    batch = E.DeviceBatch(preps)
    sw = E.Sweeper(batch, cap=1 << 22)

    def real(rec):
        r = np.asarray(rec)
        r = r[r[:, 1] != -1]  # sentinel slots carry the instance ~0
        return r[np.lexsort((r[:, 0], r[:, 1]))]

    for policy in ("dynamic", "static", "packed"):
        plan = S.make_plan(batch, policy, cbits=9, wg=256)
        _say(f"[gpu] launch_fetch {policy}: {len(plan.items)} items, {len(plan.segments)} segments")
        sw.set_items(plan.items, segments=plan.segments)
        got = real(sw.launch_fetch(plan.mode, wg_size=256, parts=4).copy())
        got_counts = sw.counts[:len(preps)].cpu().numpy().copy()
        sw.set_items(plan.items, segments=plan.segments)
        sw.launch(plan.mode, wg_size=256)
        want = real(sw.fetch_records().copy())
        want_counts = sw.counts[:len(preps)].cpu().numpy()
        assert np.array_equal(got_counts, want_counts), policy
        assert np.array_equal(got, want), policy
        assert len(got) == int(want_counts.sum())


def test_records_in_pinned_host_memory(E):
    # the sweep writes its records straight into pinned host memory: the same
    # counts and the same records as with records in device memory
    insts = [i for i in W.batch(E.kdim, count=96) if i.meta["k"] <= 24][:32]
    preps = E.prepare_many(insts)
    batch = E.DeviceBatch(preps)
    items = E.build_queue(batch.k, 10, 256)
    out = []
    for host in (False, True):
        sw = E.Sweeper(batch, cap=1 << 22, records_on_host=host)
        sw.set_items(items)
        _say(f"[gpu] records on host: {host}")
        rec = sw.launch_fetch(2, wg_size=256).copy()
        rec = rec[rec[:, 1] != -1]
        out.append((sw.counts[:len(preps)].cpu().numpy(), rec[np.lexsort((rec[:, 0], rec[:, 1]))]))
        if host:
            assert sw.collect() == oracle_sets(preps)
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert len(out[1][1]) == int(out[1][0].sum())


def test_collect_through_pinned_staging(E):
    # records in HBM, copied by collect into the reserved pinned buffer and
    # read there in place: the oracle's sets, the same as without staging
    insts = [i for i in W.batch(E.kdim, count=96, start=7000) if i.meta["k"] <= 22][:24]
    preps = E.prepare_many(insts)
    batch = E.DeviceBatch(preps)
    sw = E.Sweeper(batch, cap=1 << 22)
    sw.set_items(E.build_queue(batch.k, 10, 256))
    sw.launch(2, wg_size=256)
    plain = sw.collect()
    sw.reserve_host_staging()
    assert sw._staging is not None and sw._staging.is_pinned()
    _say(f"[gpu] collect through pinned staging: {len(preps)} instances")
    staged = sw.collect()
    assert staged == plain == oracle_sets(preps)


def test_capacity_overflow_keeps_counts_exact(E):
    from paper_2301_00806_amd import _lib as L
    f = W.fano()
    p = E.prepare(3, 7, lam=f.lam, max_facets=0)
    full, _ = run(E, [p], want_sets=False)
    batch = E.DeviceBatch([p])
    sw = E.Sweeper(batch, cap=100)
    sw.set_items(E.build_queue(batch.k, 7, 64))
    sw.launch(2, wg_size=64)
    res = sw.result()
    want = O.count_wpm(3, [int(f) for f in p.facets], 0)
    assert res.total == full.total == want and int(res.counts[0]) == want
    with pytest.raises(L.WpmError) as ei:
        sw.collect()
    assert ei.value.status == L.WPM_ECAP


def test_stress_literal_density(E):
    insts = W.stress_literal(count=8)
    preps = E.prepare_many(insts)
    res, sets = run(E, preps)
    assert sets == oracle_sets(preps)


def test_stress_large_k_outputs_verified(E):
    insts = W.stress(E.kdim, count=2)
    preps = E.prepare_many(insts)
    for p in preps:
        assert 32 <= p.k <= 40
    res, sets = run(E, preps, cbits=16, max_items_per_instance=256)
    for p, s in zip(preps, sets):
        F = [int(f) for f in p.facets]
        for K in s:
            assert O.verify(p.n, list(K), F, p.max_facets)
    # the oracle's own enumeration, time-boxed by a node budget
    for p, s in zip(preps, sets):
        try:
            want = O.enumerate_wpm(p.n, [int(f) for f in p.facets], p.max_facets, node_limit=20_000_000)
        except TimeoutError:
            continue
        assert s == want


def test_deferred_ridges_checked_in_the_sweep(E):
    # one or two resident groups: the other critical ridges are checked by
    # the sweep itself before a vector is counted, so counts stay exact
    insts = [i for i in W.batch(E.kdim, count=64) if 14 <= i.meta["k"] <= 22][:12]
    preps = [E.prepare(i.n, i.m, lam=i.lam, max_groups=1 + (j % 2)) for j, i in enumerate(insts)]
    for v in (7, 8):
        F = [(1 << a) | (1 << b) for a, b in itertools.combinations(range(v), 2)]
        preps.append(E.prepare(2, v, facets=F, max_facets=0, max_groups=1))
    assert sum(p.info.n_deferred for p in preps) > 0
    want = oracle_sets(preps)
    for mode, cbits in ((2, 9), (0, 7)):
        res, sets = run(E, preps, mode=mode, cbits=cbits, cap=1 << 22)
        assert sets == want
        assert list(res.counts) == [len(w) for w in want] and res.total == sum(len(w) for w in want)


def test_deferred_ridges_exact_counts_after_record_overflow(E):
    # a record buffer of 64 slots and a single resident group: most records
    # are lost, yet every count equals the oracle's (deferred ridges are
    # checked before counting), and collect reports the overflow
    from paper_2301_00806_amd import _lib as L
    insts = [i for i in W.batch(E.kdim, count=64) if 14 <= i.meta["k"] <= 20 and i.n >= 6][:6]
    preps = [E.prepare(i.n, i.m, lam=i.lam, max_groups=1) for i in insts]
    F = [(1 << a) | (1 << b) for a, b in itertools.combinations(range(8), 2)]
    preps.append(E.prepare(2, 8, facets=F, max_facets=0, max_groups=1))
    assert all(p.info.n_deferred > 0 for p in preps)
    want = [O.count_wpm(p.n, [int(f) for f in p.facets], p.max_facets) for p in preps]
    batch = E.DeviceBatch(preps)
    sw = E.Sweeper(batch, cap=64)
    sw.set_items(E.build_queue(batch.k, 8, 64))
    _say(f"[gpu] deferred ridges, cap 64: {len(preps)} instances")
    sw.launch(2, wg_size=64)
    res = sw.result()
    assert res.slots > 64
    assert [int(c) for c in res.counts] == want and res.total == sum(want)
    with pytest.raises(L.WpmError) as ei:
        sw.collect()
    assert ei.value.status == L.WPM_ECAP


def test_mixed_slot_strides_in_one_launch(E):
    # instances packed with 4 slot words per ridge (the batch workload) and
    # with 8 (complete graphs: ridges of 6 and 7 parents), swept together in
    # one launch: every table is read with its own stride
    insts = [i for i in W.batch(E.kdim, count=48) if i.meta["k"] <= 20][:10]
    preps = E.prepare_many(insts)
    for v in (7, 8):
        F = [(1 << a) | (1 << b) for a, b in itertools.combinations(range(v), 2)]
        preps.append(E.prepare(2, v, facets=F, max_facets=0))
    assert {p.info.slots for p in preps} == {4, 8}
    batch = E.DeviceBatch(preps)
    sw = E.Sweeper(batch, cap=1 << 22)
    sw.set_items(E.build_queue(batch.k, 9, 256), split_classes=False)
    _say(f"[gpu] mixed strides, one launch: {len(preps)} instances")
    sw.launch(2, wg_size=256)
    sw.result()
    assert sw.collect() == oracle_sets(preps)


@pytest.mark.parametrize("waves", [7, 8])
def test_both_register_budgets(E, waves):
    insts = [i for i in W.batch(E.kdim, count=96) if i.meta["k"] <= 22][:24]
    preps = E.prepare_many(insts)
    batch = E.DeviceBatch(preps)
    sw = E.Sweeper(batch, cap=1 << 22)
    sw.set_items(E.build_queue(batch.k, 13, 128))
    _say(f"[gpu] {waves} waves per SIMD: {len(preps)} instances")
    sw.launch(2, wg_size=128, waves=waves)
    sw.result()
    assert sw.collect() == oracle_sets(preps)


def test_malformed_items_are_skipped_and_reported(E):
    # items the kernel must refuse: chunk bits below 7, a lane window that
    # crosses an aligned group of 512 chunks, chunks beyond 2^k, an unknown
    # instance; each is skipped and counted, and the valid items still run
    from paper_2301_00806_amd import _lib as L
    insts = [i for i in W.batch(E.kdim, count=32) if i.meta["k"] <= 16][:2]
    preps = E.prepare_many(insts)
    batch = E.DeviceBatch(preps)
    good = E.build_queue(batch.k, 7, 64)
    bad = np.zeros(4, dtype=E.ITEM_DTYPE)
    bad[0] = (0, 5, 64, 0)                                   # cbits < 7
    bad[1] = (0, 7, 64, 480)                                 # 480 + 64 > 512
    bad[2] = (1, 7, 64, (1 << (max(preps[1].k, 7) - 7)))     # beyond 2^k
    bad[3] = (len(preps), 7, 64, 0)                          # unknown instance
    items = np.concatenate([good, bad])
    sw = E.Sweeper(batch, cap=1 << 20)
    sw.set_items(items, split_classes=False)
    _say("[gpu] malformed items")
    sw.launch(2, wg_size=64)
    torch.cuda.synchronize()
    tot = sw.total.cpu().numpy()
    assert int(tot[2]) == 4
    assert [int(c) for c in sw.counts[:2].cpu().numpy()] == [len(s) for s in oracle_sets(preps)]
    with pytest.raises(L.WpmError):
        sw.result()
    with pytest.raises(L.WpmError) as ei:
        sw.collect()
    assert ei.value.status == L.WPM_EINVAL
