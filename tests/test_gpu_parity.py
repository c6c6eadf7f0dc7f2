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
    # 2^14-step chunks: each lane's state P changes at the 4096-step segment
    # boundaries inside its chunk, and candidates of odd segments use Gray
    # bit 11 toggled by the segment parity
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


def test_deferred_ridges_verification_pass(E):
    # one or two resident groups: the other critical ridges are checked on
    # the survivor records by the verification pass, counts stay exact
    insts = [i for i in W.batch(E.kdim, count=64) if 14 <= i.meta["k"] <= 22][:12]
    preps = [E.prepare(i.n, i.m, lam=i.lam, max_groups=1 + (j % 2)) for j, i in enumerate(insts)]
    for v in (7, 8):
        F = [(1 << a) | (1 << b) for a, b in itertools.combinations(range(v), 2)]
        preps.append(E.prepare(2, v, facets=F, max_facets=0, max_groups=1))
    assert sum(p.info.n_deferred for p in preps) > 0
    want = oracle_sets(preps)
    # with one resident group every vector of K_8 is a candidate (its ridges
    # have 7 parents, too many for the filter): records before verification
    # exceed the default buffer
    for mode, cbits in ((2, 9), (0, 7)):
        res, sets = run(E, preps, mode=mode, cbits=cbits, cap=1 << 24)
        assert sets == want
        assert list(res.counts) == [len(w) for w in want] and res.total == sum(len(w) for w in want)
