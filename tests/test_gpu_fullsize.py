"""Parity at the benchmark's full size, in the launch configuration bench.py
times: the 16384-instance learned-scheduler batch, one persistent launch per
launch class, dynamic queue, 12 chunk bits, 256-thread workgroups.

  - the count of every instance equals the oracle's (golden/learned16384_counts.json,
    written by golden/make_counts.py from the oracle alone);
  - every instance with 1 <= k <= 10, and a sample across every larger k (up to
    the k = 34 maximum of the batch), compared set for set with the oracle;
  - a random sample of survivor records, from all instances, checked by the
    oracle's verifier from their facet lists alone;
  - the counts agree with the total, and with a second schedule (static);
  - the pruned sweep over convenient bases (Section 2.1) gives the same
    counts, and its sampled survivors verify.
"""
import json
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as O
import wpm_inputs as W
from setcheck import kvec, kvec_of_sets, canon, facet_list

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

THREADS = min(16, os.cpu_count() or 1)


def golden_counts():
    with open(os.path.join(os.path.dirname(__file__), "golden", "learned16384_counts.json")) as f:
        g = json.load(f)
    return np.array(g["counts"], dtype=np.uint64)


@pytest.fixture(scope="module")
def run():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_00806_amd import engine as E, scheduler as S
    print("[fullsize] building 16384 instances", flush=True)
    preps = E.prepare_many(W.learned(E.kdim, count=16384))
    batch = E.DeviceBatch(preps)
    sw = E.Sweeper(batch, cap=1 << 26)
    plan = S.make_plan(batch, "dynamic", cbits=12, wg=256)
    sw.set_items(plan.items, segments=plan.segments)
    print(f"[fullsize] sweeping {batch.vectors:.3e} vectors", flush=True)
    sw.launch(plan.mode, wg_size=256)
    res = sw.result()
    rec = sw.fetch_records().copy()
    rec = rec[rec[:, 1] != -1]
    return E, S, preps, batch, sw, res, rec


def test_counts_total_and_schedule_invariance(run):
    E, S, preps, batch, sw, res, rec = run
    assert int(res.counts.sum()) == res.total == len(rec)
    gold = golden_counts()
    bad = np.flatnonzero(res.counts != gold)
    assert len(bad) == 0, f"{len(bad)} instance counts differ from the oracle, first {bad[:8]}"
    plan = S.make_plan(batch, "static", cbits=12, wg=256)
    sw.set_items(plan.items, segments=plan.segments)
    sw.launch(plan.mode, wg_size=256)
    res2 = sw.result()
    assert np.array_equal(res2.counts, res.counts)


def test_sets_match_oracle_small_and_sampled(run):
    E, S, preps, batch, sw, res, rec = run
    ks = np.array([p.k for p in preps])
    rng = np.random.default_rng(11)
    chosen = list(np.flatnonzero((ks >= 1) & (ks <= 10)))
    for k in sorted(set(ks[ks > 10])):
        idx = np.flatnonzero(ks == k)
        chosen += list(rng.choice(idx, size=min(3, len(idx)), replace=False))
    print(f"[fullsize] oracle on {len(chosen)} instances", flush=True)
    order = np.argsort(rec[:, 1], kind="stable")
    rs = rec[order]
    starts = np.searchsorted(rs[:, 1], np.arange(len(preps)))
    ends = np.searchsorted(rs[:, 1], np.arange(len(preps)), side="right")

    def one(i):
        p = preps[i]
        want = O.enumerate_wpm(p.n, [int(f) for f in p.facets], p.max_facets)
        got = canon(kvec(p, rs[starts[i]:ends[i], 0].astype(np.uint64)))
        ref = canon(kvec_of_sets(p, want))
        return i, got.shape == ref.shape and np.array_equal(got, ref), len(want)

    with ThreadPoolExecutor(THREADS) as ex:
        for i, ok, n in ex.map(one, chosen):
            assert ok, f"instance {i} (k={preps[i].k}) differs from the oracle ({n} expected)"
            assert int(res.counts[i]) == n


def test_sampled_survivors_verify(run):
    E, S, preps, batch, sw, res, rec = run
    rng = np.random.default_rng(5)
    pick = rng.choice(len(rec), size=20000, replace=False)
    for r in pick:
        x, i = int(rec[r, 0]), int(rec[r, 1])
        p = preps[i]
        assert O.verify(p.n, facet_list(p, x), [int(f) for f in p.facets], p.max_facets), (i, x)


def test_pruned_full_size_counts_and_survivors(run):
    E, S, preps, batch, sw, res, rec = run
    print("[fullsize] building pruned instances", flush=True)
    preps_p = E.prepare_many(W.learned(E.kdim, count=16384), prune=True)
    batch_p = E.DeviceBatch(preps_p)
    assert batch_p.visited < batch.vectors // 2
    sw_p = E.Sweeper(batch_p, cap=1 << 26)
    plan = S.make_plan(batch_p, "dynamic", cbits=12, wg=256)
    sw_p.set_items(plan.items, segments=plan.segments)
    print(f"[fullsize] pruned sweep visits {batch_p.visited:.3e} vectors", flush=True)
    sw_p.launch(plan.mode, wg_size=256)
    res_p = sw_p.result()
    gold = golden_counts()
    bad = np.flatnonzero(res_p.counts != gold)
    assert len(bad) == 0, f"{len(bad)} pruned counts differ from the oracle, first {bad[:8]}"
    rec_p = sw_p.fetch_records().copy()
    rec_p = rec_p[rec_p[:, 1] != -1]
    assert len(rec_p) == res_p.total == int(gold.sum())
    rng = np.random.default_rng(6)
    for r in rng.choice(len(rec_p), size=5000, replace=False):
        x, i = int(rec_p[r, 0]), int(rec_p[r, 1])
        p = preps_p[i]
        assert O.verify(p.n, facet_list(p, x), [int(f) for f in p.facets], p.max_facets), (i, x)
