"""Parity of the batched workloads at their full sizes, on the GPU through
the C ABI, against counts and sets of the oracle (no self-comparison):

  - batch: 4096 instances, n = 4..7, m = n + 4, 12 <= k <= 32 (the cost
    model's training workload), in the benchmark's launch configuration
    (one persistent launch per launch class, dynamic queue, 2^12-step lane
    chunks, 256-thread workgroups) and again with static round robin and
    2^14-step chunks (lanes cross 4096-step segments);
  - stress: 64 random 0.75-dense subsets of the 7-subsets of [11],
    32 <= k <= 40, with 2^16-step chunks (16 segments per lane chunk).

For each: every per-instance count equals the oracle's stored count
(golden/batch4096_counts.json, golden/stress64_counts.json, written by
golden/make_counts.py from the oracle alone); the result sets of a sample
spread over every kernel dimension equal the oracle's enumeration; and
sampled survivor records pass the oracle's verifier from their facet lists
alone.
"""
import json
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as O
import wpm_inputs as W
import setcheck as SC

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

THREADS = min(16, os.cpu_count() or 1)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def golden(name):
    with open(os.path.join(os.path.dirname(__file__), "golden", f"{name}_counts.json")) as f:
        g = json.load(f)
    return np.array(g["counts"], dtype=np.uint64), g


def sweep_records(E, S, preps, policy, cbits, wg=256, cap=1 << 25):
    batch = E.DeviceBatch(preps)
    sw = E.Sweeper(batch, cap=cap)
    plan = S.make_plan(batch, policy, cbits=cbits, wg=wg)
    _say(f"[configs] {len(preps)} instances, {batch.vectors:.3e} vectors, {policy}, cbits {cbits}, "
         f"{len(plan.items)} items, {len(plan.segments)} launches")
    sw.set_items(plan.items, segments=plan.segments)
    sw.launch(plan.mode, wg_size=wg)
    res = sw.result()
    assert res.slots <= cap
    rec = sw.fetch_records().copy()
    return res, rec


def check_full(preps, res, rec, gold, per_k, seed):
    bad = np.flatnonzero(res.counts != gold)
    assert len(bad) == 0, f"{len(bad)} instance counts differ from the oracle, first {bad[:8]}"
    rs, starts, ends = SC.records_by_instance(rec, len(preps))
    assert len(rs) == res.total == int(gold.sum())
    ks = np.array([p.k for p in preps])
    rng = np.random.default_rng(seed)
    chosen = []
    for k in sorted(set(ks)):
        idx = np.flatnonzero(ks == k)
        chosen += [int(i) for i in rng.choice(idx, size=min(per_k, len(idx)), replace=False)]
    _say(f"[configs] oracle sets of {len(chosen)} instances, k = {sorted(set(ks))}")

    def one(i):
        p = preps[i]
        want = O.enumerate_wpm(p.n, [int(f) for f in p.facets], p.max_facets)
        return i, SC.same_set(p, rs[starts[i]:ends[i], 0], want), len(want)

    with ThreadPoolExecutor(THREADS) as ex:
        for i, ok, n in ex.map(one, chosen):
            assert ok, f"instance {i} (k={preps[i].k}) differs from the oracle ({n} expected)"
            assert int(res.counts[i]) == n
    for r in rng.choice(len(rs), size=min(4000, len(rs)), replace=False):
        x, i = int(rs[r, 0]), int(rs[r, 1])
        p = preps[i]
        assert O.verify(p.n, SC.facet_list(p, x), [int(f) for f in p.facets], p.max_facets), (i, x)


@pytest.fixture(scope="module")
def eng():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_00806_amd import engine as E, scheduler as S
    E.device_query()
    return E, S


@pytest.fixture(scope="module")
def batch_preps(eng):
    E, S = eng
    _say("[configs] preparing the 4096-instance batch workload")
    return E.prepare_many(W.batch(E.kdim, count=4096))


def test_batch_full_size_bench_configuration(eng, batch_preps):
    E, S = eng
    gold, g = golden("batch4096")
    assert [p.k for p in batch_preps] == g["k"]
    res, rec = sweep_records(E, S, batch_preps, "dynamic", 12)
    check_full(batch_preps, res, rec, gold, per_k=2, seed=31)


def test_batch_full_size_static_segments(eng, batch_preps):
    E, S = eng
    gold, _ = golden("batch4096")
    res, rec = sweep_records(E, S, batch_preps, "static", 14)
    check_full(batch_preps, res, rec, gold, per_k=1, seed=32)


def test_stress_full_size(eng):
    E, S = eng
    preps = E.prepare_many(W.stress(E.kdim, count=64))
    gold, g = golden("stress64")
    assert [p.k for p in preps] == g["k"]
    res, rec = sweep_records(E, S, preps, "dynamic", 16)
    check_full(preps, res, rec, gold, per_k=1, seed=33)
