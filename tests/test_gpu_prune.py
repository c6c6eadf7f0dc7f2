"""Pruned sweep over a convenient kernel basis (Section 2.1) on the GPU vs the
CPU oracle, through the C ABI: the same result sets as the plain sweep, from
the product of the blocks' allowed sets instead of all 2^k vectors."""
import itertools
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


def oracle_sets(preps):
    return [O.enumerate_wpm(p.n, [int(f) for f in p.facets], p.max_facets) for p in preps]


def run(E, preps, **kw):
    _say(f"[gpu] pruned sweep {len(preps)} instance(s) k={[p.k for p in preps][:8]} "
         f"blocks={[0 if p.blocks is None else int(p.blocks.num_blocks) for p in preps][:8]} {kw}")
    return E.sweep(preps, **kw)


def test_pruned_fano_and_graphs(E):
    preps = [E.prepare(3, 7, lam=W.fano().lam, max_facets=mf, prune=True, min_free=7)
             for mf in (None, 0)]
    for v in (7, 8):   # n = 2: ridges of K_v have v - 1 parents
        F = [(1 << a) | (1 << b) for a, b in itertools.combinations(range(v), 2)]
        preps.append(E.prepare(2, v, facets=F, max_facets=0, prune=True, min_free=7))
    assert all(p.blocks.num_blocks > 0 for p in preps)
    res, sets = run(E, preps, cbits=7, wg_size=64)
    want = oracle_sets(preps)
    assert sets == want
    assert list(res.counts) == [len(w) for w in want]


@pytest.mark.parametrize("min_free,cbits,wg", [(7, 9, 256), (10, 12, 64)])
def test_pruned_batch_matches_oracle(E, min_free, cbits, wg):
    insts = [i for i in W.batch(E.kdim, count=96) if i.meta["k"] <= 22][:48]
    preps = E.prepare_many(insts, prune=True, min_free=min_free)
    assert sum(p.visited for p in preps) < sum(p.vectors for p in preps)
    res, sets = run(E, preps, cbits=cbits, wg_size=wg, order=1,
                    cost=np.arange(1, len(preps) + 1, dtype=np.float32))
    want = oracle_sets(preps)
    for i, (g, w) in enumerate(zip(sets, want)):
        assert g == w, f"instance {i} k={preps[i].k} blocks={preps[i].blocks.num_blocks}"


def test_pruned_single_and_schedules(E):
    inst = W.single(E.kdim)
    p = E.prepare(inst.n, inst.m, lam=inst.lam, prune=True)
    q = E.prepare(inst.n, inst.m, lam=inst.lam)
    assert p.blocks.num_blocks > 0 and p.visited < p.vectors
    want = oracle_sets([p])[0]
    ref = None
    for mode in (0, 1, 2):
        res, sets = run(E, [p], mode=mode, cbits=12)
        assert sets[0] == want
        ref = res.counts if ref is None else ref
        assert np.array_equal(res.counts, ref)
    res_q, _ = run(E, [q], cbits=12, want_sets=False)
    assert np.array_equal(res_q.counts, ref)


def test_pruned_stress_outputs_verified(E):
    insts = W.stress(E.kdim, count=2)
    preps = E.prepare_many(insts, prune=True)
    res, sets = run(E, preps, cbits=12)
    for i, (p, s) in enumerate(zip(preps, sets)):
        F = [int(f) for f in p.facets]
        for K in s:
            assert O.verify(p.n, list(K), F, p.max_facets)
        assert int(res.counts[i]) == len(s)
    plain = E.prepare_many(insts)
    res_q, _ = run(E, plain, cbits=12, want_sets=False)
    assert np.array_equal(res_q.counts, res.counts)


def test_pruned_autotuner_keeps_counts(E):
    # the tuner re-prepares the batch for each min_free and times each chunk
    # size; every shape must give the oracle's counts
    from paper_2301_00806_amd import tune as T
    insts = [i for i in W.batch(E.kdim, count=64) if i.meta["k"] <= 20][:24]
    _say(f"[gpu] pruned autotuner over {len(insts)} instances")
    entry, preps = T.tune_pruned(insts, cache=None, min_frees=(8, 10), cbits=(8, 10))
    assert entry["min_free"] in (8, 10) and entry["cbits"] in (8, 10)
    assert len(entry["results"]) == 4 and not entry["cached"]
    assert any(p.blocks is not None and p.blocks.num_blocks > 0 for p in preps)
    res, sets = run(E, preps, cbits=int(entry["cbits"]), wg_size=256, order=1)
    want = oracle_sets(preps)
    assert sets == want
    assert list(res.counts) == [len(w) for w in want]
