"""Facet conditions and affine properties on the GPU vs the oracle's plain
enumeration post-filtered by the same conditions (Section 2.1 properties,
Section 4.3 forced facets), through the C ABI."""
import sys

import numpy as np
import pytest

import oracle as O
import wpm_inputs as W
from test_conditions import _conditions_for, oracle_filtered

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def E():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_00806_amd import engine
    engine.device_query()
    return engine


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_conditioned_batch_matches_oracle(E):
    insts = [W.fano()] + [i for i in W.batch(E.kdim, count=64) if i.meta["k"] <= 20][:23]
    preps, wants = [], []
    for j, inst in enumerate(insts):
        F = E.candidates(inst.n, inst.m, inst.lam)
        mf = E.default_max_facets(inst.n, inst.m)
        I, J, props = _conditions_for(inst.n, F, mf, j)
        mode = j % 4      # forced in + out; out only; properties only; everything
        kw = [dict(forced_in=I, forced_out=J), dict(forced_out=J), dict(properties=props),
              dict(forced_in=I, forced_out=J, properties=props)][mode]
        preps.append(E.prepare(inst.n, inst.m, lam=inst.lam, **kw))
        wants.append(oracle_filtered(inst.n, F, mf, kw.get("forced_in") or (),
                                     kw.get("forced_out") or (), kw.get("properties") or ()))
    # plain instances in the same batch keep their own semantics
    plain = [E.prepare(i.n, i.m, lam=i.lam) for i in insts[:4]]
    preps += plain
    wants += [O.enumerate_wpm(p.n, [int(f) for f in p.facets], p.max_facets) for p in plain]
    for cbits, wg, mode in ((7, 64, 2), (9, 256, 1), (12, 256, 0)):
        _say(f"[gpu] conditions: {len(preps)} instances cbits={cbits} wg={wg} mode={mode}")
        res, sets = E.sweep(preps, mode=mode, cbits=cbits, wg_size=wg)
        for i, (g, w) in enumerate(zip(sets, wants)):
            assert g == w, f"instance {i} k={preps[i].k} offset={preps[i].offset is not None}"
        assert list(res.counts) == [len(w) for w in wants]


def test_single_complex_and_infeasible_cosets(E):
    lam = W.fano().lam
    F = E.candidates(3, 7, lam)
    res0 = O.enumerate_wpm(3, [int(f) for f in F], 0)
    K1 = res0[5]
    rest = [int(f) for f in F if int(f) not in K1]
    one = E.prepare(3, 7, lam=lam, max_facets=0, forced_in=list(K1), forced_out=rest)
    none = E.prepare(3, 7, lam=lam, max_facets=0, forced_in=list(K1) + [rest[0]],
                     forced_out=rest[1:])
    assert one.k == 0 and not none.feasible
    _say("[gpu] single-complex and infeasible cosets")
    res, sets = E.sweep([one, none], cbits=7, wg_size=64)
    assert sets == [[tuple(sorted(K1))], []]
    assert list(res.counts) == [1, 0]


def test_conditioned_single_large(E):
    inst = W.single(E.kdim)
    F = E.candidates(inst.n, inst.m, inst.lam)
    mf = E.default_max_facets(inst.n, inst.m)
    I, J, props = _conditions_for(inst.n, F, mf, 7)
    p = E.prepare(inst.n, inst.m, lam=inst.lam, forced_in=I, forced_out=J, properties=props)
    want = oracle_filtered(inst.n, F, mf, I, J, props)
    _say(f"[gpu] conditioned single instance k={p.k} (unconditioned {inst.meta['k']})")
    res, sets = E.sweep([p], cbits=12)
    assert sets[0] == want
