"""Facet conditions and affine properties on the host (Section 2.1's problem
statement with its collection of properties; Section 4.3's forced facets).

The reference is the oracle's plain enumeration post-filtered by the same
conditions: forced-in facets contained, forced-out facets avoided, every
property c0 + sum_c w_c |K & S_c| > 0.  The packed table (offset row and
property section) is interpreted on the CPU by tests/tablesim.py.
"""
import ctypes
import itertools

import numpy as np
import pytest

import oracle as O
import wpm_inputs as W
from paper_2301_00806_amd import _lib as L
from paper_2301_00806_amd import engine as E
import tablesim as TS


def oracle_filtered(n, F, max_facets, I=(), J=(), props=()):
    out = []
    for K in O.enumerate_wpm(n, [int(f) for f in F], max_facets):
        S = set(K)
        if not set(I) <= S or set(J) & S:
            continue
        if any(c0 + sum(w * len(S & set(fs)) for w, fs in cls) <= 0 for c0, cls in props):
            continue
        out.append(K)
    return out


def span_sets(basis, facets, offset=None):
    """Every complex K* + sum y_t basis_t, as facet tuples (k small)."""
    k = basis.shape[0]
    return [TS.facets_of_x(basis, facets, y, offset) for y in range(1 << k)]


def _cases():
    out = [("fano", 3, 7, W.fano().lam), ("octa", 2, 6, [1, 2, 1, 2, 3, 3])]
    for i, inst in enumerate(W.batch(O.kdim_of, count=12)):
        if inst.meta["k"] <= 13:
            out.append((f"batch{i}", inst.n, inst.m, inst.lam))
    return out[:5]


def _conditions_for(n, F, mf, seed):
    """Forced facets and properties built from the instance's own results so
    that they cut the result set without emptying it."""
    rng = np.random.default_rng(seed)
    res = O.enumerate_wpm(n, [int(f) for f in F], mf)
    K1 = res[int(rng.integers(len(res)))]
    I = list(K1[:2])
    others = [int(f) for f in F if int(f) not in K1]
    J = [others[int(i)] for i in rng.choice(len(others), size=min(3, len(others)), replace=False)]
    v0 = [int(f) for f in F if int(f) & 1]           # facets containing vertex 0
    v1 = [int(f) for f in F if int(f) & 2]           # facets containing vertex 1
    props = [(len(K1), [(-1, v0)]),                    # fewer facets at vertex 0 than |K1|
             (0, [(1, v1), (2, v0)])]                  # vertex 0 or 1 is used
    return I, J, props


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_coset_is_the_conditioned_part_of_the_span(case):
    _, n, m, lam = case
    F = E.candidates(n, m, lam)
    _, B, k = E.kernel_basis(n, m, F)
    I, J, _ = _conditions_for(n, F, 0, 1)
    B2, k2, off, feas = E.facet_conditions(n, m, F, B, k, I, J)
    want = sorted(K for K in span_sets(B, F) if set(I) <= set(K) and not set(J) & set(K))
    assert feas and want
    got = span_sets(B2, F, off)
    assert len(set(got)) == len(got) == 1 << k2        # the coset basis is independent
    assert sorted(got) == want
    # only forced-out facets: a subspace (offset zero)
    B3, k3, off3, _ = E.facet_conditions(n, m, F, B, k, (), J)
    assert not off3.any()
    assert sorted(span_sets(B3, F)) == sorted(K for K in span_sets(B, F) if not set(J) & set(K))


def test_infeasible_and_single_complex_cosets():
    n, m, lam = 3, 7, W.fano().lam
    F = E.candidates(n, m, lam)
    _, B, k = E.kernel_basis(n, m, F)
    allK = span_sets(B, F)
    # all facets forced in: feasible iff the full set lies in the span
    _, k2, _, feas = E.facet_conditions(n, m, F, B, k, [int(f) for f in F], ())
    assert feas == (tuple(sorted(int(f) for f in F)) in set(allK))
    # a WPM with everything else forced out: exactly that complex (k' = 0)
    K1 = O.enumerate_wpm(n, [int(f) for f in F], 0)[5]
    rest = [int(f) for f in F if int(f) not in K1]
    p = E.prepare(n, m, lam=lam, max_facets=0, forced_in=list(K1), forced_out=rest)
    assert p.k == 0 and p.feasible and p.offset is not None
    assert TS.survivors_direct(p.table) == [0]
    assert TS.facets_of_x(p.basis, p.facets, 0, p.offset) == tuple(sorted(K1))
    # K1 plus one more facet, everything else out: K1 + {f} would have to be a
    # kernel vector, so e_f would be one, but a single facet's ridges have degree 1
    f = rest[0]
    q = E.prepare(n, m, lam=lam, max_facets=0, forced_in=list(K1) + [f], forced_out=rest[1:])
    assert not q.feasible and q.k == 0 and q.offset is None
    assert not any(set(K1) | {f} == set(K) for K in allK)
    assert TS.survivors_direct(q.table) == []


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_packed_conditions_match_oracle(case):
    name, n, m, lam = case
    F = E.candidates(n, m, lam)
    mf = E.default_max_facets(n, m)
    for seed in (1, 2):
        I, J, props = _conditions_for(n, F, mf, seed)
        for use_I, use_props in ((True, False), (False, True), (True, True)):
            kw = dict(forced_in=I if use_I else None, forced_out=J,
                      properties=props if use_props else None)
            p = E.prepare(n, m, lam=lam, **kw)
            want = oracle_filtered(n, F, mf, I if use_I else (), J, props if use_props else ())
            got_x = TS.survivors_direct(p.table)
            got = sorted(TS.facets_of_x(p.basis, p.facets, x, p.offset) for x in got_x)
            assert got == want, (name, seed, use_I, use_props)


def test_conditions_reject_bad_input():
    lib = L.lib()
    n, m, lam = 3, 7, W.fano().lam
    F = E.candidates(n, m, lam)
    _, B, k = E.kernel_basis(n, m, F)
    with pytest.raises(L.WpmError):           # a facet on both sides
        E.facet_conditions(n, m, F, B, k, [int(F[0])], [int(F[0])])
    Wd = (len(F) + 31) // 32
    bad = np.zeros(Wd, np.uint32)
    bad[-1] = np.uint32(1 << 31)              # bit 31 of word 0: facet 31 >= M = 28
    Bf = np.ascontiguousarray(B.reshape(-1))
    out = np.zeros_like(Bf)
    off = np.zeros(Wd, np.uint32)
    ko, fe = ctypes.c_int32(), ctypes.c_int32()
    assert lib.wpm_facet_conditions(n, m, E._ptr(F), len(F), E._ptr(Bf), k, E._ptr(bad), None,
                                    E._ptr(out), ctypes.byref(ko), E._ptr(off),
                                    ctypes.byref(fe)) == L.WPM_EINVAL
    with pytest.raises(ValueError):           # pruning needs a linear span
        E.prepare(n, m, lam=lam, forced_in=[int(F[0])], prune=True, min_free=0)
    with pytest.raises(L.WpmError):           # more properties than the table holds
        E.prepare(n, m, lam=lam, properties=[(1, [])] * (L.MAX_PROPS + 1))
