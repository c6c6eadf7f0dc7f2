"""Filters after the sweep (Algorithm 4.4) on the host: the engine's
Picard/seedness flags and isomorphism classes against the oracle's plain
definitions (oracle/seeds.py), and Table 2's third row (isomorphism classes of
seeds of Picard number 4 supporting an IDCM) for n = 2, 3, 4 with the oracle's
enumeration standing in for the GPU sweep."""
import json
import os

import numpy as np
import pytest

import oracle as O
from oracle import seeds as OS
from paper_2301_00806_amd import _lib as L
from paper_2301_00806_amd import engine as E
from paper_2301_00806_amd import seeds as S

TABLE2_CLASSES = {2: 2, 3: 5, 4: 49, 5: 256, 6: 1791, 7: 2194, 8: 1401, 9: 381, 10: 56}


def oracle_enumerator(preps):
    return [O.enumerate_wpm(p.n, [int(f) for f in p.facets], p.max_facets) for p in preps]


def union_of(n):
    m = n + 4
    out = set()
    for lam in E.idcm_orbits(n):
        F = O.candidates(n, m, lam)
        out |= {tuple(sorted(K)) for K in O.enumerate_wpm(n, F, O.default_max_facets(n, m))}
    return sorted(out)


@pytest.mark.parametrize("n", [2, 3])
def test_filters_match_oracle(n):
    m = n + 4
    U = union_of(n)
    flags = S.complex_filters(n, m, U)
    for K, f in zip(U, flags):
        assert bool(f & L.CX_FULL_PICARD) == (OS.picard(K, n) == m - n)
        assert bool(f & L.CX_SEED) == OS.is_seed(K, m)


@pytest.mark.parametrize("n,sample", [(2, None), (3, None), (4, 400)])
def test_iso_classes_match_oracle_partition(n, sample):
    m = n + 4
    U = union_of(n)
    flags = S.complex_filters(n, m, U)
    kept = [K for K, f in zip(U, flags) if f == (L.CX_FULL_PICARD | L.CX_SEED)]
    if sample:
        rng = np.random.default_rng(3)
        kept = [kept[i] for i in sorted(rng.choice(len(kept), size=sample, replace=False))]
    cls, num = S.iso_classes(m, kept)
    forms = [OS.canonical_form(K, m) for K in kept]
    # the same partition: equal class <=> equal canonical form
    pairs = {}
    for c, fm in zip(cls, forms):
        pairs.setdefault(int(c), set()).add(fm)
    assert all(len(v) == 1 for v in pairs.values())
    assert len({fm for fm in forms}) == num


@pytest.mark.parametrize("n", [2, 3, 4])
def test_table2_classes_with_oracle_enumeration(n):
    rep = S.colorable_seeds_pic4(n, enumerate_sets=oracle_enumerator)
    assert rep.orbits == [7, 16, 28][n - 2]
    assert rep.classes == TABLE2_CLASSES[n]


def test_filters_reject_bad_input():
    offs = np.array([0, 1], np.int64)
    fac = np.array([1 << 20], np.uint32)          # vertex 20 >= m
    import ctypes
    flags = np.zeros(1, np.uint8)
    st = L.lib().wpm_complex_filters(2, 6, 1, E._ptr(offs, L.c_i64p), E._ptr(fac),
                                     flags.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    assert st == L.WPM_EINVAL
    assert L.lib().wpm_iso_classes(17, 0, None, None, E._ptr(np.zeros(1, np.int64), L.c_i64p),
                                   E._ptr(np.zeros(1, np.int64), L.c_i64p)) == L.WPM_EINVAL


def test_saved_orbit_results_give_the_same_report(tmp_path):
    n, m = 4, 8
    lams = E.idcm_orbits(n)
    per = [O.enumerate_wpm(n, O.candidates(n, m, lam), O.default_max_facets(n, m)) for lam in lams]
    files = []
    for i, sets in enumerate(per):
        f = str(tmp_path / f"orbit{i}.npz")
        S.save_complexes(f, sets)
        files.append(f)
        assert S.load_complexes(f) == [tuple(K) for K in sets]
    rep = S.filter_report(n, [S.load_complexes(f) for f in files])
    ref = S.colorable_seeds_pic4(n, enumerate_sets=oracle_enumerator)
    assert (rep.union, rep.filtered, rep.classes) == (ref.union, ref.filtered, ref.classes) == \
        (ref.union, ref.filtered, TABLE2_CLASSES[n])
