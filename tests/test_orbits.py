"""IDCM orbit generator (Section 4.2) against Table 1 and the oracle's
definition-level enumeration (oracle/idcm.py)."""
import json
import os

import pytest

from oracle import idcm as OI
import oracle as O
from paper_2301_00806_amd import engine as E


def _table1():
    with open(os.path.join(os.path.dirname(__file__), "golden", "table1.json")) as f:
        return json.load(f)


def test_orbit_counts_match_table1():
    t = _table1()
    for n, want in zip(t["n"], t["idcm_orbits"]):
        assert len(E.idcm_orbits(n)) == want, n


@pytest.mark.parametrize("n", list(range(2, 12)))
def test_representatives_match_oracle(n):
    got = E.idcm_orbits(n)
    want = [OI.lambda_of(rows) for rows in OI.orbit_representatives(n)]
    assert got == want
    for lam in got:
        assert lam[:n] == [1 << i for i in range(n)]     # [I_n | M]


@pytest.mark.parametrize("n", list(range(2, 12)))
def test_max_kernel_dimension_over_orbits_matches_table1(n):
    t = _table1()
    ks = []
    for lam in E.idcm_orbits(n):
        F = E.candidates(n, n + 4, lam)
        ks.append(E.kernel_basis(n, n + 4, F)[2])
    assert max(ks) == t["max_dim_ker_idcm"][t["n"].index(n)]
    # and the oracle's own candidates and rank agree on every representative
    for lam, k in zip(E.idcm_orbits(n)[:6], ks[:6]):
        assert O.kernel_dim(n, O.candidates(n, n + 4, lam)) == k


def test_orbits_reject_bad_input():
    import ctypes
    from paper_2301_00806_amd import _lib as L
    c = ctypes.c_int64()
    assert L.lib().wpm_idcm_orbits(3, 7, None, 0, ctypes.byref(c)) == L.WPM_EINVAL
    assert L.lib().wpm_idcm_orbits(0, 4, None, 0, ctypes.byref(c)) == L.WPM_EINVAL
    assert L.lib().wpm_idcm_orbits(12, 4, None, 0, ctypes.byref(c)) == L.WPM_OK and c.value == 0
