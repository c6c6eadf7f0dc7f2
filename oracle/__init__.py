"""CPU oracle for the weak-pseudo-manifold enumeration (test infrastructure).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the GPU engine in
``paper_2301_00806_amd``: the arithmetic lives in ``wpm_oracle.c`` (plain C,
built by ``build()`` into ``liboracle.so``) and in ``mlp_ref.py`` (numpy fp64).

Canonical form of a result set (used to compare with the engine): each weak
pseudo-manifold is the ascending tuple of its facet vertex masks; the set is
the ascending list of those tuples.  It does not depend on any facet, ridge or
basis order.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import struct
import subprocess
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wpm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OR_OK, OR_EINVAL, OR_ECAP, OR_ENOMEM = 0, -1, -2, -3


def build(force: bool = True) -> str:
    """Compile wpm_oracle.c with gcc into liboracle.so (in place)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.or_binom.restype = ctypes.c_int64
        L.or_binom.argtypes = [ctypes.c_int, ctypes.c_int]
        L.or_ubt_bound.restype = ctypes.c_int64
        L.or_ubt_bound.argtypes = [ctypes.c_int]
        L.or_candidates.restype = ctypes.c_int
        L.or_candidates.argtypes = [ctypes.c_int, ctypes.c_int, u32p, u32p, ctypes.c_int]
        L.or_ridges.restype = ctypes.c_int
        L.or_ridges.argtypes = [ctypes.c_int, u32p, ctypes.c_int, u32p, ctypes.c_int]
        L.or_incidence_rank.restype = ctypes.c_int
        L.or_incidence_rank.argtypes = [ctypes.c_int, u32p, ctypes.c_int]
        L.or_kernel_dim.restype = ctypes.c_int
        L.or_kernel_dim.argtypes = [ctypes.c_int, u32p, ctypes.c_int]
        L.or_enumerate.restype = ctypes.c_int
        L.or_enumerate.argtypes = [ctypes.c_int, u32p, ctypes.c_int, ctypes.c_int64, u32p,
                                   ctypes.c_int64, i64p, i64p, ctypes.c_int64, i64p]
        L.or_bruteforce.restype = ctypes.c_int
        L.or_bruteforce.argtypes = [ctypes.c_int, u32p, ctypes.c_int, ctypes.c_int64, u32p,
                                    ctypes.c_int64, i64p, i64p]
        L.or_verify.restype = ctypes.c_int
        L.or_verify.argtypes = [ctypes.c_int, u32p, ctypes.c_int, u32p, ctypes.c_int, ctypes.c_int64]
        _lib = L
    return _lib


def _u32(seq: Sequence[int]):
    arr = np.ascontiguousarray(np.asarray(list(seq), dtype=np.uint32))
    return arr, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def ubt_bound(n: int) -> int:
    """Facet count of the cyclic polytope C^n(n+4) (Section 4.2)."""
    return int(lib().or_ubt_bound(n))


def default_max_facets(n: int, m: int) -> int:
    """The paper applies the upper-bound property when m = n + 4 (Picard
    number 4, Algorithm 4.4); otherwise no bound (0)."""
    return ubt_bound(n) if m == n + 4 else 0


def candidates(n: int, m: int, lam: Sequence[int]) -> List[int]:
    arr, p = _u32(lam)
    cap = 1
    for i in range(n):
        cap = cap * (m - i) // (i + 1)
    out, po = _u32([0] * max(cap, 1))
    c = lib().or_candidates(n, m, p, po, cap)
    if c < 0:
        raise ValueError(f"or_candidates status {c}")
    return [int(x) for x in out[:c]]


def ridges(n: int, facets: Sequence[int]) -> List[int]:
    arr, p = _u32(facets)
    cap = max(len(facets) * n, 1)
    out, po = _u32([0] * cap)
    c = lib().or_ridges(n, p, len(facets), po, cap)
    if c < 0:
        raise ValueError(f"or_ridges status {c}")
    return [int(x) for x in out[:c]]


def kernel_dim(n: int, facets: Sequence[int]) -> int:
    """dim ker over F2 of the ridge-facet incidence matrix = M - rank."""
    arr, p = _u32(facets)
    return int(lib().or_kernel_dim(n, p, len(facets)))


def facets_of(inst) -> List[int]:
    """Candidate facets of a wpm_inputs.Instance."""
    if inst.facets is not None:
        return list(inst.facets)
    return candidates(inst.n, inst.m, inst.lam)


def kdim_of(inst) -> int:
    return kernel_dim(inst.n, facets_of(inst))


def _parse(buf: np.ndarray, words: int) -> List[Tuple[int, ...]]:
    res = []
    i = 0
    while i < words:
        ln = int(buf[i])
        res.append(tuple(sorted(int(x) for x in buf[i + 1:i + 1 + ln])))
        i += 1 + ln
    return res


def _run(fn, n: int, facets: Sequence[int], max_facets: int, extra=()):
    arr, p = _u32(facets)
    cap = 1 << 16
    while True:
        out = np.zeros(cap, dtype=np.uint32)
        ln = ctypes.c_int64(0)
        cnt = ctypes.c_int64(0)
        st = fn(n, p, len(facets), max_facets, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                cap, ctypes.byref(ln), ctypes.byref(cnt), *extra)
        if st not in (OR_OK, OR_ECAP):
            raise ValueError(f"oracle status {st}")
        if ln.value <= cap:
            return st, cnt.value, _parse(out, ln.value)
        cap = int(ln.value) + 16


def enumerate_wpm(n: int, facets: Sequence[int], max_facets: int = 0,
                  node_limit: int = 0) -> List[Tuple[int, ...]]:
    """Every weak pseudo-manifold with facets in `facets` (at most max_facets
    facets when max_facets > 0), in canonical order.  Raises TimeoutError
    when node_limit > 0 is exceeded."""
    nodes = ctypes.c_int64(0)
    st, cnt, res = _run(lib().or_enumerate, n, facets, max_facets, (node_limit, ctypes.byref(nodes)))
    if st == OR_ECAP:
        raise TimeoutError(f"oracle search exceeded {node_limit} nodes")
    assert cnt == len(res)
    return sorted(res)


def count_wpm(n: int, facets: Sequence[int], max_facets: int = 0) -> int:
    """Number of weak pseudo-manifolds enumerate_wpm would list (the same
    search, counting only)."""
    arr, p = _u32(facets)
    ln = ctypes.c_int64(0)
    cnt = ctypes.c_int64(0)
    st = lib().or_enumerate(n, p, len(facets), max_facets, None, 0, ctypes.byref(ln),
                            ctypes.byref(cnt), 0, None)
    if st != OR_OK:
        raise ValueError(f"oracle status {st}")
    return int(cnt.value)


def bruteforce_wpm(n: int, facets: Sequence[int], max_facets: int = 0) -> List[Tuple[int, ...]]:
    """Same set as enumerate_wpm, by checking all 2^M subsets (M <= 40)."""
    st, cnt, res = _run(lib().or_bruteforce, n, facets, max_facets)
    assert cnt == len(res)
    return sorted(res)


def verify(n: int, K: Sequence[int], cands: Sequence[int], max_facets: int = 0) -> bool:
    ka, kp = _u32(K)
    ca, cp = _u32(cands)
    r = lib().or_verify(n, kp, len(K), cp, len(cands), max_facets)
    if r < 0:
        raise ValueError(f"or_verify status {r}")
    return bool(r)


def canonical_bytes(wpms: Sequence[Sequence[int]]) -> bytes:
    """Canonical serialisation: sorted list of sorted facet-mask tuples, each
    as a uint32 length followed by the masks (little endian)."""
    parts = []
    for K in sorted(tuple(sorted(k)) for k in wpms):
        parts.append(struct.pack("<I", len(K)))
        parts.append(struct.pack(f"<{len(K)}I", *K))
    return b"".join(parts)


def digest(wpms: Sequence[Sequence[int]]) -> str:
    return hashlib.sha256(canonical_bytes(wpms)).hexdigest()
