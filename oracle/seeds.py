"""Oracle for the filters after the sweep (test infrastructure: only tests
may use it; it shares no code with the engine).  Plain Python definitions:

  - Picard number of K: its number of vertices minus n (Section 3);
  - minimal non-faces: the subsets of [m] that are not faces but whose
    proper subsets all are;
  - seedness condition (Section 3, seedness from minimal non-faces): no edge
    {v, w} of K such that every minimal non-face contains both or neither;
  - isomorphism (Section 3): colour every vertex by the increasing sizes of
    the minimal non-faces containing it; the canonical form is the least
    sorted image of the minimal non-faces over all relabellings that order
    the colour classes by colour, tried exhaustively.
"""
from __future__ import annotations

import itertools
from typing import List, Sequence, Tuple


def faces(K: Sequence[int]) -> set:
    out = set()
    for f in K:
        verts = [v for v in range(32) if (f >> v) & 1]
        for r in range(len(verts) + 1):
            for c in itertools.combinations(verts, r):
                out.add(sum(1 << v for v in c))
    return out


def minimal_nonfaces(K: Sequence[int], m: int) -> List[int]:
    F = faces(K)
    out = []
    for s in range(1, 1 << m):
        if s in F:
            continue
        if all((s & ~(1 << v)) in F for v in range(m) if (s >> v) & 1):
            out.append(s)
    return out


def picard(K: Sequence[int], n: int) -> int:
    used = 0
    for f in K:
        used |= f
    return bin(used).count("1") - n


def is_seed(K: Sequence[int], m: int) -> bool:
    M = minimal_nonfaces(K, m)
    for f in K:
        verts = [v for v in range(m) if (f >> v) & 1]
        for a, b in itertools.combinations(verts, 2):
            e = (1 << a) | (1 << b)
            if all((s & e) in (0, e) for s in M):
                return False
    return True


def canonical_form(K: Sequence[int], m: int) -> Tuple:
    M = minimal_nonfaces(K, m)
    col = [tuple(sorted(bin(s).count("1") for s in M if (s >> v) & 1)) for v in range(m)]
    order = sorted(range(m), key=lambda v: col[v])
    groups = [list(g) for _, g in itertools.groupby(order, key=lambda v: col[v])]
    slots, pos = [], 0
    for g in groups:
        slots.append(list(range(pos, pos + len(g))))
        pos += len(g)
    best = None
    for choice in itertools.product(*[itertools.permutations(s) for s in slots]):
        img = {}
        for g, ch in zip(groups, choice):
            img.update(zip(g, ch))
        form = tuple(sorted(sum(1 << img[v] for v in range(m) if (s >> v) & 1) for s in M))
        if best is None or form < best:
            best = form
    return tuple(sorted(col)), best
