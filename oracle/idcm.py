"""Oracle for the IDCM orbit generator (test infrastructure: only tests may
use it; it shares no code with the engine).

Section 4.2: Lambda(n, p) is the set of (n+p) x p matrices [M; I_p] over F2
with no repeated rows, and S_n x S_p acts by permuting the rows of M and the
columns of the whole matrix; an IDCM orbit is one class.  A dual
characteristic map sends every vertex to a nonzero vector, so the n rows of M
are distinct vectors of F2^p that are neither 0 nor a row of I_p (weight at
least 2).  Permuting rows only reorders the set of rows, so an orbit is an
n-subset of those vectors up to permutations of the p coordinates.  This
module writes that definition out directly: every subset, every coordinate
permutation, the least image as the canonical form.
"""
from __future__ import annotations

import itertools
from typing import List, Tuple


def weight2_vectors(p: int) -> List[int]:
    return [v for v in range(1 << p) if bin(v).count("1") >= 2]


def permute_bits(v: int, perm) -> int:
    """Coordinate i of v moves to coordinate perm[i]."""
    return sum(((v >> i) & 1) << perm[i] for i in range(len(perm)))


def canonical(rows, p: int) -> Tuple[int, ...]:
    """Least sorted row set over all coordinate permutations."""
    return min(tuple(sorted(permute_bits(v, t) for v in rows))
               for t in itertools.permutations(range(p)))


def orbit_representatives(n: int, p: int = 4) -> List[Tuple[int, ...]]:
    """One row set M per IDCM orbit of Lambda(n, p): the least element of the
    orbit, listed in increasing order."""
    reps = set()
    for S in itertools.combinations(weight2_vectors(p), n):
        reps.add(canonical(S, p))
    return sorted(reps)


def lambda_of(rows, p: int = 4) -> List[int]:
    """Characteristic matrix [I_n | M] as columns (bit t = row t): the dual
    of [M; I_p] (Section 3.1)."""
    n = len(rows)
    cols = [1 << i for i in range(n)]
    for c in range(p):
        cols.append(sum(((rows[i] >> c) & 1) << i for i in range(n)))
    return cols
