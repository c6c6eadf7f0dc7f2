"""Seeded synthetic inputs for the weak-pseudo-manifold sweep.

This module holds random number generation and the recipes of the synthetic
workloads only: it draws characteristic matrices (one column per vertex, bit t
of a column = coordinate t over F2) and random facet subsets. It contains none
of the method's arithmetic. Where a recipe redraws an instance until its kernel
dimension lies in a range, the caller passes the function that computes that
dimension, so the CPU oracle and the GPU engine each select instances with
their own code and the two selections can be compared.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), one stream per instance, seeded base + i.
A uniform vector of F2^n is the low n bits of one draw; a Bernoulli(p) draw is
(next >> 11) * 2^-53 < p. A redraw continues the same stream.

Workloads (stand-ins for the characteristic maps of Picard number 4 that the
paper feeds to its enumeration, Section 4.2, Table 1; the orbit
representatives themselves are not printed, so seeded draws of the same
shapes are used):
  fano    n=3, m=7, lambda = all seven nonzero vectors of F2^3
  single  n=6, m=10, lambda = [e1..e6 | 4 uniform columns], 24 <= k <= 34
  batch   4096 instances, n = 4 + (i mod 4), m = n + 4, 12 <= k <= 32
  learned 16384 instances, n = 5 + (i mod 4), m = n + 4, k <= 36
  stress  random subsets of the 7-subsets of [11]; density 0.6 (literal) and
          0.75 with 32 <= k <= 40 (the density that reaches that k range)
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

MASK64 = (1 << 64) - 1

SEED_SINGLE = 0x2301_0806_0002
SEED_BATCH = 0x2301_0806_0003_0000
SEED_LEARNED = 0x2301_0806_0004_0000
SEED_STRESS = 0x2301_0806_0005_0000
SEED_STRESS_LITERAL = 0x2301_0806_0006_0000


class SplitMix64:
    """SplitMix64 stream (published constants; 64-bit state, 64-bit output)."""

    __slots__ = ("state",)

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform_f2(self, n: int) -> int:
        return self.next() & ((1 << n) - 1)

    def bernoulli(self, p: float) -> bool:
        return (self.next() >> 11) * (2.0 ** -53) < p


@dataclass
class Instance:
    """One input of the enumeration: either a characteristic matrix
    (``lam``: m columns as n-bit integers) or an explicit facet list
    (``facets``: vertex masks)."""
    n: int
    m: int
    lam: Optional[List[int]] = None
    facets: Optional[List[int]] = None
    seed: int = 0
    draws: int = 1
    tag: str = ""
    meta: dict = field(default_factory=dict)


# The kernel-dimension callback: (instance) -> k.  Supplied by the caller.
KFn = Callable[[Instance], int]


def identity_columns(n: int) -> List[int]:
    return [1 << t for t in range(n)]


def fano() -> Instance:
    """n=3, m=7: lambda(i) = i + 1, i.e. every nonzero vector of F2^3."""
    return Instance(n=3, m=7, lam=[i + 1 for i in range(7)], tag="fano")


def draw_picard4(rng: SplitMix64, n: int) -> List[int]:
    """lambda = [I_n | 4 uniform columns of F2^n] (m = n + 4)."""
    return identity_columns(n) + [rng.uniform_f2(n) for _ in range(4)]


def _redraw(seed: int, n: int, kfn: Optional[KFn], lo: int, hi: int,
            tag: str, max_draws: int = 100000) -> Instance:
    rng = SplitMix64(seed)
    for d in range(1, max_draws + 1):
        inst = Instance(n=n, m=n + 4, lam=draw_picard4(rng, n), seed=seed,
                        draws=d, tag=tag)
        if kfn is None:
            return inst
        k = kfn(inst)
        if lo <= k <= hi:
            inst.meta["k"] = k
            return inst
    raise RuntimeError(f"no accepted draw for seed {seed:#x} after {max_draws}")


def single(kfn: Optional[KFn], seed: int = SEED_SINGLE) -> Instance:
    """n=6, m=10, redrawn until 24 <= k <= 34."""
    return _redraw(seed, 6, kfn, 24, 34, "single")


def batch(kfn: Optional[KFn], count: int = 4096, seed: int = SEED_BATCH,
          start: int = 0) -> List[Instance]:
    """count instances; n_i = 4 + (i mod 4); redrawn until 12 <= k <= 32."""
    return [_redraw(seed + i, 4 + (i % 4), kfn, 12, 32, "batch")
            for i in range(start, start + count)]


def learned(kfn: Optional[KFn], count: int = 16384, seed: int = SEED_LEARNED,
            start: int = 0) -> List[Instance]:
    """count instances; n_i = 5 + (i mod 4); redrawn until k <= 36."""
    return [_redraw(seed + i, 5 + (i % 4), kfn, 0, 36, "learned")
            for i in range(start, start + count)]


def all_subsets_lex(m: int, n: int) -> List[int]:
    """Vertex masks of the n-subsets of {0..m-1}, lexicographic order of the
    sorted tuples (used to lay out random facet subsets)."""
    out: List[int] = []
    idx = list(range(n))
    while True:
        out.append(sum(1 << v for v in idx))
        i = n - 1
        while i >= 0 and idx[i] == m - n + i:
            i -= 1
        if i < 0:
            return out
        idx[i] += 1
        for j in range(i + 1, n):
            idx[j] = idx[j - 1] + 1


def draw_facet_subset(rng: SplitMix64, universe: Sequence[int], p: float) -> List[int]:
    return [f for f in universe if rng.bernoulli(p)]


def stress(kfn: Optional[KFn], count: int = 64, density: float = 0.75,
           lo: int = 32, hi: int = 40, seed: int = SEED_STRESS,
           start: int = 0) -> List[Instance]:
    """Random subsets of the 330 7-subsets of [11], redrawn until lo <= k <= hi."""
    universe = all_subsets_lex(11, 7)
    out = []
    for i in range(start, start + count):
        rng = SplitMix64(seed + i)
        for d in range(1, 100001):
            inst = Instance(n=7, m=11, facets=draw_facet_subset(rng, universe, density),
                            seed=seed + i, draws=d, tag="stress")
            if kfn is None:
                break
            k = kfn(inst)
            if lo <= k <= hi:
                inst.meta["k"] = k
                break
        else:
            raise RuntimeError("no accepted stress draw")
        out.append(inst)
    return out


def stress_literal(count: int = 8, seed: int = SEED_STRESS_LITERAL) -> List[Instance]:
    """Density 0.6, no redraw (kernel dimensions come out small)."""
    universe = all_subsets_lex(11, 7)
    return [Instance(n=7, m=11, facets=draw_facet_subset(SplitMix64(seed + i), universe, 0.6),
                     seed=seed + i, tag="stress-0.6") for i in range(count)]
