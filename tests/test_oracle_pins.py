"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (Table 1), textbook closed forms (cycle spaces of graphs,
2-regular subgraph counts, Gale's evenness condition for cyclic polytopes),
invariances (GL(n, F2) action, vertex relabelling) and brute force over all
facet subsets.
"""
import itertools
import json
import math
import os
import random

import pytest

import oracle as O
import wpm_inputs as W

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1.json")


def table1():
    with open(GOLD) as f:
        return json.load(f)


def edges_of(graph_edges):
    return [(1 << a) | (1 << b) for a, b in graph_edges]


# ---------------------------------------------------------------- generator

def test_splitmix64_published_vector():
    # Reference outputs of SplitMix64 seeded 1234567 (Steele-Lea-Flood / Vigna).
    r = W.SplitMix64(1234567)
    assert [r.next() for _ in range(3)] == [6457827717110365317, 3203168211198807973,
                                            9817491932198370423]


def test_all_subsets_lex_order():
    subs = W.all_subsets_lex(5, 3)
    tuples = [tuple(v for v in range(5) if (s >> v) & 1) for s in subs]
    assert tuples == list(itertools.combinations(range(5), 3))


# ---------------------------------------------------------------- UBT bound

def gale_facets(m, n):
    """Facets of the cyclic polytope C(m, n) by Gale's evenness condition."""
    cnt = 0
    for S in itertools.combinations(range(m), n):
        s = set(S)
        out = [v for v in range(m) if v not in s]
        ok = all(sum(1 for x in S if i < x < j) % 2 == 0 for i, j in itertools.combinations(out, 2))
        cnt += ok
    return cnt


@pytest.mark.parametrize("n", range(2, 10))
def test_ubt_bound_matches_cyclic_polytope(n):
    assert O.ubt_bound(n) == gale_facets(n + 4, n)


def test_ubt_bound_closed_forms():
    # n = 2d: m/(m-d) C(m-d, d); n = 2d+1: 2 C(m-d-1, d), m = n + 4.
    for n in range(2, 12):
        m, d = n + 4, n // 2
        want = (m * math.comb(m - d, d)) // (m - d) if n % 2 == 0 else 2 * math.comb(m - d - 1, d)
        assert O.ubt_bound(n) == want


# ---------------------------------------------------------------- candidates

def rank_f2(cols):
    basis = []
    for v in cols:
        for b in basis:
            v = min(v, v ^ b)
        if v:
            basis.append(v)
    return len(basis)


def test_candidates_definition_small():
    rng = random.Random(5)
    for _ in range(40):
        n = rng.randint(2, 5)
        m = n + rng.randint(1, 5)
        lam = [rng.randrange(1 << n) for _ in range(m)]
        got = O.candidates(n, m, lam)
        want = [sum(1 << v for v in S) for S in itertools.combinations(range(m), n)
                if rank_f2([lam[v] for v in S]) == n]
        assert got == want


def test_fano_shape():
    F = O.candidates(3, 7, W.fano().lam)
    assert len(F) == 28
    lines = [sum(1 << v for v in S) for S in itertools.combinations(range(7), 3)
             if ((S[0] + 1) ^ (S[1] + 1) ^ (S[2] + 1)) == 0]
    assert len(lines) == 7 and not set(lines) & set(F)
    R = O.ridges(3, F)
    assert len(R) == 21
    for r in R:
        assert sum(1 for f in F if f & r == r) == 4
    assert O.kernel_dim(3, F) == 13


# ---------------------------------------------------------------- Table 1

@pytest.mark.parametrize("n", range(2, 12))
def test_table1_full_kernel_dim(n):
    t = table1()
    full = W.all_subsets_lex(n + 4, n)
    k = O.kernel_dim(n, full)
    assert k == t["dim_ker_full"][t["n"].index(n)]
    assert k == math.comb(n + 3, n)


def idcm_lambdas(n):
    """lambda = [I_n | M] whose dual [M; I_4] has distinct rows of weight >= 2."""
    rows = [v for v in range(16) if bin(v).count("1") >= 2]
    for R in itertools.combinations(rows, n):
        cols = [sum(((R[i] >> t) & 1) << i for i in range(n)) for t in range(4)]
        yield W.identity_columns(n) + cols


@pytest.mark.parametrize("n", range(2, 12))
def test_table1_max_kernel_dim_over_idcm(n):
    # every printed value of the row, n = 2..11 (C(11, n) row sets each)
    t = table1()
    best = max(O.kernel_dim(n, O.candidates(n, n + 4, lam)) for lam in idcm_lambdas(n))
    assert best == t["max_dim_ker_idcm"][t["n"].index(n)]


# ---------------------------------------------------------------- graphs (n = 2)

def two_regular_count(j):
    """Labelled 2-regular graphs on j vertices (partitions into cycles of
    length >= 3, a cycle of length L in (L-1)!/2 ways)."""
    @__import__("functools").lru_cache(None)
    def a(j):
        if j == 0:
            return 1
        # the cycle through the smallest vertex has length L
        return sum(math.comb(j - 1, L - 1) * (math.factorial(L - 1) // 2) * a(j - L)
                   for L in range(3, j + 1))
    return a(j)


@pytest.mark.parametrize("v", range(3, 8))
def test_complete_graph_cycle_space_and_unions_of_cycles(v):
    E = edges_of(itertools.combinations(range(v), 2))
    assert O.kernel_dim(2, E) == len(E) - v + 1
    want = sum(math.comb(v, j) * two_regular_count(j) for j in range(3, v + 1))
    got = O.enumerate_wpm(2, E, 0)
    assert len(got) == want
    if len(E) <= 21:
        assert got == O.bruteforce_wpm(2, E, 0)


def test_k4_counts():
    E = edges_of(itertools.combinations(range(4), 2))
    got = O.enumerate_wpm(2, E, 0)
    assert sorted(len(k) for k in got) == [3, 3, 3, 3, 4, 4, 4]


def test_octahedron_graph_lambda():
    # n = 2, m = 6, lambda = [e1, e2, e1, e2, e1+e2, e1+e2]: F(lambda) is K_{2,2,2}.
    lam = [1, 2, 1, 2, 3, 3]
    F = O.candidates(2, 6, lam)
    assert len(F) == 12
    assert O.kernel_dim(2, F) == 12 - 6 + 1 == table1()["max_dim_ker_idcm"][0]
    for mf in (0, O.ubt_bound(2)):
        assert O.enumerate_wpm(2, F, mf) == O.bruteforce_wpm(2, F, mf)


def test_disconnected_graph_kernel_dim():
    # two disjoint triangles and a path: |E| - |V| + c = 7 - 8 + 3 = 2
    E = edges_of([(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5), (6, 7)])
    assert O.kernel_dim(2, E) == 2
    assert len(O.enumerate_wpm(2, E, 0)) == 3


# ---------------------------------------------------------------- Fano (n = 3)

def test_fano_bruteforce_equals_backtracking():
    F = O.candidates(3, 7, W.fano().lam)
    for mf in (0, O.ubt_bound(3)):
        assert O.enumerate_wpm(3, F, mf) == O.bruteforce_wpm(3, F, mf)


def test_fano_tetrahedra():
    F = O.candidates(3, 7, W.fano().lam)
    got = [k for k in O.enumerate_wpm(3, F, 0) if len(k) == 4]
    lines = [set(S) for S in itertools.combinations(range(7), 3)
             if ((S[0] + 1) ^ (S[1] + 1) ^ (S[2] + 1)) == 0]
    want = []
    for L in lines:
        Q = [v for v in range(7) if v not in L]
        want.append(tuple(sorted(sum(1 << v for v in T) for T in itertools.combinations(Q, 3))))
    assert sorted(got) == sorted(want)


# ---------------------------------------------------------------- full sets

def test_full_set_contains_simplex_boundaries():
    n, m = 3, 6
    full = W.all_subsets_lex(m, n)
    got = set(O.enumerate_wpm(n, full, 0))
    for S in itertools.combinations(range(m), n + 1):
        bd = tuple(sorted(sum(1 << v for v in T) for T in itertools.combinations(S, n)))
        assert bd in got
    assert sorted(got) == O.bruteforce_wpm(n, full, 0)


# ---------------------------------------------------------------- invariances

def relabel(mask, perm):
    return sum(1 << perm[v] for v in range(32) if (mask >> v) & 1)


def test_gl_action_invariance():
    rng = random.Random(7)
    n, m = 4, 8
    base = W.draw_picard4(W.SplitMix64(99), n)
    F = O.candidates(n, m, base)
    ref = O.enumerate_wpm(n, F, O.ubt_bound(n))
    for _ in range(3):
        while True:
            G = [rng.randrange(1, 1 << n) for _ in range(n)]
            if rank_f2(G) == n:
                break
        lam2 = [0] * m
        for i, c in enumerate(base):
            v = 0
            for t in range(n):
                if (c >> t) & 1:
                    v ^= G[t]
            lam2[i] = v
        assert O.candidates(n, m, lam2) == F
        assert O.enumerate_wpm(n, O.candidates(n, m, lam2), O.ubt_bound(n)) == ref


def test_relabel_invariance():
    rng = random.Random(11)
    n, m = 3, 7
    lam = W.fano().lam
    ref = O.enumerate_wpm(n, O.candidates(n, m, lam), 0)
    perm = list(range(m))
    rng.shuffle(perm)
    inv = [0] * m
    for v, p in enumerate(perm):
        inv[p] = v
    lam2 = [lam[inv[v]] for v in range(m)]
    got = O.enumerate_wpm(n, O.candidates(n, m, lam2), 0)
    mapped = sorted(tuple(sorted(relabel(f, perm) for f in K)) for K in ref)
    assert got == mapped


# ---------------------------------------------------------------- verifier

def test_verifier_accepts_outputs_rejects_breaks():
    F = O.candidates(3, 7, W.fano().lam)
    res = O.enumerate_wpm(3, F, O.ubt_bound(3))
    for K in res:
        assert O.verify(3, K, F, O.ubt_bound(3))
    K = list(res[0])
    assert not O.verify(3, K[:-1], F, 0)          # dropped facet leaves open ridges
    assert not O.verify(3, [], F, 0)              # empty complex
    assert not O.verify(3, K + [K[0]], F, 0)      # duplicate facet
    big = max(res, key=len)
    assert not O.verify(3, list(big), F, len(big) - 1)  # bound
    line = 0b111  # {0,1,2}: 1^2^3 = 0, a Fano line, not a candidate
    assert not O.verify(3, [line], F, 0)


def test_random_small_sets_bruteforce():
    rng = random.Random(3)
    for trial in range(12):
        n = rng.choice([2, 3, 4])
        m = n + rng.randint(2, 4)
        allf = W.all_subsets_lex(m, n)
        F = sorted(rng.sample(allf, min(len(allf), rng.randint(6, 22))))
        mf = rng.choice([0, 6, 10])
        assert O.enumerate_wpm(n, F, mf) == O.bruteforce_wpm(n, F, mf)
