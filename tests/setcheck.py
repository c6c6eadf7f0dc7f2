"""Helpers of the GPU parity tests (host side): survivor records to facet bit
vectors, the oracle's facet lists to the same vectors, and a canonical order
of those vectors, so that result sets are compared in facet space, which does
not depend on the basis, the order of facets or the schedule."""
import numpy as np


def kvec(p, xs):
    """Facet bit vectors K = sum_t x_t K_t (+ K* of a coset; rows of W uint32)
    of kernel vectors x of a prepared instance p."""
    xs = np.asarray(xs, dtype=np.uint64)
    K = np.zeros((len(xs), p.W), dtype=np.uint32)
    if p.offset is not None:
        K[:] = np.asarray(p.offset, dtype=np.uint32)[None, :p.W]
    for t in range(p.k):
        sel = ((xs >> np.uint64(t)) & np.uint64(1)).astype(bool)
        K[sel] ^= p.basis[t]
    return K


def kvec_of_sets(p, sets):
    """The same bit vectors for lists of facet masks (the oracle's output)."""
    pos = {int(f): j for j, f in enumerate(p.facets)}
    K = np.zeros((len(sets), p.W), dtype=np.uint32)
    for r, S in enumerate(sets):
        for f in S:
            j = pos[f]
            K[r, j // 32] |= np.uint32(1 << (j % 32))
    return K


def canon(K):
    return K[np.lexsort(K.T[::-1])] if len(K) else K


def facet_list(p, x):
    K = kvec(p, [x])[0]
    return [int(p.facets[w * 32 + b]) for w in range(p.W) for b in range(32) if (int(K[w]) >> b) & 1]


def records_by_instance(rec, num):
    """Used records (instance != ~0) sorted by instance, with the start and
    end row of every instance."""
    rec = rec[rec[:, 1] != -1]
    rs = rec[np.argsort(rec[:, 1], kind="stable")]
    starts = np.searchsorted(rs[:, 1], np.arange(num))
    ends = np.searchsorted(rs[:, 1], np.arange(num), side="right")
    return rs, starts, ends


def same_set(p, xs, oracle_sets):
    """True iff the records' complexes equal the oracle's list, as sets."""
    got = canon(kvec(p, xs))
    ref = canon(kvec_of_sets(p, oracle_sets))
    return got.shape == ref.shape and bool(np.array_equal(got, ref))
