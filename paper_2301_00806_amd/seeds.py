"""Algorithm 4.4 up to its isomorphism step, on the engine.

For Picard number 4 and dimension n - 1 (m = n + 4):
  1. one characteristic matrix per IDCM orbit (wpm_idcm_orbits);
  2. for each, every weak pseudo-manifold with facets in F(lambda) and at
     most f(n) facets (the GPU sweep; the upper-bound property of Section
     4.2) -- the union is the set K(n, 4), Table 2's first row;
  3. discard complexes with Pic(K) < 4 or failing the seedness condition
     (wpm_complex_filters) -- Table 2's second row;
  4. one representative per isomorphism class (wpm_iso_classes) -- Table 2's
     third row.
The PL-sphere test of the algorithm's last step is not part of this engine.
The first two rows count labelled complexes, so they depend on which
representative each orbit gets; the isomorphism classes do not.
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

from . import _lib as L
from . import engine as E

Complex = Tuple[int, ...]


def _pack(complexes: Sequence[Sequence[int]]):
    offs = np.zeros(len(complexes) + 1, dtype=np.int64)
    if complexes:
        offs[1:] = np.cumsum([len(K) for K in complexes])
    fac = np.zeros(max(1, int(offs[-1])), dtype=np.uint32)
    pos = 0
    for K in complexes:
        fac[pos:pos + len(K)] = K
        pos += len(K)
    return offs, fac


def complex_filters(n: int, m: int, complexes: Sequence[Sequence[int]]) -> np.ndarray:
    """Flags per complex: CX_FULL_PICARD, CX_SEED (wpm_complex_filters)."""
    offs, fac = _pack(complexes)
    flags = np.zeros(max(1, len(complexes)), dtype=np.uint8)
    L.check("wpm_complex_filters", L.lib().wpm_complex_filters(
        n, m, len(complexes), E._ptr(offs, L.c_i64p), E._ptr(fac),
        flags.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
    return flags[:len(complexes)]


def iso_classes(m: int, complexes: Sequence[Sequence[int]]):
    """(class of each complex, number of classes) (wpm_iso_classes)."""
    offs, fac = _pack(complexes)
    cls = np.zeros(max(1, len(complexes)), dtype=np.int64)
    num = ctypes.c_int64(0)
    L.check("wpm_iso_classes", L.lib().wpm_iso_classes(
        m, len(complexes), E._ptr(offs, L.c_i64p), E._ptr(fac), E._ptr(cls, L.c_i64p),
        ctypes.byref(num)))
    return cls[:len(complexes)], int(num.value)


@dataclass
class SeedReport:
    n: int
    orbits: int
    max_k: int
    union: int                 # |K(n,4)|: union of the sweeps' outputs
    filtered: int              # after the Picard-number and seedness filters
    classes: int               # isomorphism classes
    representatives: List[Complex] = field(default_factory=list)
    seconds: dict = field(default_factory=dict)


def sliced_sweep(p, cbits: int = 12, wg: int = 256, cap: int = 1 << 24,
                 max_items: int = 1 << 22, log: Optional[Callable[[str], None]] = None):
    """Sweep one (pruned) instance in slices of at most about max_items items:
    each slice fixes the choices of the highest blocks, so its queue is the
    product of the remaining blocks' choices (the table is the same for every
    slice).  Each slice's results are collected before the next launch, so
    the record buffer only ever holds one slice.  Returns the result list of
    the instance."""
    import itertools
    batch = E.DeviceBatch([p])
    sw = E.Sweeper(batch, cap=cap)
    cls = int(batch.cls[0])
    blk = p.blocks
    nb = 0 if blk is None else int(blk.num_blocks)
    # fix the top blocks until the rest yields at most max_items items
    per_tuple = 1
    if blk is not None and nb:
        c = min(cbits, max(7, int(blk.free_dims) - 8))
        per_tuple = max(1, (1 << (int(blk.free_dims) - c)) // wg)
    fixed = 0
    rest = 1 if blk is None else int(np.prod([int(blk.count[b]) for b in range(nb)], dtype=np.float64))
    while fixed < nb and rest * per_tuple > max_items:
        rest //= int(blk.count[nb - 1 - fixed])
        fixed += 1
    top = list(range(nb - fixed, nb))
    combos = list(itertools.product(*[range(int(blk.count[b])) for b in top])) if fixed else [()]
    t0 = time.perf_counter()
    results = []
    for si, digits in enumerate(combos):
        if blk is not None:
            part = L.Blocks()
            ctypes.pointer(part)[0] = blk
            for b, d in zip(top, digits):
                part.choice[b][0] = blk.choice[b][d]
                part.count[b] = 1
            items = E.build_queue(np.array([p.k], np.int32), cbits, wg, blocks=(L.Blocks * 1)(part))
        else:
            items = E.build_queue(np.array([p.k], np.int32), cbits, wg)
        sw.set_items(items, segments=[E.Segment(cls, 0, len(items))])
        sw.launch(L.SCHED_DYNAMIC, wg_size=wg)
        results.extend(sw.collect()[0])   # raises on a record-buffer overflow
        if log and (si % max(1, len(combos) // 20) == 0 or si == len(combos) - 1):
            log(f"slice {si + 1}/{len(combos)} ({len(items)} items), {len(results)} complexes, "
                f"{time.perf_counter() - t0:.1f}s")
    return sorted(results)


def gpu_enumerator(cbits: int = 12, wg: int = 256, prune: bool = False, cap: int = 1 << 24,
                   per_instance: bool = False, log: Optional[Callable[[str], None]] = None,
                   sliced: bool = False):
    """Enumerator over a list of prepared orbit instances on the GPU sweep:
    one batched sweep, or one sweep per instance (with a log line each)."""
    def run(preps):
        if not per_instance:
            _, sets = E.sweep(preps, cbits=cbits, wg_size=wg, cap=cap)
            return sets
        out = []
        for i, p in enumerate(preps):
            t0 = time.perf_counter()
            if sliced:
                out.append(sliced_sweep(p, cbits=cbits, wg=wg, cap=cap, log=log))
            else:
                _, sets = E.sweep([p], cbits=cbits, wg_size=wg, cap=cap)
                out.append(sets[0])
            if log:
                log(f"orbit {i + 1}/{len(preps)}: k={p.k}, {p.visited:.3e} vectors, "
                    f"{len(out[-1])} complexes, {time.perf_counter() - t0:.1f}s")
        return out
    run.prune = prune
    return run


def save_complexes(path: str, sets: Sequence[Sequence[int]]) -> None:
    """Store a list of complexes (facet mask tuples) as offsets + facets."""
    offs, fac = _pack(sets)
    np.savez_compressed(path, offsets=offs, facets=fac[:int(offs[-1])])


def load_complexes(path: str) -> List[Complex]:
    z = np.load(path)
    offs, fac = z["offsets"], z["facets"]
    return [tuple(int(v) for v in fac[offs[i]:offs[i + 1]]) for i in range(len(offs) - 1)]


def filter_report(n: int, per_orbit: Sequence[Sequence[Sequence[int]]]) -> SeedReport:
    """Lines 7 to 15 of the algorithm from the swept complexes of each orbit."""
    m = n + 4
    union = sorted({tuple(sorted(K)) for s in per_orbit for K in s})
    flags = complex_filters(n, m, union)
    want = L.CX_FULL_PICARD | L.CX_SEED
    kept = [K for K, f in zip(union, flags) if (int(f) & want) == want]
    cls, num = iso_classes(m, kept)
    reps = [None] * num
    for K, c in zip(kept, cls):
        if reps[c] is None:
            reps[c] = K
    return SeedReport(n=n, orbits=len(per_orbit), max_k=0, union=len(union), filtered=len(kept),
                      classes=num, representatives=reps)


def colorable_seeds_pic4(n: int, enumerate_sets: Optional[Callable] = None,
                         prune: bool = False, min_free: int = E.DEFAULT_MIN_FREE,
                         max_orbits: int = 0) -> SeedReport:
    """Algorithm 4.4 for Picard number 4 up to its isomorphism step.
    `enumerate_sets(preps) -> per-instance result lists` defaults to the GPU
    sweep; any exact enumerator of weak pseudo-manifolds may stand in."""
    m = n + 4
    t = {}
    t0 = time.perf_counter()
    lams = E.idcm_orbits(n)
    if max_orbits:
        lams = lams[:max_orbits]
    preps = [E.prepare(n, m, lam=lam, prune=prune and getattr(enumerate_sets, "prune", True),
                       min_free=min_free) for lam in lams]
    t["prepare"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    run = enumerate_sets or gpu_enumerator(prune=prune)
    sets = run(preps)
    t["enumerate"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    rep = filter_report(n, sets)
    t["filters"] = time.perf_counter() - t0
    rep.orbits, rep.max_k, rep.seconds = len(lams), max(p.k for p in preps), t
    return rep


def main(argv=None) -> None:
    """Run the pipeline for the given dimensions and print one JSON line each."""
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="Algorithm 4.4 (Picard number 4) up to the "
                                             "isomorphism step, on the GPU sweep")
    ap.add_argument("n", type=int, nargs="+")
    ap.add_argument("--prune", action="store_true", help="sweep convenient bases")
    ap.add_argument("--min-free", type=int, default=0,
                    help="free coordinates of a pruned instance (0 = engine default)")
    ap.add_argument("--sliced", action="store_true",
                    help="sweep each orbit in slices over its highest blocks (large n)")
    ap.add_argument("--orbits", type=int, default=0, help="only the first N orbits (timing)")
    ap.add_argument("--only-orbit", type=int, default=-1,
                    help="sweep only this orbit (0-based) and --save its complexes")
    ap.add_argument("--save", default="", help="file for the swept complexes (with --only-orbit)")
    ap.add_argument("--load", nargs="*", default=[],
                    help="files of saved orbit results: unite them and run the filters")
    args = ap.parse_args(argv)
    log = lambda msg: print(f"[seeds] {msg}", file=sys.stderr, flush=True)
    if args.only_orbit >= 0 or args.load:
        n = args.n[0]
        if args.only_orbit >= 0:
            lam = E.idcm_orbits(n)[args.only_orbit]
            p = E.prepare(n, n + 4, lam=lam, prune=args.prune,
                          min_free=args.min_free or E.DEFAULT_MIN_FREE)
            log(f"orbit {args.only_orbit}: k={p.k}, {p.visited:.3e} vectors")
            sets = sliced_sweep(p, log=log) if args.sliced else E.sweep([p])[1][0]
            save_complexes(args.save, sets)
            print(json.dumps({"n": n, "orbit": args.only_orbit, "k": p.k, "complexes": len(sets)}),
                  flush=True)
            return
        rep = filter_report(n, [load_complexes(f) for f in args.load])
        print(json.dumps({"n": n, "orbits_loaded": len(args.load), "union": rep.union,
                          "filtered": rep.filtered, "classes": rep.classes}), flush=True)
        return
    for n in args.n:
        run = gpu_enumerator(prune=args.prune, per_instance=True, log=log, sliced=args.sliced)
        rep = colorable_seeds_pic4(n, enumerate_sets=run, prune=args.prune,
                                   min_free=args.min_free or E.DEFAULT_MIN_FREE,
                                   max_orbits=args.orbits)
        print(json.dumps({"n": n, "orbits": rep.orbits, "max_k": rep.max_k, "union": rep.union,
                          "filtered": rep.filtered, "classes": rep.classes,
                          "seconds": {k: round(v, 2) for k, v in rep.seconds.items()}}),
              flush=True)


if __name__ == "__main__":
    main()
