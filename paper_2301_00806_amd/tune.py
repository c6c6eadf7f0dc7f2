"""Autotuner for the persistent sweep: lane chunk bits, workgroup size and
the kernel's register budget (7 or 8 waves per SIMD); for a pruned sweep
also the free coordinates a convenient basis keeps (min_free).

It times candidate launch shapes on the batch itself when a sweep of it takes
well under a second, else on a sample that keeps the batch's mix (every
instance whose index falls on a stride, so that large and small kernels are
represented as in the batch), keeps the fastest, and
caches the choice in a JSON file keyed by the GPU architecture, the kernel
source and a shape bucket of the batch (widest table row, log2 of the vectors
per instance, pruned or not).  Counts are identical for every shape; the
tuner checks that too.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Optional, Sequence

import numpy as np

from . import _lib as L
from . import engine as E

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "wpm_tune.json")
CBITS = (10, 11, 12, 13, 14)
WGS = (256, 512)
WAVES = (7, 8)


def shape_key(batch: "E.DeviceBatch") -> str:
    import hashlib
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    b = batch.c_batch
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "sweep_kernel.h")
    with open(src, "rb") as f:
        kh = hashlib.sha256(f.read()).hexdigest()[:12]
    lv = int(np.log2(max(1.0, batch.visited / max(1, len(batch.preps)))))
    pr = "/pruned" if batch.blocks is not None else ""
    return f"{arch}/{kh}/rs{b.max_row_words}/v{lv}{pr}"


def _sample(preps, budget_vectors: float):
    """All instances when their vectors fit the budget, else every s-th
    instance with the smallest stride s that fits it."""
    total = float(sum(p.visited for p in preps))
    if total <= budget_vectors:
        return list(range(len(preps)))
    stride = int(np.ceil(total / budget_vectors))
    while True:
        idx = list(range(0, len(preps), stride))
        if float(sum(preps[i].visited for i in idx)) <= budget_vectors or stride > len(preps):
            return idx
        stride += 1


def tune(preps: Sequence, cache: Optional[str] = DEFAULT_CACHE, budget_vectors: float = 3e12,
         cbits=CBITS, wgs=WGS, waves=WAVES, repeats: int = 1, force: bool = False, log=None) -> Dict:
    import torch
    full = E.DeviceBatch(preps)
    key = shape_key(full)
    db = {}
    if cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                db = json.load(f)
        except (OSError, ValueError):
            db = {}
    if key in db and not force:
        return dict(db[key], cached=True, key=key)
    idx = _sample(preps, budget_vectors)
    sub = [preps[i] for i in idx]
    batch = E.DeviceBatch(sub)
    sw = E.Sweeper(batch, cap=1 << 26)
    vec = batch.visited
    results, ref = [], None
    for wg in wgs:
        for cb in cbits:
            items = E.build_queue(batch.k, cb, wg, cost=np.ones(len(sub), np.float32), order=1,
                                  blocks=batch.blocks)
            sw.set_items(items)
            for wv in waves:
                sw.launch(L.SCHED_DYNAMIC, wg_size=wg, waves=wv)
                r = sw.result()
                if ref is None:
                    ref = r.counts.copy()
                if not np.array_equal(r.counts, ref):
                    raise RuntimeError(f"counts changed with cbits={cb} wg={wg} waves={wv}")
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(repeats):
                    sw.launch(L.SCHED_DYNAMIC, wg_size=wg, waves=wv)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / repeats
                results.append({"cbits": cb, "wg": wg, "waves": wv, "ms": ms,
                                "vectors_per_s": vec / ms * 1e3})
                if log:
                    log(f"tune cbits={cb} wg={wg} waves={wv}: {ms:.2f} ms ({vec / ms * 1e3:.3e} vectors/s)")
    best = max(results, key=lambda r: r["vectors_per_s"])
    entry = {"cbits": best["cbits"], "wg": best["wg"], "waves": best["waves"],
             "sample_instances": len(sub), "sample_vectors": vec, "results": results,
             "when": time.time()}
    if cache:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        db[key] = entry
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1)
        os.replace(tmp, cache)
    return dict(entry, cached=False, key=key)


MIN_FREES = (16, 18, 20)
PRUNED_CBITS = (10, 12)


def tune_pruned(insts: Sequence, cache: Optional[str] = DEFAULT_CACHE, min_frees=MIN_FREES,
                cbits=PRUNED_CBITS, wg: int = 256, waves: int = 8, force: bool = False,
                log=None):
    """Free coordinates and chunk bits of a pruned sweep, chosen by the
    time of the whole batch: fewer free coordinates prune more vectors but
    shorten the lane chunks of each block tuple (one tuple spans 2^min_free
    indices).  The score is the covered vectors (the plain sweep's 2^k) per
    second.  Returns (entry, preps prepared with the chosen min_free)."""
    import torch
    db = {}
    if cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                db = json.load(f)
        except (OSError, ValueError):
            db = {}
    prepared = {}

    def prep(mf):
        if mf not in prepared:
            prepared[mf] = E.prepare_many(insts, prune=True, min_free=mf)
        return prepared[mf]

    first = prep(min_frees[len(min_frees) // 2])
    key = shape_key(E.DeviceBatch(first)) + "/minfree"
    if key in db and not force:
        e = db[key]
        return dict(e, cached=True, key=key), prep(int(e["min_free"]))
    results, ref = [], None
    covered = float(sum(1 << p.k for p in first))
    for mf in min_frees:
        batch = E.DeviceBatch(prep(mf))
        sw = E.Sweeper(batch, cap=1 << 26)
        for cb in cbits:
            items = E.build_queue(batch.k, cb, wg, cost=np.ones(len(batch.preps), np.float32),
                                  order=1, blocks=batch.blocks)
            sw.set_items(items)
            sw.launch(L.SCHED_DYNAMIC, wg_size=wg, waves=waves)
            r = sw.result()
            if ref is None:
                ref = r.counts.copy()
            if not np.array_equal(r.counts, ref):
                raise RuntimeError(f"counts changed with min_free={mf} cbits={cb}")
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            sw.launch(L.SCHED_DYNAMIC, wg_size=wg, waves=waves)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            results.append({"min_free": mf, "cbits": cb, "ms": ms, "visited": batch.visited,
                            "covered_per_s": covered / ms * 1e3})
            if log:
                log(f"tune pruned min_free={mf} cbits={cb}: {ms:.2f} ms, visits {batch.visited:.3e} "
                    f"({covered / ms * 1e3:.3e} covered vectors/s)")
        del sw, batch
    best = max(results, key=lambda r: r["covered_per_s"])
    entry = {"min_free": best["min_free"], "cbits": best["cbits"], "wg": wg, "waves": waves,
             "results": results, "when": time.time()}
    if cache:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        db[key] = entry
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1)
        os.replace(tmp, cache)
    return dict(entry, cached=False, key=key), prep(int(best["min_free"]))
