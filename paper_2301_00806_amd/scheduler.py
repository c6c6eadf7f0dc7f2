"""Scheduling policies for batched sweeps (host side; results never depend on them).

  plain     one launch per instance (the per-instance baseline)
  static    one persistent launch; workgroup g takes items g, g+G, ... in
            instance order (round robin, no cost information: the fallback)
  dynamic   one persistent launch; workgroups pop items from a device queue
            ordered by decreasing estimated cost (LPT)
  packed    one launch; items assigned to workgroups ahead of time by LPT bin
            packing on estimated cost (no queue at run time)

Estimated cost of an item = (vectors in the item) x (per-vector cost of its
instance).  The per-vector cost comes either from the learned model
(costmodel.CostModel, predicting ns per vector) or from the "cost is
proportional to 2^k" heuristic (per-vector cost 1).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import _lib as L
from . import engine as E

POLICIES = ("plain", "static", "dynamic", "packed")


@dataclass
class Plan:
    policy: str
    mode: int
    items: np.ndarray
    segments: Optional[list] = None
    predicted_makespan: float = 0.0


def per_vector_cost(model, features: np.ndarray, stream=None) -> np.ndarray:
    """ns per vector from the model (its first output is ln ns/vector)."""
    y = model.predict(features, stream=stream)
    return np.exp(np.clip(y[:, 0], -20.0, 20.0)).astype(np.float32)


def _items(batch, split: bool, cbits: int, wg: int, cost=None, order: int = 0,
           min_items: int = 1):
    if split:
        return E.class_items(batch, cbits, wg, cost=cost, order=order,
                             min_items_per_instance=min_items)
    items = E.build_queue(batch.k, cbits, wg, cost=cost, order=order,
                          min_items_per_instance=min_items, blocks=batch.blocks)
    return items, [E.Segment(None, 0, len(items))]


def make_plan(batch: "E.DeviceBatch", policy: str, cost: Optional[np.ndarray] = None,
              cbits: int = 16, wg: int = 256, plain_min_items: int = 512,
              split: bool = True) -> Plan:
    """Items for a policy; with `split`, grouped by launch class (one launch
    per class, each with the LDS layout its tables need), else one launch for
    the whole batch."""
    if policy == "plain":
        items, segs = _items(batch, split, cbits, wg, min_items=plain_min_items)
        return Plan(policy, L.SCHED_PLAIN, items, segs)
    if policy == "static":
        items, segs = _items(batch, split, cbits, wg)
        return Plan(policy, L.SCHED_STATIC, items, segs)
    c = np.ones(len(batch.k), np.float32) if cost is None else np.asarray(cost, np.float32)
    items, segs = _items(batch, split, cbits, wg, cost=c, order=1)
    if policy == "dynamic":
        return Plan(policy, L.SCHED_DYNAMIC, items, segs)
    if policy == "packed":
        parts, out_segs, pos, mk = [], [], 0, 0.0
        for sg in segs:
            bins = E.persistent_grid(batch, wg, sg.cls)
            it, offs, mx = E.pack_bins(items[sg.start:sg.end], bins, c)
            parts.append(it)
            out_segs.append(E.Segment(sg.cls, pos, pos + len(it), offs))
            pos += len(it)
            mk += mx
        return Plan(policy, L.SCHED_PACKED, np.concatenate(parts) if parts else items, out_segs, mk)
    raise ValueError(policy)


def measure_labels(preps, cbits: int = 12, wg: int = 256, repeats: int = 2):
    """Sweep the instances with per-item timing; return (features, labels, counts).
    Labels are averaged over `repeats` timed runs (after one warm-up)."""
    from . import costmodel as CM
    _, clk, _ = E.device_query()
    batch = E.DeviceBatch(preps)
    sw = E.Sweeper(batch, cap=1 << 22)
    items = E.build_queue(batch.k, cbits, wg, cost=np.ones(len(preps), np.float32), order=1,
                          blocks=batch.blocks)
    sw.set_items(items, want_times=True)
    items = sw._items_host  # grouped by launch class, as launched
    sw.launch(L.SCHED_DYNAMIC, wg_size=wg)
    sw.result()
    labs = []
    for _ in range(repeats):
        sw.launch(L.SCHED_DYNAMIC, wg_size=wg)
        res = sw.result()
        labs.append(CM.labels_from_sweep(preps, res, clk))
    lab = np.mean(labs, 0).astype(np.float32)
    return CM.features_of(preps), lab, res.counts
