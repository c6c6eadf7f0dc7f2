"""Python driver over the C ABI: instance preparation, device batches, sweep.

PyTorch provides device memory and the stream only; every step of the
enumeration runs in libwpm.so (host preparation in C++, the sweep in HIP).
"""
from __future__ import annotations

import ctypes
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import _lib as L

_POOL_THREADS = int(os.environ.get("WPM_PREP_THREADS", str(min(16, os.cpu_count() or 4))))


def _ptr(a: np.ndarray, t=L.c_u32p):
    return a.ctypes.data_as(t)


def ubt_bound(n: int) -> int:
    return int(L.lib().wpm_ubt_bound(n))


def default_max_facets(n: int, m: int) -> int:
    """Algorithm 4.4 applies the upper-bound property at Picard number 4."""
    return ubt_bound(n) if m == n + 4 else 0


def candidates(n: int, m: int, lam: Sequence[int]) -> np.ndarray:
    lib = L.lib()
    la = np.ascontiguousarray(np.asarray(lam, dtype=np.uint32))
    Mo = ctypes.c_int32(0)
    cap = 2048
    while True:
        out = np.zeros(cap, dtype=np.uint32)
        st = lib.wpm_build_candidates(n, m, _ptr(la), _ptr(out), cap, ctypes.byref(Mo))
        if st == L.WPM_ECAP:
            cap = Mo.value
            continue
        L.check("wpm_build_candidates", st)
        return out[:Mo.value].copy()


def kernel_basis(n: int, m: int, facets: np.ndarray) -> Tuple[np.ndarray, np.ndarray, int]:
    """(ridges, basis[k, W], k)."""
    lib = L.lib()
    F = np.ascontiguousarray(facets, dtype=np.uint32)
    M = len(F)
    W = (M + 31) // 32
    No = ctypes.c_int32(0)
    ko = ctypes.c_int32(0)
    cap_r = max(1, M * n)
    ridges = np.zeros(cap_r, dtype=np.uint32)
    st = lib.wpm_kernel_basis(n, m, _ptr(F), M, _ptr(ridges), cap_r, ctypes.byref(No), None, 0,
                              ctypes.byref(ko))
    L.check("wpm_kernel_basis", st, (L.WPM_OK, L.WPM_ECAP))
    k = ko.value
    basis = np.zeros(max(1, k * W), dtype=np.uint32)
    st = lib.wpm_kernel_basis(n, m, _ptr(F), M, _ptr(ridges), cap_r, ctypes.byref(No),
                              _ptr(basis), k, ctypes.byref(ko))
    L.check("wpm_kernel_basis", st)
    return ridges[:No.value].copy(), basis[:k * W].reshape(k, W) if W else basis[:0].reshape(0, 0), k


# Free coordinates a pruned instance keeps by default.  One allowed block
# tuple then spans at least 2^18 Gray indices: a full 256-lane workgroup with
# 2^10 indices per lane.  Fewer free coordinates prune more but shorten the
# lane chunks; on the 16384-instance learned batch 16, 18 and 20 gave kernel
# times of 99.8, 93.3 and 104.0 ms.
DEFAULT_MIN_FREE = 18


def convenient_basis(n: int, m: int, facets: np.ndarray, basis: np.ndarray, k: int,
                     min_free: int = DEFAULT_MIN_FREE):
    """(convenient basis [k, W], wpm_blocks) of wpm_convenient_basis."""
    F = np.ascontiguousarray(facets, dtype=np.uint32)
    W = (len(F) + 31) // 32
    Bf = np.ascontiguousarray(np.asarray(basis, dtype=np.uint32).reshape(-1))
    if Bf.size == 0:
        Bf = np.zeros(1, dtype=np.uint32)
    out = np.zeros(max(1, k * W), dtype=np.uint32)
    blk = L.Blocks()
    st = L.lib().wpm_convenient_basis(n, m, _ptr(F), len(F), _ptr(Bf), k, min_free, _ptr(out),
                                      ctypes.byref(blk))
    L.check("wpm_convenient_basis", st)
    return out[:k * W].reshape(k, W), blk


def blocks_vectors(blk) -> int:
    """Exact number of vectors a pruned sweep visits: 2^f * prod count[b]."""
    v = 1 << int(blk.free_dims)
    for b in range(int(blk.num_blocks)):
        v *= int(blk.count[b])
    return v


def idcm_orbits(n: int, p: int = 4) -> List[List[int]]:
    """One characteristic matrix [I_n | M] (as n + p columns) per IDCM orbit
    of Lambda(n, p) (wpm_idcm_orbits)."""
    lib = L.lib()
    cnt = ctypes.c_int64(0)
    L.check("wpm_idcm_orbits", lib.wpm_idcm_orbits(n, p, None, 0, ctypes.byref(cnt)))
    m = n + p
    out = np.zeros(max(1, cnt.value * m), dtype=np.uint32)
    L.check("wpm_idcm_orbits", lib.wpm_idcm_orbits(n, p, _ptr(out), cnt.value, ctypes.byref(cnt)))
    return [[int(v) for v in out[r * m:(r + 1) * m]] for r in range(cnt.value)]


def facet_mask(facets: np.ndarray, chosen) -> np.ndarray:
    """W-word bit mask (bit j = facet j) of the given facet vertex masks."""
    F = np.asarray(facets, dtype=np.uint32)
    pos = {int(f): j for j, f in enumerate(F)}
    out = np.zeros(max(1, (len(F) + 31) // 32), dtype=np.uint32)
    for f in chosen:
        j = pos.get(int(f))
        if j is None:
            raise ValueError(f"facet {int(f):#x} is not a candidate")
        out[j // 32] |= np.uint32(1 << (j % 32))
    return out


def facet_conditions(n: int, m: int, facets: np.ndarray, basis: np.ndarray, k: int,
                     forced_in=(), forced_out=()):
    """(basis [k', W], k', offset [W], feasible) of wpm_facet_conditions; the
    forced facets are given as vertex masks."""
    F = np.ascontiguousarray(facets, dtype=np.uint32)
    W = (len(F) + 31) // 32
    Bf = np.ascontiguousarray(np.asarray(basis, dtype=np.uint32).reshape(-1))
    if Bf.size == 0:
        Bf = np.zeros(1, dtype=np.uint32)
    fi, fo = facet_mask(F, forced_in), facet_mask(F, forced_out)
    out = np.zeros(max(1, k * W), dtype=np.uint32)
    off = np.zeros(max(1, W), dtype=np.uint32)
    ko, feas = ctypes.c_int32(0), ctypes.c_int32(0)
    st = L.lib().wpm_facet_conditions(n, m, _ptr(F), len(F), _ptr(Bf), k, _ptr(fi), _ptr(fo),
                                      _ptr(out), ctypes.byref(ko), _ptr(off), ctypes.byref(feas))
    L.check("wpm_facet_conditions", st)
    kk = ko.value
    return out[:kk * W].reshape(kk, W), kk, off[:W].copy(), bool(feas.value)


@dataclass
class Prepared:
    n: int
    m: int
    facets: np.ndarray
    k: int
    basis: np.ndarray           # [k, W] uint32
    N: int
    max_facets: int
    table: Optional[np.ndarray] = None
    info: Optional[L.InstanceInfo] = None
    tag: str = ""
    blocks: Optional[L.Blocks] = None   # convenient-basis structure (pruned sweep)
    offset: Optional[np.ndarray] = None  # [W] offset K* of an affine coset
    props: Optional[list] = None         # [(c0, [(weight, [facet masks])...])...]
    feasible: bool = True                # False: the facet conditions admit no complex
    max_groups: int = 0                  # resident ridge groups (0: engine maximum)

    @property
    def W(self) -> int:
        return (len(self.facets) + 31) // 32

    @property
    def vectors(self) -> int:
        """Size of the kernel, 2^k."""
        return 1 << self.k

    @property
    def visited(self) -> int:
        """Vectors the sweep visits: 2^k, or the pruned product."""
        return self.vectors if self.blocks is None else blocks_vectors(self.blocks)


def prepare(n: int, m: int, lam: Optional[Sequence[int]] = None,
            facets: Optional[Sequence[int]] = None, max_facets: Optional[int] = None,
            seed: int = 0, pack: bool = True, prune: bool = False,
            min_free: int = DEFAULT_MIN_FREE, forced_in=None, forced_out=None,
            properties=None, max_groups: int = 0) -> Prepared:
    """Candidates (if lambda is given), ridges, kernel basis and packed table.
    With `prune`, the basis is replaced by a convenient basis and the sweep
    visits only the product of its blocks' allowed sets (same results).
    forced_in / forced_out (facet vertex masks) keep only complexes that
    contain / avoid those facets; properties [(c0, [(weight, facets), ...])]
    keep only complexes with c0 + sum weight * |K & facets| > 0 for each."""
    if facets is None:
        F = candidates(n, m, lam)
    else:
        F = np.ascontiguousarray(np.asarray(facets, dtype=np.uint32))
    if max_facets is None:
        max_facets = default_max_facets(n, m)
    ridges, B, k = kernel_basis(n, m, F)
    blk, off, feasible = None, None, True
    if forced_in or forced_out:
        B, k, off, feasible = facet_conditions(n, m, F, B, k, forced_in or (), forced_out or ())
        if not forced_in or not feasible:
            off = None          # a subspace (no offset), or nothing to sweep
        if not feasible:
            k = 0
            B = B[:0]
    if prune and k > 0:
        if off is not None:
            raise ValueError("block pruning needs a linear span (no forced-in facets)")
        B, blk = convenient_basis(n, m, F, B, k, min_free)
    p = Prepared(n=n, m=m, facets=F, k=k, basis=np.ascontiguousarray(B), N=len(ridges),
                 max_facets=max_facets, blocks=blk, offset=off, props=properties,
                 feasible=feasible, max_groups=max_groups)
    if pack:
        pack_prepared(p, seed)
    return p


def pack_prepared(p: Prepared, seed: int = 0) -> None:
    lib = L.lib()
    info = L.InstanceInfo()
    Bf = np.ascontiguousarray(p.basis.reshape(-1), dtype=np.uint32)
    if Bf.size == 0:
        Bf = np.zeros(1, dtype=np.uint32)
    bp = None if p.blocks is None else ctypes.byref(p.blocks)
    conds, keep = _conditions(p)
    cp = None if conds is None else ctypes.byref(conds)
    st = lib.wpm_pack_instance(p.n, p.m, _ptr(p.facets), len(p.facets), _ptr(Bf), p.k, bp, cp,
                               p.max_facets, seed, None, 0, ctypes.byref(info))
    L.check("wpm_pack_instance", st, (L.WPM_ECAP,))
    tab = np.zeros(info.table_words, dtype=np.uint32)
    st = lib.wpm_pack_instance(p.n, p.m, _ptr(p.facets), len(p.facets), _ptr(Bf), p.k, bp, cp,
                               p.max_facets, seed, _ptr(tab), info.table_words, ctypes.byref(info))
    L.check("wpm_pack_instance", st)
    p.table, p.info = tab, info


def _conditions(p: Prepared):
    """wpm_conditions of a prepared instance (and the arrays it points into)."""
    if p.offset is None and not p.props and not p.max_groups:
        return None, None
    keep = []
    c = L.Conditions()
    c.max_groups = p.max_groups
    if p.offset is not None:
        off = np.ascontiguousarray(p.offset, dtype=np.uint32)
        keep.append(off)
        c.offset = off.ctypes.data
    props = p.props or []
    c.num_props = len(props)
    if props:
        c0 = np.array([int(q[0]) for q in props], dtype=np.int32)
        ncls = np.array([len(q[1]) for q in props], dtype=np.int32)
        wts = np.array([int(w) for q in props for w, _ in q[1]] or [0], dtype=np.int32)
        masks = np.concatenate([facet_mask(p.facets, fs) for q in props for _, fs in q[1]]
                               or [np.zeros(1, np.uint32)])
        keep += [c0, ncls, wts, masks]
        c.prop_c0, c.prop_classes = c0.ctypes.data, ncls.ctypes.data
        c.class_weight, c.class_mask = wts.ctypes.data, masks.ctypes.data
    return c, keep


def kdim(inst) -> int:
    """Kernel dimension of a wpm_inputs.Instance with this engine's own code."""
    F = candidates(inst.n, inst.m, inst.lam) if inst.facets is None else np.asarray(inst.facets, np.uint32)
    return kernel_basis(inst.n, inst.m, F)[2]


def prepare_many(insts, seed: int = 0, threads: int = _POOL_THREADS, prune: bool = False,
                 min_free: int = DEFAULT_MIN_FREE) -> List[Prepared]:
    """prepare() over wpm_inputs.Instance objects, in parallel host threads
    (the C calls release the GIL)."""
    def one(a):
        i, inst = a
        p = prepare(inst.n, inst.m, lam=inst.lam, facets=inst.facets, seed=seed + i,
                    prune=prune, min_free=min_free)
        p.tag = inst.tag
        return p
    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        return list(ex.map(one, enumerate(insts)))


def valu_probe(op: int = 0, waves_per_simd: int = 4, iters: int = 20000) -> float:
    """Measured 32-bit integer lane-ops/s of the device (see wpm_valu_probe)."""
    v = ctypes.c_double(0)
    L.check("wpm_valu_probe", L.lib().wpm_valu_probe(op, waves_per_simd, iters, ctypes.byref(v)))
    return v.value


def device_query():
    cus = ctypes.c_int32(0)
    clk = ctypes.c_int64(0)
    lds = ctypes.c_int32(0)
    L.check("wpm_device_query", L.lib().wpm_device_query(ctypes.byref(cus), ctypes.byref(clk),
                                                         ctypes.byref(lds)))
    return cus.value, clk.value, lds.value


ITEM_DTYPE = np.dtype([("instance", "<u4"), ("cbits", "<u2"), ("lanes", "<u2"), ("first", "<u8")])


# Row widths that bound a launch's LDS layout.  One kernel sweeps every
# instance; a launch sizes each workgroup's LDS for its widest table, so
# instances are launched in classes of similar width: 8 workgroups of 256
# threads fit a compute unit up to 44 words per row (with kp <= 36), 6 up to
# 64.
LDS_CLASSES = (44, 64, 96, L.MAX_ROW_WORDS)


def lds_class(info) -> int:
    """The launch class of an instance: the smallest row-width bound of
    LDS_CLASSES that holds its table rows."""
    return next(c for c in LDS_CLASSES if info.row_words <= c)


class DeviceBatch:
    """Packed tables of a list of prepared instances, resident in HBM."""

    def __init__(self, preps: Sequence[Prepared], device="cuda"):
        import torch
        self.preps = list(preps)
        sizes = [int(p.info.table_words) for p in self.preps]
        padded = [(s + 3) & ~3 for s in sizes]
        offs = np.zeros(len(self.preps), dtype=np.int64)
        if len(self.preps) > 1:
            offs[1:] = np.cumsum(padded[:-1])
        total = int(sum(padded)) if self.preps else 4
        host = np.zeros(max(total, 4), dtype=np.uint32)
        for p, o in zip(self.preps, offs):
            host[o:o + len(p.table)] = p.table
        self.tables = torch.from_numpy(host.view(np.int32)).to(device)
        self.offsets = torch.from_numpy(offs).to(device)
        # kernel dimensions for the queue: a coset with k = 0 still holds one
        # complex (x = 0 is K*), so it is queued as k = 1; the table's own k
        # keeps the sweep to x = 0
        self.k = np.array([p.k if (p.k > 0 or p.offset is None) else 1 for p in self.preps],
                          dtype=np.int32)
        # wpm_blocks of every instance when any is pruned (plain ones: no blocks)
        self.blocks = None
        if any(p.blocks is not None for p in self.preps):
            self.blocks = (L.Blocks * len(self.preps))()
            for i, p in enumerate(self.preps):
                if p.blocks is not None:
                    self.blocks[i] = p.blocks
                else:
                    self.blocks[i].k = p.k
                    self.blocks[i].free_dims = p.k
        self.cls = np.array([lds_class(p.info) for p in self.preps], dtype=np.int64)
        self.c_batch = self._batch_of(self.preps)
        self.class_batches = {int(c): self._batch_of([p for p, q in zip(self.preps, self.cls) if q == c])
                              for c in np.unique(self.cls)}
        self.table_bytes = total * 4

    def _batch_of(self, members) -> "L.Batch":
        return L.Batch(
            num_instances=len(self.preps),
            max_row_words=max([p.info.row_words for p in members] + [4]),
            max_groups=max([p.info.groups for p in members] + [1]),
            max_slots=max([p.info.slots for p in members] + [4]),
            max_words=max([p.info.W for p in members] + [1]),
            max_kp=max([max(p.k, 7) for p in members] + [7]),
            d_tables=self.tables.data_ptr(), d_offsets=self.offsets.data_ptr(), flags=0)

    @property
    def vectors(self) -> int:
        """Sum of 2^k: the kernel vectors the batch covers."""
        return int(sum(1 << int(k) for k in self.k))

    @property
    def visited(self) -> int:
        """Vectors a sweep of the batch visits (less than `vectors` when pruned)."""
        return int(sum(p.visited for p in self.preps))

    def class_queue_args(self):
        """Per launch class, widest first: (class, vectors visited, k with
        the other classes' instances zeroed, wpm_blocks likewise or None),
        built once per batch."""
        if getattr(self, "_cq", None) is None:
            vis = np.array([float(p.visited) if p.k > 0 else 0.0 for p in self.preps])
            out = []
            for code in sorted(np.unique(self.cls), reverse=True):
                sel = self.cls == code
                vec = float(vis[sel].sum())
                if vec == 0.0:
                    continue
                k_sel = np.where(sel, self.k, 0).astype(np.int32)
                blocks = None
                if self.blocks is not None:
                    blocks = (L.Blocks * len(self.preps))()
                    for i in np.flatnonzero(sel):
                        blocks[i] = self.blocks[i]
                out.append((int(code), vec, k_sel, blocks))
            self._cq = out
        return self._cq

    def class_grid(self, cls: int, wg_size: int) -> int:
        """persistent_grid of one launch class, cached per workgroup size."""
        if getattr(self, "_grids", None) is None:
            self._grids = {}
        key = (cls, wg_size)
        if key not in self._grids:
            self._grids[key] = persistent_grid(self, wg_size, cls)
        return self._grids[key]


class PinnedItems(np.ndarray):
    """Items in pinned host memory (`_tensor` owns it), which set_items
    copies to the device asynchronously."""

    def __array_finalize__(self, obj):
        self._tensor = getattr(obj, "_tensor", None)


def pinned_items(n: int) -> np.ndarray:
    """An item array of length n in pinned host memory (plain memory when
    no GPU is present)."""
    import torch
    if not torch.cuda.is_available():
        return np.zeros(n, dtype=ITEM_DTYPE)
    t = torch.empty(max(1, n) * ITEM_DTYPE.itemsize, dtype=torch.uint8, pin_memory=True)
    arr = t.numpy().view(ITEM_DTYPE)[:n].view(PinnedItems)
    arr._tensor = t
    return arr


def build_queue(k: np.ndarray, cbits: int, lanes: int, cost: Optional[np.ndarray] = None,
                max_items_per_instance: int = 0, order: int = 0,
                min_items_per_instance: int = 1, group: Optional[np.ndarray] = None,
                return_counts: bool = False, blocks=None, out=None, count_only: bool = False):
    """Items of a batch (wpm_build_queue; wpm_build_pruned_queue when
    `blocks`, a ctypes array of wpm_blocks, is given).  With `group`, items
    come out group by group in decreasing group key; return_counts adds the
    items per instance.  `out`, a callable taking the item count, supplies
    the array to fill (default: a new array); count_only returns the item
    count alone."""
    lib = L.lib()
    ka = np.ascontiguousarray(k, dtype=np.int32)
    ca = None if cost is None else np.ascontiguousarray(cost, dtype=np.float32)
    ga = None if group is None else np.ascontiguousarray(group, dtype=np.int32)
    n = ctypes.c_int64(0)
    cp = None if ca is None else _ptr(ca, L.c_f32p)
    gp = None if ga is None else _ptr(ga, L.c_i32p)
    per = np.zeros(max(1, len(ka)), dtype=np.int64)
    if blocks is not None:
        if len(blocks) != len(ka):
            raise ValueError("one wpm_blocks per instance")
        call, name, first = lib.wpm_build_pruned_queue, "wpm_build_pruned_queue", blocks
    else:
        call, name, first = lib.wpm_build_queue, "wpm_build_queue", _ptr(ka, L.c_i32p)
    st = call(first, cp, gp, len(ka), cbits, lanes, min_items_per_instance,
              max_items_per_instance, order, None, 0, ctypes.byref(n), None)
    L.check(name, st, (L.WPM_ECAP, L.WPM_OK))
    if count_only:
        return n.value
    arr = np.zeros(max(1, n.value), dtype=ITEM_DTYPE) if out is None else out(n.value)
    if n.value:
        st = call(first, cp, gp, len(ka), cbits, lanes, min_items_per_instance,
                  max_items_per_instance, order, arr.ctypes.data_as(ctypes.POINTER(L.Item)), n.value,
                  ctypes.byref(n), _ptr(per, L.c_i64p))
        L.check(name, st)
    arr = arr[:n.value]
    return (arr, per[:len(ka)]) if return_counts else arr


def pack_bins(items: np.ndarray, bins: int, cost: Optional[np.ndarray] = None):
    """LPT assignment of items to `bins` workgroups -> (items bin by bin, offsets[bins+1], max load)."""
    items = np.ascontiguousarray(items)
    n = len(items)
    src = (L.Item * max(1, n)).from_buffer_copy(items.tobytes() if n else bytes(16))
    out = (L.Item * max(1, n))()
    offs = np.zeros(bins + 1, dtype=np.int64)
    mx = ctypes.c_double(0)
    ca = None if cost is None else np.ascontiguousarray(cost, dtype=np.float32)
    st = L.lib().wpm_pack_bins(src, n, None if ca is None else _ptr(ca, L.c_f32p), bins, out,
                               _ptr(offs, L.c_i64p), ctypes.byref(mx))
    L.check("wpm_pack_bins", st)
    arr = np.frombuffer(out, dtype=ITEM_DTYPE, count=n).copy()
    return arr, offs, mx.value


def persistent_grid(batch: "DeviceBatch", wg_size: int, cls: Optional[int] = None) -> int:
    """Workgroups of a persistent launch (of one launch class, or of the
    whole batch with the LDS layout of its widest table)."""
    cb = batch.c_batch if cls is None else batch.class_batches[int(cls)]
    g = ctypes.c_int32(0)
    L.check("wpm_persistent_grid", L.lib().wpm_persistent_grid(ctypes.byref(cb), wg_size,
                                                               ctypes.byref(g)))
    return g.value


@dataclass
class Segment:
    """Items [start, end) launched together (one launch class)."""
    cls: Optional[int]
    start: int
    end: int
    bins: Optional[np.ndarray] = None


def split_by_class(batch: "DeviceBatch", items: np.ndarray):
    """Stable grouping of items by their instance's launch class, widest
    class first -> (items, segments)."""
    if len(items) == 0:
        return items, []
    c = batch.cls[items["instance"].astype(np.int64)]
    order = np.argsort(-c, kind="stable")
    items = items[order]
    c = c[order]
    cuts = np.flatnonzero(np.diff(c)) + 1
    starts = np.concatenate([[0], cuts])
    ends = np.concatenate([cuts, [len(items)]])
    return items, [Segment(int(c[a]), int(a), int(b)) for a, b in zip(starts, ends)]


def class_items(batch: "DeviceBatch", cbits: int, lanes: int, cost: Optional[np.ndarray] = None,
                order: int = 0, min_items_per_instance: int = 1, max_items_per_instance: int = 0,
                fill: int = 4):
    """Items grouped by launch class (widest first), with their segments:
    one launch per class.  A class too small to give its persistent grid
    `fill` items per workgroup at `cbits` gets shorter lane chunks (down to
    2^7), so that its launch spreads over the whole device instead of
    running a few long items on an otherwise idle GPU."""
    plan = []
    for code, vec, k_sel, blocks in batch.class_queue_args():
        c = cbits
        if fill > 0:
            grid = batch.class_grid(int(code), lanes)
            while c > 7 and vec / (lanes * float(1 << c)) < fill * grid:
                c -= 1
        plan.append((code, c, k_sel, blocks))
    kw = dict(cost=cost, order=order, min_items_per_instance=min_items_per_instance,
              max_items_per_instance=max_items_per_instance)
    # count each class's items, then build them all into one pinned array
    counts = [build_queue(k_sel, c, lanes, blocks=blocks, count_only=True, **kw)
              for code, c, k_sel, blocks in plan]
    items = pinned_items(int(sum(counts)))
    segs, pos = [], 0
    for (code, c, k_sel, blocks), n in zip(plan, counts):
        if n:
            build_queue(k_sel, c, lanes, blocks=blocks, out=lambda m, a=pos: items[a:a + m], **kw)
            segs.append(Segment(int(code), pos, pos + n))
            pos += n
    return items, segs


@dataclass
class SweepResult:
    counts: np.ndarray
    total: int
    slots: int
    stats: np.ndarray
    ms: float = 0.0
    item_times: Optional[np.ndarray] = None
    items: Optional[np.ndarray] = None


class Sweeper:
    """Device buffers and one call of wpm_enumerate over a DeviceBatch."""

    def __init__(self, batch: DeviceBatch, cap: int = 1 << 20, device="cuda",
                 records_on_host: bool = False):
        """With records_on_host, the survivor records live in pinned host
        memory that the sweep writes directly (no copy back afterwards)."""
        import torch
        self.torch = torch
        self.batch = batch
        self.cap = cap
        self.records_on_host = records_on_host
        self.device = torch.device(device)
        if records_on_host:
            self.surv = torch.empty((max(cap, 1), 2), dtype=torch.int64, pin_memory=True)
        else:
            self.surv = torch.empty((max(cap, 1), 2), dtype=torch.int64, device=device)
        self.counts = torch.empty(max(1, len(batch.preps)), dtype=torch.int64, device=device)
        # [results, record slots, malformed items skipped, 0]
        self.total = torch.empty(L.TOTAL_WORDS, dtype=torch.int64, device=device)
        self.stats = torch.empty(8, dtype=torch.int64, device=device)
        self.scratch = torch.empty(4, dtype=torch.int64, device=device)
        self._items_dev = None
        self._items_host = None
        self._times = None
        self._segments = []
        self._seg_bins = []
        self._staging = None  # pinned copy target of HBM records (reserve_host_staging)

    def set_items(self, items: np.ndarray, want_times: bool = False,
                  bin_offsets: Optional[np.ndarray] = None, segments=None,
                  split_classes: bool = True):
        """Upload the items.  By default items are grouped by launch class
        and launched class by class; `segments` gives that grouping
        explicitly (packed plans carry per-segment bins); bin_offsets alone
        means one packed launch with the batch-wide LDS layout."""
        torch = self.torch
        if segments is None:
            if bin_offsets is not None or not split_classes:
                segments = [Segment(None, 0, len(items), bin_offsets)]
            else:
                items, segments = split_by_class(self.batch, np.ascontiguousarray(items))
        pinned = getattr(items, "_tensor", None)
        if pinned is not None and (items.ctypes.data != pinned.data_ptr() or not items.flags["C_CONTIGUOUS"]):
            pinned = None   # a view into the pinned array: copied the plain way
        self._items_host = items if pinned is not None else np.ascontiguousarray(items)
        self._segments = segments
        self._seg_bins = [None if sg.bins is None else torch.from_numpy(
            np.ascontiguousarray(sg.bins, np.int64)).to(self.device) for sg in segments]
        if pinned is not None and len(items):
            # pinned host items (class_items builds them there): an
            # asynchronous copy on the current stream; the pinned block is
            # not reused before the copy has run
            self._items_dev = torch.empty(2 * len(items), dtype=torch.int64, device=self.device)
            self._items_dev.copy_(pinned[:16 * len(items)].view(torch.int64), non_blocking=True)
        else:
            raw = self._items_host.view(np.int64).reshape(-1) if len(items) else np.zeros(2, np.int64)
            self._items_dev = torch.from_numpy(raw.copy()).to(self.device)
        self._times = (torch.zeros((max(1, len(items)), 2), dtype=torch.int64, device=self.device)
                       if want_times else None)

    def launch(self, mode: int, wg_size: int = 256, grid: int = 0, stream=None,
               seg_events: bool = False, accumulate: bool = False, waves: int = 0) -> None:
        """One wpm_enumerate call per segment, in order, on `stream`.  With
        seg_events, HIP events bracket each segment's launch on that stream
        (self.seg_events: list of (class, start event, end event)).  With
        accumulate, counts and records add to those of earlier launches."""
        torch = self.torch
        if stream is None:
            stream = torch.cuda.current_stream()
        items = self._items_host
        segs = self._segments or [Segment(None, 0, 0)]
        self.seg_events = []
        for i, sg in enumerate(segs):
            if seg_events:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            cb = self.batch.c_batch if sg.cls is None else self.batch.class_batches[sg.cls]
            n = sg.end - sg.start
            bins = self._seg_bins[i] if self._segments else None
            s = L.Sched(mode=mode, wg_size=wg_size, grid=grid,
                        flags=L.FLAG_ACCUMULATE if (i or accumulate) else 0,
                        d_items=self._items_dev.data_ptr() + 16 * sg.start,
                        h_items=items.ctypes.data + 16 * sg.start if n else None,
                        num_items=n, d_scratch=self.scratch.data_ptr(),
                        d_item_times=(self._times.data_ptr() + 16 * sg.start) if self._times is not None else None,
                        d_bin_offsets=bins.data_ptr() if bins is not None else None,
                        waves_per_simd=waves)
            if mode == L.SCHED_PACKED:
                if bins is None:
                    raise ValueError("packed mode needs per-segment bins")
                s.grid = len(bins) - 1
            st = L.lib().wpm_enumerate(ctypes.byref(cb), ctypes.byref(s), self.surv.data_ptr(),
                                       self.cap, self.counts.data_ptr(), self.total.data_ptr(),
                                       self.stats.data_ptr(), ctypes.c_void_p(stream.cuda_stream))
            L.check("wpm_enumerate", st)
            if seg_events:
                e1.record(stream)
                self.seg_events.append((sg.cls, e0, e1))

    def launch_fetch(self, mode: int, wg_size: int = 256, grid: int = 0, stream=None,
                     parts: int = 4, seg_events: bool = False, waves: int = 0,
                     while_running=None):
        """Sweep and copy the survivor records to pinned host memory, with the
        copies overlapping the sweep: the largest segment is launched in
        `parts` consecutive item ranges, the record-slot counter is snapshot
        on `stream` after every launch (the next launch only reserves slots
        above it, and every wave closes its slot chunk before its launch
        ends), and each finished slot range is copied on a second stream
        while the next launch runs.  Returns a numpy view of all used record
        slots.  With seg_events, self.seg_events holds one (class, start,
        end) event pair per segment, bracketing all of its launches.
        while_running, if given, is called on the host once every launch is
        enqueued, before the copies: host work that overlaps the sweep."""
        torch = self.torch
        if stream is None:
            stream = torch.cuda.current_stream()
        segs = list(self._segments or [Segment(None, 0, 0)])
        if self.records_on_host:
            # the sweep writes the records into host memory itself: one
            # launch per segment, nothing to copy afterwards
            self.launch(mode, wg_size=wg_size, grid=grid, stream=stream, seg_events=seg_events,
                        waves=waves)
            self.launch_end = torch.cuda.Event(enable_timing=True)
            self.launch_end.record(stream)
            if while_running is not None:
                while_running()
            stream.synchronize()
            return self.surv[:min(int(self.total[1].item()), self.cap)].numpy()
        if mode == L.SCHED_PACKED:
            parts = 1
        big = max(range(len(segs)), key=lambda i: segs[i].end - segs[i].start)
        runs = []  # (segment index, start, end)
        for i, sg in enumerate(segs):
            n = sg.end - sg.start
            k = max(1, min(parts, n)) if i == big else 1
            cuts = [sg.start + (n * j) // k for j in range(k + 1)]
            runs += [(i, cuts[j], cuts[j + 1]) for j in range(k)]
        if getattr(self, "_snap", None) is None or self._snap.numel() < len(runs):
            self._snap = torch.zeros(max(8, len(runs)), dtype=torch.int64, device=self.device)
            self._snap_host = torch.zeros(max(8, len(runs)), dtype=torch.int64, pin_memory=True)
        if getattr(self, "_copy_stream", None) is None:
            self._copy_stream = torch.cuda.Stream(device=self.device)
        if getattr(self, "_pinned", None) is None or self._pinned.shape[0] < self.cap:
            self._pinned = torch.empty((max(self.cap, 1), 2), dtype=torch.int64, pin_memory=True)
        items = self._items_host
        ends, starts, self.seg_events = [], {}, []
        for r, (i, a0, a1) in enumerate(runs):
            sg = segs[i]
            if seg_events and i not in starts:
                starts[i] = torch.cuda.Event(enable_timing=True)
                starts[i].record(stream)
            cb = self.batch.c_batch if sg.cls is None else self.batch.class_batches[sg.cls]
            n = a1 - a0
            s = L.Sched(mode=mode, wg_size=wg_size, grid=grid,
                        flags=L.FLAG_ACCUMULATE if r else 0,
                        d_items=self._items_dev.data_ptr() + 16 * a0,
                        h_items=items.ctypes.data + 16 * a0 if n else None,
                        num_items=n, d_scratch=self.scratch.data_ptr(),
                        d_item_times=(self._times.data_ptr() + 16 * a0) if self._times is not None else None,
                        d_bin_offsets=None, waves_per_simd=waves)
            if mode == L.SCHED_PACKED:  # never split: the bins cover the whole segment
                bins = self._seg_bins[i] if self._segments else None
                if bins is None:
                    raise ValueError("packed mode needs per-segment bins")
                s.d_bin_offsets, s.grid = bins.data_ptr(), len(bins) - 1
            st = L.lib().wpm_enumerate(ctypes.byref(cb), ctypes.byref(s), self.surv.data_ptr(),
                                       self.cap, self.counts.data_ptr(), self.total.data_ptr(),
                                       self.stats.data_ptr(), ctypes.c_void_p(stream.cuda_stream))
            L.check("wpm_enumerate", st)
            with torch.cuda.stream(stream):
                self._snap[r:r + 1].copy_(self.total[1:2])
            ev = torch.cuda.Event()
            ev.record(stream)
            ends.append(ev)
            if seg_events and (r + 1 == len(runs) or runs[r + 1][0] != i):
                e1 = torch.cuda.Event(enable_timing=True)
                e1.record(stream)
                self.seg_events.append((sg.cls, starts[i], e1))
        # end of the sweep on `stream` (before the host waits for copies)
        self.launch_end = torch.cuda.Event(enable_timing=True)
        self.launch_end.record(stream)
        if while_running is not None:
            while_running()
        cs = self._copy_stream
        prev = 0
        for r, ev in enumerate(ends):
            cs.wait_event(ev)
            with torch.cuda.stream(cs):
                self._snap_host[r:r + 1].copy_(self._snap[r:r + 1], non_blocking=True)
            cs.synchronize()
            cur = min(int(self._snap_host[r]), self.cap)
            if cur > prev:
                with torch.cuda.stream(cs):
                    self._pinned[prev:cur].copy_(self.surv[prev:cur], non_blocking=True)
                prev = cur
        cs.synchronize()
        return self._pinned[:prev].numpy()

    def fetch_records(self, n: Optional[int] = None):
        """Copy the first n record slots (default: all used slots) into a
        pinned host buffer (allocated once) and return a numpy view of them.
        Unused slots carry the instance ~0 and are kept in the view.  Records
        that already live in host memory are returned as a view, uncopied."""
        torch = self.torch
        if n is None:
            n = int(self.total[1].item())
        n = min(int(n), self.cap)
        if self.records_on_host:
            torch.cuda.current_stream().synchronize()
            return self.surv[:n].numpy()
        if getattr(self, "_pinned", None) is None or self._pinned.shape[0] < n:
            self._pinned = torch.empty((max(n, 1), 2), dtype=torch.int64, pin_memory=True)
        if n:
            self._pinned[:n].copy_(self.surv[:n], non_blocking=True)
        torch.cuda.current_stream().synchronize()
        return self._pinned[:n].numpy()

    def result(self) -> SweepResult:
        self.torch.cuda.synchronize()
        counts = self.counts[:len(self.batch.preps)].cpu().numpy().astype(np.uint64)
        tot = self.total.cpu().numpy()
        if int(tot[2]):
            raise L.WpmError(f"wpm_enumerate skipped {int(tot[2])} malformed items", L.WPM_EINVAL)
        return SweepResult(counts=counts, total=int(tot[0]), slots=int(tot[1]),
                           stats=self.stats.cpu().numpy(),
                           item_times=None if self._times is None else self._times.cpu().numpy(),
                           items=self._items_host)

    def collect(self, stream=None) -> List[List[Tuple[int, ...]]]:
        """Per instance, the canonical list of results (sorted tuples of facet masks)."""
        _, out, offs = self.collect_raw(stream)
        res = []
        for i in range(len(self.batch.preps)):
            a, b = int(offs[i]), int(offs[i + 1])
            lst = []
            w = a
            while w < b:
                ln = int(out[w])
                lst.append(tuple(int(v) for v in out[w + 1:w + 1 + ln]))
                w += 1 + ln
            res.append(lst)
        return res

    def reserve_host_staging(self) -> None:
        """Pinned host memory for `cap` records, which collect_raw then uses
        to bring records from HBM to the host in one DMA copy (a set-up cost,
        like the record buffer itself)."""
        if not self.records_on_host and self._staging is None:
            self._staging = self.torch.empty((max(self.cap, 1), 2), dtype=self.torch.int64,
                                             pin_memory=True)

    def collect_raw(self, stream=None):
        """wpm_collect as flat arrays: (counts, words, offsets[num + 1]).
        Instance i's complexes are words[offsets[i]:offsets[i+1]], each as its
        facet count followed by its facet masks, in canonical order."""
        torch = self.torch
        if stream is None:
            stream = torch.cuda.current_stream()
        preps = self.batch.preps
        hosts = (L.HostInstance * max(1, len(preps)))()
        keep = []
        for i, p in enumerate(preps):
            Bf = np.ascontiguousarray(p.basis.reshape(-1), dtype=np.uint32)
            if Bf.size == 0:
                Bf = np.zeros(1, np.uint32)
            keep.append(Bf)
            off = None
            if p.offset is not None:
                off = np.ascontiguousarray(p.offset, dtype=np.uint32)
                keep.append(off)
            hosts[i] = L.HostInstance(M=len(p.facets), k=p.k, facets=p.facets.ctypes.data,
                                      basis=Bf.ctypes.data,
                                      offset=None if off is None else off.ctypes.data)
        h_counts = np.zeros(max(1, len(preps)), dtype=np.uint64)
        offs = np.zeros(len(preps) + 1, dtype=np.int64)
        words = ctypes.c_int64(0)
        lib = L.lib()
        torch.cuda.current_stream().wait_stream(stream)
        surv = self.surv.data_ptr()
        if not self.records_on_host and self._staging is not None:
            # records in HBM: one copy into the reserved pinned buffer, which
            # wpm_collect then reads in place
            slots = min(int(self.total[1].item()), self.cap)
            with torch.cuda.stream(stream):
                self._staging[:slots].copy_(self.surv[:slots], non_blocking=True)
            stream.synchronize()
            surv = self._staging.data_ptr()
        args = (hosts, len(preps), surv, self.cap, self.counts.data_ptr(),
                self.total.data_ptr(), _ptr(h_counts, L.c_u64p))
        # One call with an output sized by the bound 1 + min(M, facet bound)
        # words per result; pages past the words written are never touched.
        cnt = self.counts[:len(preps)].cpu().numpy().astype(np.int64) if len(preps) else np.zeros(0, np.int64)
        per = np.array([1 + (min(len(p.facets), p.max_facets) if p.max_facets > 0 else len(p.facets))
                        for p in preps], dtype=np.int64)
        bound = int((cnt * per).sum()) if len(preps) else 0
        out = np.empty(max(1, bound), dtype=np.uint32)
        st = lib.wpm_collect(*args, _ptr(out), bound, ctypes.byref(words),
                             _ptr(offs, L.c_i64p), ctypes.c_void_p(stream.cuda_stream))
        L.check("wpm_collect", st, (L.WPM_ECAP, L.WPM_OK))
        if words.value < 0:
            raise L.WpmError("wpm_collect (survivor buffer overflow)", L.WPM_ECAP)
        if st == L.WPM_ECAP:
            raise L.WpmError("wpm_collect (output larger than its bound)", L.WPM_ECAP)
        return h_counts[:len(preps)], out[:words.value], offs


def sweep(preps: Sequence[Prepared], mode: int = L.SCHED_DYNAMIC, cbits: int = 12,
          wg_size: int = 256, grid: int = 0, cap: int = 1 << 20, order: int = 0,
          cost: Optional[np.ndarray] = None, max_items_per_instance: int = 0,
          min_items_per_instance: int = 1, want_sets: bool = True):
    """Convenience: upload, sweep, collect.  Returns (SweepResult, sets or None)."""
    batch = DeviceBatch(preps)
    sw = Sweeper(batch, cap=cap)
    items = build_queue(batch.k, cbits, wg_size, cost=cost,
                        max_items_per_instance=max_items_per_instance, order=order,
                        min_items_per_instance=min_items_per_instance, blocks=batch.blocks)
    sw.set_items(items)
    sw.launch(mode, wg_size=wg_size, grid=grid)
    res = sw.result()
    sets = sw.collect() if want_sets else None
    return res, sets
