"""Learned cost model of the persistent scheduler (driver over the HIP kernels).

The model maps the 16 packing features of an instance to [ln(ns of sweep time
per kernel vector), log10(survivor density)].  Training labels come from the
engine itself: per-item start/end stamps of a persistent sweep give each
instance's measured workgroup time, and the exact counts give its density.
Forward, backward and the Adam step run in libwpm.so (mlp.hip); this module
only moves tensors and loops over epochs.

The model never changes a result: it orders and sizes work items, and the
static round-robin schedule is used whenever no trained model is available.
"""
from __future__ import annotations

import ctypes
import json
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from . import _lib as L


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((L.MLP_IN, L.MLP_HIDDEN), (L.MLP_HIDDEN, L.MLP_HIDDEN),
                            (L.MLP_HIDDEN, L.MLP_OUT)):
        lim = np.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, size=(fan_out, fan_in)).reshape(-1))
        parts.append(np.zeros(fan_out))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == L.MLP_PARAMS
    return p


def make_norm(X: np.ndarray, T: np.ndarray) -> np.ndarray:
    sx = X.std(0)
    sx = np.where(sx > 1e-6, sx, 1.0)
    sy = T.std(0)
    sy = np.where(sy > 1e-6, sy, 1.0)
    return np.concatenate([X.mean(0), sx, T.mean(0), sy]).astype(np.float32)


def features_of(preps) -> np.ndarray:
    return np.array([list(p.info.features) for p in preps], dtype=np.float32)


class CostModel:
    def __init__(self, params: Optional[np.ndarray] = None, norm: Optional[np.ndarray] = None,
                 device="cuda", seed: int = 0):
        import torch
        self.torch = torch
        self.device = device
        p = init_params(seed) if params is None else np.asarray(params, np.float32)
        n = np.concatenate([np.zeros(16), np.ones(16), np.zeros(2), np.ones(2)]).astype(np.float32) \
            if norm is None else np.asarray(norm, np.float32)
        self.params = torch.from_numpy(p.copy()).to(device)
        self.norm = torch.from_numpy(n.copy()).to(device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self.trained = params is not None

    # ------------------------------------------------------------- kernels
    def predict(self, X: np.ndarray, stream=None) -> np.ndarray:
        """Model outputs for features X, computed on `stream` (default: the
        current stream); the copies run on that stream too, so a side stream
        lets the inference overlap work queued on the others."""
        torch = self.torch
        st = stream or torch.cuda.current_stream()
        with torch.cuda.stream(st):
            Xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(self.device)
            Y = torch.empty((len(X), L.MLP_OUT), dtype=torch.float32, device=self.device)
            L.check("wpm_mlp_forward", L.lib().wpm_mlp_forward(
                _vp(self.params), _vp(self.norm), _vp(Xd), len(X), _vp(Y), ctypes.c_void_p(st.cuda_stream)))
            out = Y.cpu().numpy()
        return out

    def grad(self, Xd, Td, work, gbuf, loss, stream=None):
        torch = self.torch
        st = stream or torch.cuda.current_stream()
        L.check("wpm_mlp_grad", L.lib().wpm_mlp_grad(
            _vp(self.params), _vp(self.norm), _vp(Xd), _vp(Td), Xd.shape[0], _vp(gbuf), _vp(work),
            _vp(loss) if loss is not None else None, ctypes.c_void_p(st.cuda_stream)))

    def adam(self, gbuf, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0, stream=None):
        torch = self.torch
        st = stream or torch.cuda.current_stream()
        self.step += 1
        L.check("wpm_mlp_adam", L.lib().wpm_mlp_adam(
            _vp(self.params), _vp(gbuf), _vp(self.m), _vp(self.v), self.step, lr, beta1, beta2, eps,
            weight_decay, ctypes.c_void_p(st.cuda_stream)))

    # ------------------------------------------------------------- training
    def fit(self, X: np.ndarray, T: np.ndarray, epochs: int = 400, lr: float = 3e-3,
            batch: int = 1024, weight_decay: float = 1e-4, seed: int = 0, log_every: int = 0):
        """Mini-batch Adam on the GPU; sets the normalisation from the data."""
        torch = self.torch
        ok = np.isfinite(T).all(1)
        X = np.ascontiguousarray(X[ok], np.float32)
        T = np.ascontiguousarray(T[ok], np.float32)
        self.norm = torch.from_numpy(make_norm(X, T)).to(self.device)
        Xd = torch.from_numpy(X).to(self.device)
        Td = torch.from_numpy(T).to(self.device)
        n = len(X)
        bs = min(batch, n)
        work = torch.empty(int(L.lib().wpm_mlp_work_floats(bs)), dtype=torch.float32, device=self.device)
        gbuf = torch.empty(L.MLP_PARAMS, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        rng = np.random.default_rng(seed)
        hist = []
        for ep in range(epochs):
            perm = torch.from_numpy(rng.permutation(n)).to(self.device)
            tot = 0.0
            nb = 0
            for s in range(0, n - bs + 1, bs):
                idx = perm[s:s + bs]
                xb = Xd.index_select(0, idx).contiguous()
                tb = Td.index_select(0, idx).contiguous()
                self.grad(xb, tb, work, gbuf, loss)
                self.adam(gbuf, lr, weight_decay=weight_decay)
                if log_every and ep % log_every == 0:
                    tot += float(loss.item())
                    nb += 1
            if log_every and ep % log_every == 0:
                hist.append((ep, tot / max(nb, 1)))
        self.trained = True
        return hist

    def loss(self, X: np.ndarray, T: np.ndarray) -> float:
        torch = self.torch
        Xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(self.device)
        Td = torch.from_numpy(np.ascontiguousarray(T, np.float32)).to(self.device)
        work = torch.empty(int(L.lib().wpm_mlp_work_floats(len(X))), dtype=torch.float32, device=self.device)
        gbuf = torch.empty(L.MLP_PARAMS, dtype=torch.float32, device=self.device)
        out = torch.empty(1, dtype=torch.float32, device=self.device)
        self.grad(Xd, Td, work, gbuf, out)
        return float(out.item())

    # ------------------------------------------------------------- persistence
    def state(self) -> dict:
        return {"params": self.params.cpu().numpy().tolist(), "norm": self.norm.cpu().numpy().tolist()}

    def save(self, path: str) -> None:
        with open(path, "w") as f:
            json.dump(self.state(), f)

    @classmethod
    def load(cls, path: str, device="cuda") -> "CostModel":
        with open(path) as f:
            d = json.load(f)
        return cls(np.array(d["params"], np.float32), np.array(d["norm"], np.float32), device=device)


# ---------------------------------------------------------------- labels

def labels_from_sweep(preps: Sequence, res, clock_khz: float) -> np.ndarray:
    """[ln(ns per vector), log10(density)] per instance from a timed sweep:
    the sum over an instance's items of (end - start) stamps, converted with
    the stamp clock rate, divided by its 2^k vectors.  Instances that were not
    swept (k = 0: no items) get NaN labels."""
    items, times = res.items, res.item_times
    ns = np.zeros(len(preps))
    swept = np.zeros(len(preps), dtype=bool)
    dur = (times[:len(items), 1] - times[:len(items), 0]).astype(np.float64) * (1e6 / clock_khz)
    inst = items["instance"].astype(np.int64)
    np.add.at(ns, inst, dur)
    swept[inst] = True
    vec = np.array([float(1 << p.k) for p in preps])
    dens = res.counts.astype(np.float64) / vec
    lab = np.stack([np.log(np.maximum(ns / vec, 1e-6)), np.log10(np.maximum(dens, 1e-9))], 1)
    lab[~swept] = np.nan      # not swept (k = 0): no measurement
    return lab.astype(np.float32)
