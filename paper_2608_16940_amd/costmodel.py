"""Learned sweep-time cost model (argument marshalling and driver loops only).

The network, its training kernels and the planner that uses it live in
libsv (``sv_mlp.h``, ``sv_plan.h``).  The network predicts the log run
time in ms of one sweep scaled to N=30, log(ms) - (N - 30) ln 2: a sweep's
time grows as 2^N once the state leaves the caches, so the model learns the
relative costs of widths and target patterns and extrapolates in N.  This module gathers training data by
timing the library's own fused sweeps on the GPU, trains the network with
the library's HIP forward / backward / Adam kernels, and stores or loads the
trained parameters.
"""
from __future__ import annotations

import ctypes
import json
import math
import os
import time

import numpy as np

from . import _native
from ._native import check, lib

NIN = 12
HID = 64
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "costmodel_weights.json")


def _torch():
    import torch
    return torch


def param_count(nin: int = NIN, hid: int = HID) -> int:
    return int(lib().sv_mlp_param_count(nin, hid))


def features(n: int, targets, diagonal: bool, fraction: float = 1.0, launches: int = 1) -> np.ndarray:
    """Cost-model features of one sweep (sv_cost_features): a diagonal block also carries the
    fraction of the state its sweeps visit and its launch count (diag_sweep_cost)."""
    t = np.ascontiguousarray(np.asarray(targets, dtype=np.int32))
    out = np.zeros(NIN, dtype=np.float32)
    check(lib().sv_cost_features(int(n), int(t.size), t.ctypes.data_as(_native._i32p), 1 if diagonal else 0,
                                 float(fraction), int(launches),
                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return out


def diag_sweep_cost(diag, phys_targets):
    """(fraction of the state visited, launches) of the streaming lowering for a diagonal operator
    whose entry r has bit j at physical position phys_targets[j] (sv_diag_sweep_cost)."""
    d = np.ascontiguousarray(np.asarray(diag, dtype=np.complex128))
    t = np.ascontiguousarray(np.asarray(phys_targets, dtype=np.int32))
    assert d.size == 1 << t.size
    fr = ctypes.c_double()
    ln = ctypes.c_int()
    check(lib().sv_diag_sweep_cost(int(t.size), d.view(np.float64).ctypes.data_as(_native._dp),
                                   t.ctypes.data_as(_native._i32p), ctypes.byref(fr), ctypes.byref(ln)))
    return float(fr.value), int(ln.value)


def block_features(n: int, block, layout=None) -> np.ndarray:
    """Features of a plan block at the physical positions of `layout` (identity if None)."""
    L = list(range(n)) if layout is None else [int(x) for x in layout]
    ph = [L[q] for q in block["targets"]]
    if block["diag"]:
        fr, ln = diag_sweep_cost(np.diag(block["matrix"]), ph)
        return features(n, ph, True, fr, ln)
    return features(n, ph, False)


def init_params(seed: int = 0, nin: int = NIN, hid: int = HID) -> np.ndarray:
    """He-style initialisation in the library's flat parameter order."""
    rng = np.random.default_rng(seed)
    w1 = rng.standard_normal((nin, hid)) * math.sqrt(2.0 / nin)
    w2 = rng.standard_normal((hid, hid)) * math.sqrt(2.0 / hid)
    w3 = rng.standard_normal(hid) * math.sqrt(1.0 / hid)
    p = np.concatenate([w1.reshape(-1), np.zeros(hid), w2.reshape(-1), np.zeros(hid), w3, np.zeros(1)])
    assert p.size == param_count(nin, hid)
    return p.astype(np.float32)


def split_params(p, nin: int = NIN, hid: int = HID):
    """Flat vector -> (W1, b1, W2, b2, W3[hid,1], b3) views, as the oracle's MLP takes them."""
    p = np.asarray(p)
    o = 0
    W1 = p[o:o + nin * hid].reshape(nin, hid); o += nin * hid
    b1 = p[o:o + hid]; o += hid
    W2 = p[o:o + hid * hid].reshape(hid, hid); o += hid * hid
    b2 = p[o:o + hid]; o += hid
    W3 = p[o:o + hid].reshape(hid, 1); o += hid
    b3 = p[o:o + 1]
    return W1, b1, W2, b2, W3, b3


def forward_host(params, X) -> np.ndarray:
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float32))
    y = np.zeros(X.shape[0], dtype=np.float64)
    check(lib().sv_mlp_forward_host(p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), X.shape[1], HID,
                                    X.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), X.shape[0],
                                    y.ctypes.data_as(_native._dp)))
    return y


class DeviceMLP:
    """Parameters, Adam moments and buffers on the GPU; every step runs libsv kernels."""

    def __init__(self, params, batch: int, device: str = "cuda:0", nin: int = NIN, hid: int = HID):
        torch = _torch()
        self.nin, self.hid, self.batch = nin, hid, batch
        self.p = torch.from_numpy(np.asarray(params, dtype=np.float32).copy()).to(device)
        n = self.p.numel()
        self.g = torch.zeros(n, dtype=torch.float32, device=device)
        self.m = torch.zeros(n, dtype=torch.float32, device=device)
        self.v = torch.zeros(n, dtype=torch.float32, device=device)
        self.cache = torch.zeros(int(lib().sv_mlp_cache_floats(hid, batch)), dtype=torch.float32, device=device)
        self.y = torch.zeros(batch, dtype=torch.float32, device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.t = 0

    def _s(self):
        return ctypes.c_void_p(int(_torch().cuda.current_stream().cuda_stream))

    @staticmethod
    def _ptr(t):
        return ctypes.c_void_p(t.data_ptr())

    def forward(self, X):
        B = X.shape[0]
        assert B <= self.batch and X.shape[1] == self.nin and X.is_contiguous()
        check(lib().sv_mlp_forward(self._ptr(self.p), self.nin, self.hid, self._ptr(X), B, self._ptr(self.y),
                                   self._ptr(self.cache), self._s()))
        return self.y[:B]

    def backward(self, X, target):
        B = X.shape[0]
        check(lib().sv_mlp_backward(self._ptr(self.p), self.nin, self.hid, self._ptr(X), self._ptr(target), B,
                                    self._ptr(self.y), self._ptr(self.cache), self._ptr(self.g),
                                    self._ptr(self.loss), self._s()))
        return self.g

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        check(lib().sv_mlp_adam(self._ptr(self.p), self._ptr(self.g), self._ptr(self.m), self._ptr(self.v),
                                self.p.numel(), self.t, ctypes.c_float(lr), ctypes.c_float(beta1),
                                ctypes.c_float(beta2), ctypes.c_float(eps), self._s()))

    def params(self) -> np.ndarray:
        return self.p.detach().cpu().numpy().copy()


def train(X: np.ndarray, y: np.ndarray, steps: int = 3000, lr: float = 3e-3, seed: int = 0, device="cuda:0",
          log_every: int = 0):
    """Full-batch Adam on (X, y) with the library's kernels; returns (params, loss history)."""
    torch = _torch()
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(device)
    yd = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float32)).to(device)
    net = DeviceMLP(init_params(seed), X.shape[0], device)
    hist = []
    for s in range(steps):
        net.forward(Xd)
        net.backward(Xd, yd)
        net.adam(lr=lr)
        if log_every and (s % log_every == 0 or s == steps - 1):
            hist.append((s, float(net.loss.item())))
    net.forward(Xd)
    net.backward(Xd, yd)
    hist.append((steps, float(net.loss.item())))
    return net.params(), hist


# ------------------------------------------------------------------ timing data
def _random_block(rng, n, k, kind):
    """A k-qubit operator of the given structural kind on random targets: dense (Haar-like),
    diag (random phases on every entry), cdiag (random phases only where c >= 1 chosen target
    bits are all set, 1 elsewhere: controlled phases, whose sweeps cover part of the state),
    perm (a phase permutation)."""
    import workloads as W
    pat = rng.integers(0, 5)
    if pat == 4:
        w0 = int(rng.integers(0, n - (k + 3) + 1)) if n >= k + 3 else 0
        t = w0 + rng.choice(min(k + 3, n), size=k, replace=False)
    elif pat == 0:
        t = rng.choice(n, size=k, replace=False)
    elif pat == 1:
        s0 = int(rng.integers(0, n - k + 1))
        t = np.arange(s0, s0 + k)
    elif pat == 2:
        t = np.arange(n - k, n)
    else:
        t = np.arange(0, k)
    t = [int(x) for x in rng.permutation(t)]
    d = 1 << k
    if kind == "dense":
        m = W.random_dense(n, k, rng, targets=t).matrix
    else:
        ph = np.exp(1j * rng.uniform(0, 2 * np.pi, d))
        if kind == "cdiag":
            c = int(rng.integers(1, k + 1))
            ctl = rng.choice(k, size=c, replace=False)
            cmask = int(sum(1 << int(j) for j in ctl))
            ph = np.where((np.arange(d) & cmask) == cmask, ph, 1.0 + 0j)
        m = np.diag(ph)
        if kind == "perm":
            m = m[rng.permutation(d)]
    return t, np.ascontiguousarray(m, dtype=np.complex128), kind in ("diag", "cdiag")


def collect(n_values, samples_per_n, seed: int = 0, reps: int = 3, device="cuda:0", log=None):
    """Time the library's own fused sweeps on random blocks.

    Returns (X[m, NIN] float32, log_ms[m] float64, rows) where rows keeps
    (n, k, targets, kind, ms) for inspection.
    """
    import torch

    from . import StateVector
    rng = np.random.default_rng(seed)
    Xs, ys, rows = [], [], []
    for n, cnt in zip(n_values, samples_per_n):
        sv = StateVector(int(n), device=device)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        for _ in range(int(cnt)):
            k = int(rng.choice([1, 2, 3, 4, 5, 6, 7], p=[0.08, 0.12, 0.14, 0.2, 0.24, 0.12, 0.1]))
            kind = str(rng.choice(["dense", "diag", "cdiag", "perm"], p=[0.6, 0.12, 0.18, 0.1]))
            t, m, is_diag = _random_block(rng, int(n), k, kind)
            sv.apply(m, t)
            times = []
            for _ in range(reps):
                s0 = sv.stats()
                e0.record()
                sv.apply(m, t)
                e1.record()
                e1.synchronize()
                times.append(e0.elapsed_time(e1))
                s1 = sv.stats()
            ms = float(np.median(times))
            # features use the physical targets at the time of the sweep, and for a
            # diagonal block the fraction of the state its sweeps visited and its launches
            L = sv.layout()
            phys = [int(L[q]) for q in t]
            if is_diag:
                frac = (s1["diag_chunks"] - s0["diag_chunks"]) / float(1 << (int(n) - 1))
                launches = int(s1["launches"] - s0["launches"])
                Xs.append(features(int(n), phys, True, frac, launches))
            else:
                frac, launches = 1.0, 1
                Xs.append(features(int(n), phys, False))
            ys.append(math.log(ms) - (int(n) - 30) * math.log(2.0))
            rows.append((int(n), k, phys, kind, ms, frac, launches))
        if log:
            log("collect n=%d samples=%d %.1f s" % (n, cnt, time.perf_counter() - t0))
        sv.close()
        del sv
        torch.cuda.empty_cache()
    return np.stack(Xs), np.array(ys), rows


def save(params, path=WEIGHTS, meta=None):
    with open(path, "w") as f:
        json.dump({"nin": NIN, "hid": HID, "params": [float(x) for x in np.asarray(params, dtype=np.float32)],
                   "meta": meta or {}}, f)


def load(path=WEIGHTS):
    with open(path) as f:
        d = json.load(f)
    assert d["nin"] == NIN and d["hid"] == HID
    return np.asarray(d["params"], dtype=np.float32), d.get("meta", {})


# ------------------------------------------------------------------ command line
DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "costmodel_data.csv")
FIT_N = [24, 25, 26, 27, 28, 29, 30, 31, 32, 33]
FIT_SAMPLES = [250, 250, 250, 300, 300, 250, 220, 160, 100, 60]


FIT_REPS = 5  # timed sweeps per row (the median is the row's time)


def fit(seed: int = 0, steps: int = 4000, log=print, weights=WEIGHTS, data=DATA):
    """Collect sweep timings at N=24..33, hold out every fifth row, train, save."""
    X, y, rows = collect(FIT_N, FIT_SAMPLES, seed=seed, reps=FIT_REPS, log=log)
    test = np.arange(len(y)) % 5 == 0
    t0 = time.perf_counter()
    params, hist = train(X[~test], y[~test], steps=steps, seed=seed, log_every=500)
    tt = time.perf_counter() - t0
    pred = forward_host(params, X)
    rmse_tr = float(np.sqrt(np.mean((pred[~test] - y[~test]) ** 2)))
    rmse_te = float(np.sqrt(np.mean((pred[test] - y[test]) ** 2)))
    meta = {"holdout": "every fifth row", "n_values": FIT_N, "samples": FIT_SAMPLES, "rows": int(len(y)),
            "reps_per_row": FIT_REPS, "timed_sweeps": int(len(y)) * FIT_REPS,
            "train_steps": steps, "train_seconds": tt, "rmse_log_ms_train": rmse_tr, "rmse_log_ms_test": rmse_te,
            "loss_history": hist}
    save(params, path=weights, meta=meta)
    kinds = {"dense": 0, "diag": 1, "perm": 2, "cdiag": 3}
    with open(data, "w") as f:
        f.write(",".join(["f%d" % i for i in range(NIN)] + ["log_ms_at_n30", "n", "k", "kind"]) + "\n")
        for xi, yi, r in zip(X, y, rows):
            f.write(",".join("%.7g" % v for v in xi) + ",%.7g,%d,%d,%d\n" % (yi, r[0], r[1], kinds[r[3]]))
    log("fit: rows %d, train RMSE %.3f, held-out RMSE %.3f (log ms), %.1f s training"
        % (len(y), rmse_tr, rmse_te, tt))
    return params, meta


if __name__ == "__main__":
    import sys
    if len(sys.argv) > 1 and sys.argv[1] == "fit":
        # optional output paths: fit WEIGHTS_JSON DATA_CSV
        w = sys.argv[2] if len(sys.argv) > 2 else WEIGHTS
        d = sys.argv[3] if len(sys.argv) > 3 else DATA
        fit(log=lambda *a: print(*a, flush=True), weights=w, data=d)
    else:
        print("usage: python -m paper_2608_16940_amd.costmodel fit [WEIGHTS_JSON DATA_CSV]")
