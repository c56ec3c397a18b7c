"""MI355X (gfx950) state-vector engine for ordered fused k-qubit gates.

The compute path is the HIP library ``libsv.so`` (C-ABI in ``include/sv.h``);
this package only marshals arguments.  PyTorch supplies device memory and the
stream.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _native
from ._native import SvError, check, lib  # noqa: F401

__all__ = ["StateVector", "DensityMatrix", "sample_probs", "sample_probs_noalloc", "workspace_bytes", "SvError"]


def _torch():
    import torch
    return torch


def workspace_bytes(n: int) -> int:
    return int(lib().sv_workspace_bytes(int(n)))


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream)), stream


class StateVector:
    """An n-qubit complex64 state in caller-owned (PyTorch) device memory.

    ``amps`` holds the amplitudes in PHYSICAL order; ``layout()`` returns the
    logical-to-physical map L (physical bit of logical qubit q).
    """

    def __init__(self, n: int, device: str = "cuda:0", stream=None):
        torch = _torch()
        self.n = int(n)
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.amps = torch.empty(1 << self.n, dtype=torch.complex64, device=self.device)
            self.ws = torch.empty(workspace_bytes(self.n), dtype=torch.uint8, device=self.device)
            sp, self.stream = _stream_ptr(stream)
        self._h = ctypes.c_void_p()
        check(lib().sv_alloc(ctypes.byref(self._h), self.n, ctypes.c_void_p(self.amps.data_ptr()),
                             self.amps.numel() * 8, ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), sp))

    # ------------------------------------------------------------ lifetime
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sv_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------ operations
    def reset(self):
        check(lib().sv_reset(self._h))

    def apply(self, matrix, targets):
        m = np.ascontiguousarray(np.asarray(matrix, dtype=np.complex128))
        t = np.ascontiguousarray(np.asarray(targets, dtype=np.int32))
        check(lib().sv_apply_fused(self._h, m.ctypes.data_as(_native._dp), t.ctypes.data_as(_native._i32p),
                                   int(t.size)))

    def apply_gates(self, gates):
        for g in gates:
            self.apply(g.matrix, g.targets)

    def permute_layout(self, layout):
        L = np.ascontiguousarray(np.asarray(layout, dtype=np.int32))
        check(lib().sv_permute_layout(self._h, L.ctypes.data_as(_native._i32p)))

    def canonicalize(self):
        self.permute_layout(np.arange(self.n))

    def layout(self) -> np.ndarray:
        L = np.empty(self.n, dtype=np.int32)
        check(lib().sv_get_layout(self._h, L.ctypes.data_as(_native._i32p)))
        return L

    def probs(self, logical: bool = True):
        torch = _torch()
        out = torch.empty(1 << self.n, dtype=torch.float64, device=self.device)
        check(lib().sv_probs(self._h, ctypes.c_void_p(out.data_ptr()), 1 if logical else 0))
        return out

    def norm(self) -> float:
        v = ctypes.c_double()
        check(lib().sv_norm(self._h, ctypes.byref(v)))
        return v.value

    def sample(self, seed: int, shots: int) -> np.ndarray:
        out = np.empty(int(shots), dtype=np.uint64)
        check(lib().sv_sample(self._h, ctypes.c_uint64(seed & (2**64 - 1)), int(shots),
                              out.ctypes.data_as(_native._u64p)))
        return out

    def sync(self):
        check(lib().sv_sync(self._h))

    def set_option(self, key: int, value: int):
        check(lib().sv_set_option(self._h, int(key), int(value)))

    def get_option(self, key: int) -> int:
        v = ctypes.c_int()
        check(lib().sv_get_option(self._h, int(key), ctypes.byref(v)))
        return v.value

    def set_variant(self, name: str):
        self.set_option(_native.OPT_VARIANT, _native.VARIANT[name])

    def set_precision(self, name: str):
        self.set_option(_native.OPT_PRECISION, _native.PRECISION[name])

    def stats(self) -> dict:
        s = _native.sv_stats()
        check(lib().sv_get_stats(self._h, ctypes.byref(s)))
        return {"gate_sweeps": s.gate_sweeps, "swap_half_sweeps": s.swap_half_sweeps, "relabels": s.relabels,
                "launches": s.launches, "by_variant": list(s.by_variant), "permute_sweeps": s.permute_sweeps,
                "layout_only": s.layout_only, "diag_chunks": s.diag_chunks}

    def set_relabel(self, on: bool, low_bits: int = 12, policy: str = "belady"):
        self.set_option(_native.OPT_LAZY_RELABEL, 1 if on else 0)
        self.set_option(_native.OPT_LOW_BITS, int(low_bits))
        self.set_option(_native.OPT_POLICY, _native.POLICY[policy])

    def hint_next_use(self, next_use):
        a = np.ascontiguousarray(np.asarray(next_use, dtype=np.int64))
        check(lib().sv_hint_next_use(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))

    def copy_out(self, logical: bool = True) -> np.ndarray:
        """Host complex64 copy of the state (sv_copy_out): logical basis order, or physical order."""
        out = np.empty(1 << self.n, dtype=np.complex64)
        check(lib().sv_copy_out(self._h, out.ctypes.data_as(ctypes.c_void_p), 1 if logical else 0))
        return out

    def physical_state(self) -> np.ndarray:
        """Host copy of the stored amplitudes (physical order), complex128."""
        self.sync()
        return self.amps.detach().cpu().numpy().astype(np.complex128)


def sample_probs(probs_dev, seed: int, shots: int, stream=None) -> np.ndarray:
    """Sample indices of a device FP64 probability tensor of length 2^n."""
    torch = _torch()
    n = int(probs_dev.numel()).bit_length() - 1
    assert probs_dev.numel() == 1 << n and probs_dev.dtype == torch.float64 and probs_dev.is_cuda
    ws = torch.empty(workspace_bytes(n), dtype=torch.uint8, device=probs_dev.device)
    sp, _ = _stream_ptr(stream)
    out = np.empty(int(shots), dtype=np.uint64)
    check(lib().sv_sample_probs(ctypes.c_void_p(probs_dev.data_ptr()), n, ctypes.c_uint64(seed & (2**64 - 1)),
                                int(shots), out.ctypes.data_as(_native._u64p), ctypes.c_void_p(ws.data_ptr()),
                                ws.numel(), sp))
    return out


def sample_probs_noalloc(probs_dev, seed: int, shots: int, stream=None) -> np.ndarray:
    """sample_probs without a workspace: the library's fixed per-GPU scratch array
    (n <= 26; concurrent calls on one GPU race and must be serialised)."""
    torch = _torch()
    n = int(probs_dev.numel()).bit_length() - 1
    assert probs_dev.numel() == 1 << n and probs_dev.dtype == torch.float64 and probs_dev.is_cuda
    sp, _ = _stream_ptr(stream)
    out = np.empty(int(shots), dtype=np.uint64)
    check(lib().sv_sample_probs_noalloc(ctypes.c_void_p(probs_dev.data_ptr()), n,
                                        ctypes.c_uint64(seed & (2**64 - 1)), int(shots),
                                        out.ctypes.data_as(_native._u64p), sp))
    return out


def policy_simulate(n: int, frames: int, tuples, policy: str = "belady") -> int:
    """Promotions made by a victim policy in the all-frame demand model (host only)."""
    ks = np.array([len(t) for t in tuples], dtype=np.int32)
    tg = np.array([q for t in tuples for q in t], dtype=np.int32)
    out = ctypes.c_int64()
    check(lib().sv_policy_simulate(int(n), int(frames), _native.POLICY[policy], len(tuples),
                                   ks.ctypes.data_as(_native._i32p), tg.ctypes.data_as(_native._i32p),
                                   ctypes.byref(out)))
    return int(out.value)


class Plan:
    """Fused blocks produced by a planner in libsv (host object)."""

    def __init__(self, handle: ctypes.c_void_p, n: int):
        self._h = handle
        self.n = n

    @staticmethod
    def _flat(gates):
        ks = np.array([len(g.targets) for g in gates], dtype=np.int32)
        tg = np.array([t for g in gates for t in g.targets], dtype=np.int32)
        mats = (np.concatenate([np.ascontiguousarray(g.matrix, dtype=np.complex128).reshape(-1) for g in gates])
                .view(np.float64) if gates else np.zeros(0))
        dg = np.array([1 if getattr(g, "diag", False) else 0 for g in gates], dtype=np.int8)
        return ks, tg, mats, dg

    @classmethod
    def greedy(cls, n: int, gates, k_max: int = 5) -> "Plan":
        ks, tg, mats, dg = cls._flat(gates)
        h = ctypes.c_void_p()
        check(lib().sv_plan_greedy(int(n), len(gates), ks.ctypes.data_as(_native._i32p),
                                   tg.ctypes.data_as(_native._i32p), mats.ctypes.data_as(_native._dp),
                                   dg.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), int(k_max), ctypes.byref(h)))
        return cls(h, int(n))

    @classmethod
    def dp(cls, n: int, gates, k_max: int = 5, diag_max: int = 6, window: int = 64, params=None,
           nin: int = 12, hid: int = 64, reorder: bool = False, search_cap: bool = False,
           repeat: bool = False, score: str = None) -> "Plan":
        """Windowed DP fusion on a block score: "paper" (4^k / 1), "learned" (the MLP's predicted
        sweep time; params) or "roofline" (the analytic sweep time at MI355X's peaks); the default
        is learned when params are given, else paper.  reorder=True first applies the
        commute-aware reorder; search_cap=True lets a time score pick the dense width cap
        (4..k_max); repeat=True reruns reorder-and-fuse on the blocks, at most four rounds in all."""
        ks, tg, mats, dg = cls._flat(gates)
        h = ctypes.c_void_p()
        if score is None:
            score = "paper" if params is None else "learned"
        pp = None
        if score == "learned":
            params = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
            pp = params.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        check(lib().sv_plan_dp(int(n), len(gates), ks.ctypes.data_as(_native._i32p),
                               tg.ctypes.data_as(_native._i32p), mats.ctypes.data_as(_native._dp),
                               dg.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), int(k_max), int(diag_max),
                               int(window), _native.SCORE[score], pp, int(nin), int(hid),
                               (1 if reorder else 0) | (2 if search_cap else 0) | (4 if repeat else 0),
                               ctypes.byref(h)))
        return cls(h, int(n))

    @classmethod
    def paper(cls, n: int, gates, k_max: int = 6, diag_max: int = 6, window: int = 64) -> "Plan":
        """The paper's pipeline (Section IV-C): commute-aware reorder, windowed DP on the 4^k / 1
        score, cross-window merge, repeated up to four rounds; caps as the paper's GPU runs use."""
        return cls.dp(n, gates, k_max=k_max, diag_max=diag_max, window=window, reorder=True, repeat=True)

    @classmethod
    def learned(cls, n: int, gates, params, k_max: int = 7, window: int = 64, swaps: bool = True,
                horizon: int = 32, margin: float = 0.25) -> "Plan":
        """The learned planner: the same pipeline on predicted sweep times, dense cap chosen by the model,
        then (swaps=True) layout swaps where the model predicts they pay (sv_plan_swaps)."""
        plan = cls.dp(n, gates, k_max=k_max, diag_max=k_max, window=window, params=params, reorder=True,
                      search_cap=True, repeat=True)
        if swaps:
            plan.swaps_inserted = plan.add_swaps(params, horizon, margin)
        return plan

    @classmethod
    def roofline(cls, n: int, gates, k_max: int = 7, window: int = 64) -> "Plan":
        """The learned planner's pipeline with the analytic score instead of the network (the
        ablation of the cost model): reorder, DP with the cap search, cross-window merge, four rounds."""
        return cls.dp(n, gates, k_max=k_max, diag_max=k_max, window=window, reorder=True, search_cap=True,
                      repeat=True, score="roofline")

    def add_swaps(self, params, horizon: int = 32, margin: float = 0.25, nin: int = 12, hid: int = 64) -> int:
        """Insert layout-swap blocks where the cost model predicts a net gain; returns how many."""
        params = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        out = ctypes.c_int()
        check(lib().sv_plan_swaps(self._h, params.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), int(nin),
                                  int(hid), int(horizon), float(margin), ctypes.byref(out)))
        return out.value

    def __len__(self) -> int:
        v = ctypes.c_int()
        check(lib().sv_plan_num_blocks(self._h, ctypes.byref(v)))
        return v.value

    def block(self, i: int):
        """A fused block {k, targets, n_gates, diag, matrix}, or a layout-swap block
        {k, targets, swap: True, dest} (logical targets[j] moves to physical bit dest[j])."""
        k = ctypes.c_int()
        ng = ctypes.c_int()
        dg = ctypes.c_int()
        t = np.zeros(64, dtype=np.int32)
        check(lib().sv_plan_block_info(self._h, int(i), ctypes.byref(k), t.ctypes.data_as(_native._i32p),
                                       ctypes.byref(ng), ctypes.byref(dg)))
        sw = ctypes.c_int()
        dest = np.zeros(64, dtype=np.int32)
        check(lib().sv_plan_block_swap(self._h, int(i), ctypes.byref(sw), dest.ctypes.data_as(_native._i32p)))
        if sw.value:
            return {"k": k.value, "targets": tuple(int(x) for x in t[:k.value]), "swap": True,
                    "dest": tuple(int(x) for x in dest[:k.value]), "n_gates": 0, "diag": False}
        m = np.empty((1 << k.value, 1 << k.value), dtype=np.complex128)
        check(lib().sv_plan_block_matrix(self._h, int(i), m.view(np.float64).ctypes.data_as(_native._dp)))
        return {"k": k.value, "targets": tuple(int(x) for x in t[:k.value]), "n_gates": ng.value,
                "diag": bool(dg.value), "matrix": m}

    def blocks(self):
        return [self.block(i) for i in range(len(self))]

    def run(self, sv: "StateVector"):
        check(lib().sv_run_plan(sv._h, self._h))

    def bind(self, sv: "StateVector") -> "BoundPlan":
        """Lower every block once for ``sv`` (its layout, options, precision) with operands in device memory."""
        return BoundPlan(self, sv)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sv_plan_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BoundPlan:
    """A plan bound to one state: runs are kernel launches only, and can replay as one HIP graph."""

    def __init__(self, plan: Plan, sv: StateVector):
        import torch
        need = ctypes.c_size_t()
        check(lib().sv_bound_bytes(sv._h, plan._h, ctypes.byref(need)))
        self.sv = sv
        self.ops = torch.empty(max(int(need.value), 256), dtype=torch.uint8, device=sv.amps.device)
        self._h = ctypes.c_void_p()
        check(lib().sv_plan_bind(sv._h, plan._h, ctypes.c_void_p(self.ops.data_ptr()), int(self.ops.numel()),
                                 ctypes.byref(self._h)))

    def run(self):
        check(lib().sv_bound_run(self._h))

    def run_graph(self):
        check(lib().sv_bound_graph_run(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sv_bound_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


from .density import DensityMatrix, SuperGate, superop, superop_gates  # noqa: E402,F401
