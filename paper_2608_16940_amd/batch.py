"""Batched small circuits through libsv's persistent kernel (argument marshalling only)."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _native
from ._native import check, lib

KIND_1Q = 0
KIND_CNOT = 1


def _torch():
    import torch
    return torch


class Batch:
    """A list of (n_qubits, gates) circuits marshalled for sv_batch_run.

    Gates are objects with ``targets`` and ``matrix``: single-qubit gates, or
    CNOT with ``kind == "cnot"`` and targets (control, target).
    """

    def __init__(self, circuits):
        self._keep = []
        arr = (_native.sv_batch_circuit * len(circuits))()
        offsets = np.zeros(len(circuits), dtype=np.int64)
        off = 0
        self.n = []
        for i, (n, gates) in enumerate(circuits):
            kinds = np.zeros(len(gates), dtype=np.int32)
            qubits = np.full(2 * len(gates), -1, dtype=np.int32)
            mats = np.zeros(8 * len(gates), dtype=np.float64)
            for j, g in enumerate(gates):
                if len(g.targets) == 1:
                    kinds[j] = KIND_1Q
                    qubits[2 * j] = g.targets[0]
                    mats[8 * j:8 * j + 8] = np.ascontiguousarray(g.matrix, dtype=np.complex128).reshape(-1).view(np.float64)
                elif getattr(g, "kind", "") == "cnot":
                    kinds[j] = KIND_CNOT
                    qubits[2 * j] = g.targets[0]
                    qubits[2 * j + 1] = g.targets[1]
                else:
                    raise ValueError("batched path takes single-qubit gates and CNOT only")
            self._keep += [kinds, qubits, mats]
            arr[i].n_qubits = int(n)
            arr[i].n_gates = len(gates)
            arr[i].kinds = kinds.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            arr[i].qubits = qubits.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            arr[i].mats = mats.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            offsets[i] = off
            off += 8 << int(n)
            self.n.append(int(n))
        self.arr = arr
        self.count = len(circuits)
        self.offsets = offsets
        self.state_bytes = max(off, 8)

    def records(self, i: int):
        """Host only: the gate records the kernel runs for circuit i (after 1q fusion and slice passes)
        as (int32[m, 4] kind/q0/q1/0, float32[m, 8] 2x2 complex64 matrices)."""
        cap = 3 * max(1, int(self.arr[i].n_gates)) + 2
        rec = np.zeros((cap, 4), dtype=np.int32)
        mats = np.zeros((cap, 8), dtype=np.float32)
        m = ctypes.c_int()
        check(lib().sv_batch_records(ctypes.byref(self.arr[i]), cap, rec.ctypes.data_as(_native._i32p),
                                     mats.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(m)))
        return rec[:m.value], mats[:m.value]

    def allocate(self, device="cuda:0"):
        torch = _torch()
        self.states = torch.empty(self.state_bytes // 8, dtype=torch.complex64, device=device)
        nb = int(lib().sv_batch_workspace_bytes(self.count, self.arr))
        self.ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=device)
        return self

    def _common(self):
        torch = _torch()
        sp = ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream))
        return (ctypes.c_void_p(self.states.data_ptr()), ctypes.c_size_t(self.state_bytes),
                self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), sp)

    def run(self, config=None) -> np.ndarray:
        sd, sb, so, sp = self._common()
        z0 = np.zeros(self.count, dtype=np.float64)
        cfg = None
        if config is not None:
            cfg = np.ascontiguousarray(np.asarray(config, dtype=np.int32))
            assert cfg.size == _native.BATCH_CONFIG_LEN
        check(lib().sv_batch_run(self.count, self.arr, sd, sb, so, z0.ctypes.data_as(_native._dp),
                                 cfg.ctypes.data_as(_native._i32p) if cfg is not None else None,
                                 ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), sp))
        return z0

    def prepare(self, config=None):
        """Pack and upload once; then launch() runs the kernel only."""
        sd, sb, so, sp = self._common()
        self.close_prepared()
        cfg = None
        if config is not None:
            cfg = np.ascontiguousarray(np.asarray(config, dtype=np.int32))
            assert cfg.size == _native.BATCH_CONFIG_LEN
        self._prep = ctypes.c_void_p()
        check(lib().sv_batch_prepare(self.count, self.arr, sb, so,
                                     cfg.ctypes.data_as(_native._i32p) if cfg is not None else None,
                                     ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), sp,
                                     ctypes.byref(self._prep)))
        return self

    def launch(self, want_z0: bool = True):
        sd, sb, so, sp = self._common()
        z0 = np.zeros(self.count, dtype=np.float64) if want_z0 else None
        check(lib().sv_batch_launch(self._prep, sd, z0.ctypes.data_as(_native._dp) if want_z0 else None, sp))
        return z0

    def close_prepared(self):
        if getattr(self, "_prep", None) is not None and self._prep.value:
            lib().sv_batch_prepared_free(self._prep)
        self._prep = None

    def __del__(self):
        try:
            self.close_prepared()
        except Exception:
            pass

    def autotune(self, sample_per_size: int = 32):
        sd, sb, so, sp = self._common()
        cfg = np.zeros(_native.BATCH_CONFIG_LEN, dtype=np.int32)
        times = np.zeros(_native.BATCH_CONFIG_LEN, dtype=np.float64)
        check(lib().sv_batch_autotune(self.count, self.arr, sd, sb, so, int(sample_per_size),
                                      cfg.ctypes.data_as(_native._i32p), times.ctypes.data_as(_native._dp),
                                      ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), sp))
        return cfg, times

    def state(self, i: int) -> np.ndarray:
        o = int(self.offsets[i]) // 8
        return self.states[o:o + (1 << self.n[i])].cpu().numpy().astype(np.complex128)
