"""Density matrices on the fused-operator path (argument marshalling only).

An N-qubit density matrix is a 2N-qubit complex64 state holding vec(rho)
column by column (index row + 2^N column, Section IV-B); channels are
applied by ``libsv`` as 2k-target superoperators through the same kernels,
layout map and planners as state vectors (C-ABI in ``include/sv_density.h``).
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import List, Sequence, Tuple

import numpy as np

from . import StateVector, _native, _stream_ptr, _torch
from ._native import check, lib


def _kraus_array(kraus) -> np.ndarray:
    ks = np.ascontiguousarray(np.stack([np.asarray(e, dtype=np.complex128) for e in kraus]))
    d = ks.shape[1]
    if ks.ndim != 3 or ks.shape[2] != d or d & (d - 1):
        raise ValueError("Kraus operators must be square 2^k x 2^k matrices")
    return ks


def superop(kraus) -> np.ndarray:
    """sum_i conj(E_i) (x) E_i (4^k x 4^k, complex128), built by libsv."""
    ks = _kraus_array(kraus)
    k = int(ks.shape[1]).bit_length() - 1
    out = np.empty((1 << (2 * k), 1 << (2 * k)), dtype=np.complex128)
    check(lib().sv_dm_superop(ks.view(np.float64).ctypes.data_as(_native._dp), int(ks.shape[0]), k,
                              out.view(np.float64).ctypes.data_as(_native._dp)))
    return out


@dataclasses.dataclass
class SuperGate:
    """A channel as a gate on the 2N vector qubits, for the planners."""
    kind: str
    targets: Tuple[int, ...]
    matrix: np.ndarray
    diag: bool = False


def superop_gates(n: int, channels) -> List[SuperGate]:
    """Channels (objects with .kraus, .targets) as 2k-target gates on vec(rho) of n qubits."""
    out = []
    for ch in channels:
        t = tuple(int(q) for q in ch.targets)
        diag = all(np.count_nonzero(e - np.diag(np.diag(e))) == 0 for e in ch.kraus)
        out.append(SuperGate(getattr(ch, "kind", "channel"), t + tuple(q + n for q in t), superop(ch.kraus), diag))
    return out


class DensityMatrix(StateVector):
    """An n-qubit density matrix in caller-owned (PyTorch) device memory.

    ``amps`` holds vec(rho) in PHYSICAL order over 2n vector qubits;
    ``layout()`` is the map of those 2n qubits.  Every StateVector call applies
    to the vector (``apply`` takes a raw operator on vector qubits, ``norm``
    is sum |rho_ij|^2); ``probs``, ``sample`` and ``trace`` read the diagonal.
    """

    def __init__(self, n: int, device: str = "cuda:0", stream=None):
        torch = _torch()
        self.rows = int(n)
        self.n = 2 * self.rows
        self.device = torch.device(device)
        nbytes = int(lib().sv_dm_state_bytes(self.rows))
        wbytes = int(lib().sv_dm_workspace_bytes(self.rows))
        if nbytes == 0 or wbytes == 0:
            raise ValueError("density-matrix qubit count out of range [2, 17]")
        with torch.cuda.device(self.device):
            self.amps = torch.empty(nbytes // 8, dtype=torch.complex64, device=self.device)
            self.ws = torch.empty(wbytes, dtype=torch.uint8, device=self.device)
            sp, self.stream = _stream_ptr(stream)
        self._h = ctypes.c_void_p()
        check(lib().sv_dm_alloc(ctypes.byref(self._h), self.rows, ctypes.c_void_p(self.amps.data_ptr()), nbytes,
                                ctypes.c_void_p(self.ws.data_ptr()), wbytes, sp))

    def apply_channel(self, kraus, targets: Sequence[int]):
        ks = _kraus_array(kraus)
        t = np.ascontiguousarray(np.asarray(targets, dtype=np.int32))
        check(lib().sv_dm_apply_channel(self._h, ks.view(np.float64).ctypes.data_as(_native._dp), int(ks.shape[0]),
                                        t.ctypes.data_as(_native._i32p), int(t.size)))

    def apply_unitary(self, u, targets: Sequence[int]):
        self.apply_channel([u], targets)

    def apply_channels(self, channels):
        for ch in channels:
            self.apply_channel(ch.kraus, ch.targets)

    def probs(self, logical: bool = True):
        """Re rho_xx (FP64, device) by logical basis index x."""
        torch = _torch()
        out = torch.empty(1 << self.rows, dtype=torch.float64, device=self.device)
        check(lib().sv_dm_probs(self._h, ctypes.c_void_p(out.data_ptr())))
        return out

    def trace(self) -> float:
        v = ctypes.c_double()
        check(lib().sv_dm_trace(self._h, ctypes.byref(v)))
        return v.value

    def purity(self) -> float:
        return self.norm()

    def sample(self, seed: int, shots: int) -> np.ndarray:
        torch = _torch()
        scratch = torch.empty(1 << self.rows, dtype=torch.float64, device=self.device)
        out = np.empty(int(shots), dtype=np.uint64)
        check(lib().sv_dm_sample(self._h, ctypes.c_uint64(seed & (2**64 - 1)), int(shots),
                                 out.ctypes.data_as(_native._u64p), ctypes.c_void_p(scratch.data_ptr())))
        return out

    def matrix(self):
        """rho[row, column] as a device complex64 view, after moving the layout to identity."""
        self.canonicalize()
        d = 1 << self.rows
        return self.amps.view(d, d).transpose(0, 1)
