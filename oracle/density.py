"""Density-matrix reference.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: imported by
``tests/``, ``__graft_entry__.smoke`` and the bench's CPU legs, never by the
product package, and sharing no code with the HIP path.

What it computes (Section IV-B, the vectorised density matrix): an N-qubit
density matrix rho, initially |0..0><0..0|, goes through channels; a channel
with Kraus operators E_i on the ordered targets V maps rho to
sum_i E_i rho E_i^dagger, each E_i acting on V with the little-endian target
convention of Section II.  The oracle applies exactly that definition with
dense 2^N x 2^N complex128 matrices: every E_i is embedded into the full
space column by column with the state-vector oracle's gate application
(``apply_gate`` on basis vectors), and the sum is formed with plain matrix
products.  No vectorisation, superoperator or fusion is used here, so the
paper's vectorised form is checked against it rather than built into it.

``vec`` is the column-major stacking the paper fixes: vector index
row + 2^N * column, so the lower N bits select the row.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from . import apply_gate


def zero(n: int) -> np.ndarray:
    rho = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    rho[0, 0] = 1.0
    return rho


def embed(op: np.ndarray, targets: Sequence[int], n: int) -> np.ndarray:
    """The 2^N x 2^N matrix of a k-qubit operator on ordered ``targets``."""
    d = 1 << n
    full = np.empty((d, d), dtype=np.complex128)
    for c in range(d):
        col = np.zeros(d, dtype=np.complex128)
        col[c] = 1.0
        apply_gate(col, op, list(targets))
        full[:, c] = col
    return full


def apply_channel(rho: np.ndarray, kraus, targets: Sequence[int]) -> np.ndarray:
    """sum_i E_i rho E_i^dagger (a new array)."""
    n = int(rho.shape[0]).bit_length() - 1
    out = np.zeros_like(rho)
    for e in kraus:
        f = embed(np.asarray(e, dtype=np.complex128), targets, n)
        out += f @ rho @ f.conj().T
    return out


def run(n: int, channels, rho: np.ndarray | None = None) -> np.ndarray:
    """Apply channels (objects with .kraus and .targets) in order."""
    if rho is None:
        rho = zero(n)
    for ch in channels:
        rho = apply_channel(rho, ch.kraus, ch.targets)
    return rho


def vec(rho: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(rho.reshape(-1, order="F"))


def unvec(v: np.ndarray) -> np.ndarray:
    d = int(round(np.sqrt(v.size)))
    return np.ascontiguousarray(np.asarray(v).reshape((d, d), order="F"))


def probs(rho: np.ndarray) -> np.ndarray:
    """Outcome probabilities of a computational-basis measurement: Re rho_xx."""
    return np.ascontiguousarray(rho.diagonal().real)


def trace(rho: np.ndarray) -> float:
    return float(np.trace(rho).real)


def purity(rho: np.ndarray) -> float:
    """Tr(rho^dagger rho) = sum |rho_ij|^2 (equals Tr rho^2 for Hermitian rho)."""
    return float(np.vdot(rho, rho).real)
