"""Seeded noise channels for the density-matrix path.

Inputs only, like the circuit families: a channel is an ordered target tuple
plus its Kraus operators, each a complex128 (2^k, 2^k) matrix in the
little-endian convention of the fused-operator interface (target q_j supplies
bit j of the row and column index).  Nothing here applies a channel.

* unitary(gate): the one-operator channel of a gate.
* depolarizing(targets, p): sqrt(1 - p) I and sqrt(p / (4^k - 1)) P for the
  4^k - 1 non-identity Pauli strings P.
* amplitude_damping(q, gamma), dephasing(q, p): the textbook one-qubit sets.
* random_channel(targets, r, rng): r Kraus operators cut from a Haar-random
  isometry (QR of a complex Ginibre matrix), so sum E_i^dagger E_i = I.
* noisy_brickwork(n, depth, p, seed): the brickwork family with a two-qubit
  depolarizing channel after every CZ.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import List, Sequence, Tuple

import numpy as np

from .circuits import Gate, brickwork

_PAULI = [np.eye(2, dtype=np.complex128),
          np.array([[0, 1], [1, 0]], dtype=np.complex128),
          np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
          np.array([[1, 0], [0, -1]], dtype=np.complex128)]


@dataclasses.dataclass
class Channel:
    kind: str
    targets: Tuple[int, ...]
    kraus: List[np.ndarray]
    diag: bool = False  # every Kraus operator is diagonal

    @property
    def k(self) -> int:
        return len(self.targets)


def unitary(g: Gate) -> Channel:
    return Channel(g.kind, tuple(g.targets), [np.asarray(g.matrix, dtype=np.complex128)], g.diag)


def pauli_string(codes: Sequence[int]) -> np.ndarray:
    """Pauli string with codes[j] in {0: I, 1: X, 2: Y, 3: Z} on bit j."""
    m = np.ones((1, 1), dtype=np.complex128)
    for c in codes:
        m = np.kron(_PAULI[c], m)  # later targets are more significant
    return m


def depolarizing(targets: Sequence[int], p: float) -> Channel:
    k = len(targets)
    ops = [math.sqrt(1.0 - p) * np.eye(1 << k, dtype=np.complex128)]
    w = math.sqrt(p / float(4 ** k - 1))
    for codes in itertools.product(range(4), repeat=k):
        if any(codes):
            ops.append(w * pauli_string(codes))
    return Channel("depolarizing", tuple(targets), ops)


def amplitude_damping(q: int, gamma: float) -> Channel:
    e0 = np.array([[1, 0], [0, math.sqrt(1.0 - gamma)]], dtype=np.complex128)
    e1 = np.array([[0, math.sqrt(gamma)], [0, 0]], dtype=np.complex128)
    return Channel("amp_damp", (q,), [e0, e1])


def dephasing(q: int, p: float) -> Channel:
    return Channel("dephasing", (q,), [math.sqrt(1.0 - p) * _PAULI[0], math.sqrt(p) * _PAULI[3]], diag=True)


def random_channel(targets: Sequence[int], r: int, rng: np.random.Generator) -> Channel:
    d = 1 << len(targets)
    z = (rng.standard_normal((r * d, d)) + 1j * rng.standard_normal((r * d, d))) / math.sqrt(2)
    v, _ = np.linalg.qr(z)  # r*d x d with orthonormal columns
    return Channel("random", tuple(targets), [np.ascontiguousarray(v[i * d:(i + 1) * d, :]) for i in range(r)])


def noisy_brickwork(n: int, depth: int, p: float, seed: int = 0) -> List[Channel]:
    out: List[Channel] = []
    for g in brickwork(n, depth, seed):
        out.append(unitary(g))
        if g.kind == "cz":
            out.append(depolarizing(g.targets, p))
    return out
