"""Seeded synthetic circuit families.

These generators are the only code shared by the CPU oracle and the GPU
path.  They build input gate lists and hold none of the simulation method's
arithmetic: a gate is an ordered target tuple plus its dense complex128
matrix, in the little-endian convention of the fused-operator interface
(Section II, "Fused gates and requests": target q_j supplies bit j of the
row and column index).

Families (stand-ins for the paper's random-brickwork ``rand{N}x50``,
``qft{N}`` and depth-20 weak-scaling inputs of Section V-A, whose files are
not available; the shapes, sizes and seeds follow the paper's workloads):

* brickwork(n, depth, seed): each layer applies a Haar-random SU(2) to every
  qubit, then CZ on neighbour pairs (2i, 2i+1) on even layers and
  (2i+1, 2i+2) on odd layers.
* qft(n): H and controlled-phase ladder, most significant qubit first, then
  the final bit-reversal swaps; maps |x> to 2^{-n/2} sum_y e^{+2 pi i x y / 2^n} |y>.
* param_ladder(n, depth, rng): RY then RZ on every qubit with angles uniform
  in [0, 2 pi), then CNOT(q -> q+1) for q = 0..n-2, per layer.
* batch_family(count, seed): ``count`` param_ladder circuits with n uniform
  in [10, 18] and depth uniform in [8, 32].
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Gate:
    kind: str
    targets: Tuple[int, ...]
    matrix: np.ndarray  # complex128, shape (2^k, 2^k), row r / column c bit j <-> targets[j]
    diag: bool = False

    @property
    def k(self) -> int:
        return len(self.targets)


# ---------------------------------------------------------------- gate matrices
_H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)
_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)


def haar_su2(rng: np.random.Generator) -> np.ndarray:
    """Haar-random SU(2): a unit quaternion from four i.i.d. normals."""
    v = rng.standard_normal(4)
    v = v / np.linalg.norm(v)
    a = complex(v[0], v[1])
    b = complex(v[2], v[3])
    return np.array([[a, -b.conjugate()], [b, a.conjugate()]], dtype=np.complex128)


def ry(theta: float) -> np.ndarray:
    c, s = math.cos(theta / 2.0), math.sin(theta / 2.0)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def rz(phi: float) -> np.ndarray:
    return np.array([[complex(math.cos(phi / 2), -math.sin(phi / 2)), 0],
                     [0, complex(math.cos(phi / 2), math.sin(phi / 2))]], dtype=np.complex128)


def cz() -> np.ndarray:
    return np.diag([1, 1, 1, -1]).astype(np.complex128)


def cphase(theta: float) -> np.ndarray:
    return np.diag([1, 1, 1, complex(math.cos(theta), math.sin(theta))]).astype(np.complex128)


def cnot() -> np.ndarray:
    """CNOT on targets (control, target): row/col bit 0 = control, bit 1 = target."""
    m = np.zeros((4, 4), dtype=np.complex128)
    for c in range(4):
        ctl, tgt = c & 1, (c >> 1) & 1
        r = ctl | ((tgt ^ ctl) << 1)
        m[r, c] = 1.0
    return m


def swap() -> np.ndarray:
    m = np.zeros((4, 4), dtype=np.complex128)
    for c in range(4):
        r = ((c & 1) << 1) | ((c >> 1) & 1)
        m[r, c] = 1.0
    return m


# ---------------------------------------------------------------- families
def brickwork(n: int, depth: int, seed: int = 0) -> List[Gate]:
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    for layer in range(depth):
        for q in range(n):
            gates.append(Gate("su2", (q,), haar_su2(rng)))
        start = 0 if layer % 2 == 0 else 1
        for a in range(start, n - 1, 2):
            gates.append(Gate("cz", (a, a + 1), cz(), diag=True))
    return gates


def qft(n: int) -> List[Gate]:
    gates: List[Gate] = []
    for q in range(n - 1, -1, -1):
        gates.append(Gate("h", (q,), _H.copy()))
        for p in range(q - 1, -1, -1):
            gates.append(Gate("cp", (p, q), cphase(math.pi / (1 << (q - p))), diag=True))
    for q in range(n // 2):
        gates.append(Gate("swap", (q, n - 1 - q), swap()))
    return gates


def basis_prep(n: int, x: int) -> List[Gate]:
    """X on every qubit set in x: prepares |x> from |0...0>."""
    return [Gate("x", (q,), _X.copy()) for q in range(n) if (x >> q) & 1]


def ghz(n: int) -> List[Gate]:
    gates = [Gate("h", (0,), _H.copy())]
    for q in range(n - 1):
        gates.append(Gate("cnot", (q, q + 1), cnot()))
    return gates


def inverse(gates: Sequence[Gate]) -> List[Gate]:
    return [Gate(g.kind + "_dg", g.targets, g.matrix.conj().T.copy(), g.diag) for g in reversed(gates)]


def param_ladder(n: int, depth: int, rng: np.random.Generator) -> List[Gate]:
    gates: List[Gate] = []
    for _ in range(depth):
        th = rng.uniform(0.0, 2 * math.pi, size=n)
        ph = rng.uniform(0.0, 2 * math.pi, size=n)
        for q in range(n):
            gates.append(Gate("ry", (q,), ry(float(th[q]))))
            gates.append(Gate("rz", (q,), rz(float(ph[q])), diag=True))
        for q in range(n - 1):
            gates.append(Gate("cnot", (q, q + 1), cnot()))
    return gates


def batch_family(count: int, seed: int = 0, n_lo: int = 10, n_hi: int = 18,
                 d_lo: int = 8, d_hi: int = 32) -> List[Tuple[int, List[Gate]]]:
    out = []
    for i in range(count):
        rng = np.random.default_rng([seed, i])
        n = int(rng.integers(n_lo, n_hi + 1))
        d = int(rng.integers(d_lo, d_hi + 1))
        out.append((n, param_ladder(n, d, rng)))
    return out


def headline(n: int = 30, depth: int = 24, seed: int = 0) -> List[Gate]:
    """Random brickwork of the given depth followed by a full QFT on n qubits."""
    return brickwork(n, depth, seed) + qft(n)


def random_dense(n: int, k: int, rng: np.random.Generator, targets=None) -> Gate:
    """A Haar-distributed k-qubit unitary (QR of a complex Ginibre matrix)."""
    d = 1 << k
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / math.sqrt(2)
    q, r = np.linalg.qr(z)
    q = q * (np.diag(r) / np.abs(np.diag(r)))
    if targets is None:
        targets = tuple(int(t) for t in rng.choice(n, size=k, replace=False))
    return Gate("dense", tuple(targets), q.astype(np.complex128))


# ---------------------------------------------------------------- flat packing
def pack(gates: Sequence[Gate]):
    """Flatten a gate list into (ks int32[G], targets int32[sum k], mats float64[sum 2*4^k])."""
    ks = np.array([g.k for g in gates], dtype=np.int32)
    tg = np.array([t for g in gates for t in g.targets], dtype=np.int32)
    mats = np.concatenate([np.ascontiguousarray(g.matrix, dtype=np.complex128).reshape(-1).view(np.float64)
                           for g in gates]) if gates else np.zeros(0, np.float64)
    return ks, tg, mats


def gate_count(gates: Sequence[Gate]) -> int:
    return len(gates)
