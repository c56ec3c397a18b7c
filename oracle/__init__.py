"""CPU oracle for the fused-operator state-vector path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``; never by the product package.
It shares no code with the HIP path: the only common module is the seeded
input generator ``workloads``.

The core (``sv_oracle.c``) is plain complex128 C compiled with gcc; this
module wraps it and adds the FP64 reference pieces that are easiest to read
in numpy:

* ``run``/``apply_gate`` -- gate-by-gate application on the unfused circuit
  (Section IV-B, the R2 semantics with the little-endian target convention of
  Section II);
* ``decode`` -- read a physically stored state through a layout map
  (Section IV-D, y_{L(q)} = x_q);
* ``sample`` -- strict-upper-bound inverse-CDF sampling (Section IV-E);
* ``metrics`` -- fidelity, max |delta|, relative L2 in FP64;
* ``block_matrix`` -- the fused matrix of a block, later gates multiplied on
  the left (Section IV-C);
* ``mlp_*`` -- FP64 forward, backward and Adam step for the cost model.

Every function here is
pinned by a ``-m "not gpu"`` test in ``tests/test_oracle.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C core with gcc (-O2, OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        up = ctypes.POINTER(ctypes.c_uint64)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.orc_apply_gate.argtypes = [dp, ctypes.c_int, dp, ip, ctypes.c_int]
        L.orc_apply_gate.restype = ctypes.c_int
        L.orc_apply_circuit.argtypes = [dp, ctypes.c_int, ctypes.c_int, ip, ip, dp]
        L.orc_apply_circuit.restype = ctypes.c_int
        L.orc_zero_state.argtypes = [dp, ctypes.c_int]
        L.orc_probs.argtypes = [dp, ctypes.c_int, dp]
        L.orc_decode.argtypes = [dp, ctypes.c_int, ip, dp]
        L.orc_expect_z.argtypes = [dp, ctypes.c_int, ctypes.c_int]
        L.orc_expect_z.restype = ctypes.c_double
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_shot_bits.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_shot_bits.restype = ctypes.c_uint64
        L.orc_sample.argtypes = [dp, ctypes.c_int, ctypes.c_uint64, ctypes.c_int64, up]
        L.orc_sample.restype = ctypes.c_int
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def threads() -> int:
    return lib().orc_max_threads()


def set_threads(t: int) -> None:
    lib().orc_set_threads(int(t))


# ------------------------------------------------------------------ states
def zero_state(n: int) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().orc_zero_state(_dp(psi.view(np.float64)), n)
    return psi


def apply_gate(psi: np.ndarray, matrix: np.ndarray, targets: Sequence[int]) -> None:
    """In place: apply ``matrix`` on ordered ``targets`` (q_j <-> bit j)."""
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous
    n = int(psi.size).bit_length() - 1
    m = np.ascontiguousarray(matrix, dtype=np.complex128)
    t = np.ascontiguousarray(np.asarray(targets, dtype=np.int32))
    k = t.size
    assert m.shape == (1 << k, 1 << k)
    rc = lib().orc_apply_gate(_dp(psi.view(np.float64)), n, _dp(m.view(np.float64)), _ip(t), k)
    if rc:
        raise ValueError("oracle: bad gate (targets %r)" % (list(targets),))


def run(n: int, gates, psi: np.ndarray | None = None) -> np.ndarray:
    """Apply a gate list (objects with .matrix and .targets) gate by gate."""
    if psi is None:
        psi = zero_state(n)
    if not gates:
        return psi
    ks = np.array([len(g.targets) for g in gates], dtype=np.int32)
    tg = np.array([t for g in gates for t in g.targets], dtype=np.int32)
    mats = np.concatenate([np.ascontiguousarray(g.matrix, dtype=np.complex128).reshape(-1)
                           for g in gates]).view(np.float64)
    rc = lib().orc_apply_circuit(_dp(psi.view(np.float64)), n, len(gates), _ip(ks), _ip(tg), _dp(mats))
    if rc:
        raise ValueError("oracle: bad gate in circuit")
    return psi


def probs(psi: np.ndarray) -> np.ndarray:
    n = int(psi.size).bit_length() - 1
    p = np.empty(psi.size, dtype=np.float64)
    lib().orc_probs(_dp(psi.view(np.float64)), n, _dp(p))
    return p


def decode(phys: np.ndarray, layout: Sequence[int]) -> np.ndarray:
    """Logical-order state from a physically stored one: out[x] = phys[y], y_{L(q)} = x_q."""
    phys = np.ascontiguousarray(phys, dtype=np.complex128)
    n = int(phys.size).bit_length() - 1
    lay = np.ascontiguousarray(np.asarray(layout, dtype=np.int32))
    assert lay.size == n and sorted(lay.tolist()) == list(range(n))
    out = np.empty_like(phys)
    lib().orc_decode(_dp(phys.view(np.float64)), n, _ip(lay), _dp(out.view(np.float64)))
    return out


def expect_z(psi: np.ndarray, q: int) -> float:
    n = int(psi.size).bit_length() - 1
    return float(lib().orc_expect_z(_dp(psi.view(np.float64)), n, int(q)))


# ------------------------------------------------------------------ sampling
def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    kk = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, kk, o)
    return [int(v) for v in o]


def shot_bits(seed: int, shot: int) -> int:
    return int(lib().orc_shot_bits(seed & (2**64 - 1), shot & (2**64 - 1)))


def sample(p: np.ndarray, seed: int, shots: int) -> np.ndarray:
    """Indices drawn by the strict-upper-bound integer CDF (see sv_oracle.c)."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    n = int(p.size).bit_length() - 1
    assert p.size == 1 << n
    out = np.empty(int(shots), dtype=np.uint64)
    rc = lib().orc_sample(_dp(p), n, seed & (2**64 - 1), int(shots),
                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    if rc:
        raise ValueError("oracle: zero total probability")
    return out


def decode_index(y: np.ndarray, layout: Sequence[int]) -> np.ndarray:
    """Logical basis index of physical index y: x_q = y_{L(q)}."""
    y = np.asarray(y, dtype=np.uint64)
    x = np.zeros_like(y)
    for q, pos in enumerate(layout):
        x |= ((y >> np.uint64(pos)) & np.uint64(1)) << np.uint64(q)
    return x


# ------------------------------------------------------------------ metrics
def metrics(o: np.ndarray, g: np.ndarray) -> dict:
    """FP64 comparison of oracle state o and test state g (same basis order)."""
    o = np.asarray(o, dtype=np.complex128)
    g = np.asarray(g, dtype=np.complex128)
    oo = float(np.sum(np.abs(o) ** 2))
    gg = float(np.sum(np.abs(g) ** 2))
    og = complex(np.sum(np.conj(o) * g))
    f = abs(og) ** 2 / (oo * gg) if oo > 0 and gg > 0 else 0.0
    d = o - g
    return {
        "fidelity": f,
        "infidelity": 1.0 - f,
        "max_abs": float(np.max(np.abs(d))) if d.size else 0.0,
        "rel_l2": float(np.sqrt(np.sum(np.abs(d) ** 2) / oo)) if oo > 0 else float("inf"),
        "norm_o": oo,
        "norm_g": gg,
    }


# ------------------------------------------------------------------ fusion reference
def block_matrix(gates, block_targets: Sequence[int]) -> np.ndarray:
    """FP64 fused matrix of consecutive gates on the ordered tuple ``block_targets``.

    Each gate is embedded into the k-qubit space of the tuple by applying it
    (with the gate-by-gate definition) to every basis column of the identity;
    the block matrix is the product in circuit order with later gates on the
    left (Section IV-C).
    """
    bt = list(block_targets)
    k = len(bt)
    pos = {q: j for j, q in enumerate(bt)}
    total = np.eye(1 << k, dtype=np.complex128)
    for g in gates:
        local = [pos[q] for q in g.targets]
        emb = np.empty((1 << k, 1 << k), dtype=np.complex128)
        for c in range(1 << k):
            col = np.zeros(1 << k, dtype=np.complex128)
            col[c] = 1.0
            apply_gate(col, g.matrix, local)
            emb[:, c] = col
        total = emb @ total
    return total


# ------------------------------------------------------------------ MLP cost-model reference
def mlp_forward(params, x):
    """FP64 forward of the 2-hidden-layer ReLU MLP: returns (y, cache).

    params = (W1[in,h], b1[h], W2[h,h], b2[h], W3[h,1], b3[1]); x[B,in].
    """
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, dtype=np.float64) for p in params]
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    y = (h2 @ W3 + b3)[:, 0]
    return y, (x, z1, h1, z2, h2)


def mlp_loss_grad(params, x, target):
    """Mean-squared error 0.5 * mean((y - t)^2) and its FP64 gradients by the chain rule."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, dtype=np.float64) for p in params]
    y, (x, z1, h1, z2, h2) = mlp_forward(params, x)
    B = x.shape[0]
    t = np.asarray(target, dtype=np.float64)
    r = y - t
    loss = 0.5 * float(np.mean(r * r))
    dy = (r / B)[:, None]               # dL/dy
    gW3 = h2.T @ dy
    gb3 = dy.sum(axis=0)
    dh2 = dy @ W3.T
    dz2 = dh2 * (z2 > 0)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2.T
    dz1 = dh1 * (z1 > 0)
    gW1 = x.T @ dz1
    gb1 = dz1.sum(axis=0)
    return loss, (gW1, gb1, gW2, gb2, gW3, gb3)


def adam_step(params, grads, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) with bias correction; returns new (params, m, v)."""
    newp, newm, newv = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = beta1 * mm + (1 - beta1) * g
        vv = beta2 * vv + (1 - beta2) * g * g
        mhat = mm / (1 - beta1 ** t)
        vhat = vv / (1 - beta2 ** t)
        newp.append(p - lr * mhat / (np.sqrt(vhat) + eps))
        newm.append(mm)
        newv.append(vv)
    return newp, newm, newv
