"""Batched path, host side (no GPU): the records the kernel runs.

Circuits with more than 2^14 amplitudes are cut into LDS slice passes.  This
test replays the records exactly as the kernel does — gather each slice of
14 qubits, apply the pass's gates in slice coordinates, scatter back — in
complex128 numpy, and compares with the oracle applying the original gates.
"""
import os

import numpy as np
import pytest

import oracle
import workloads as W

SLICE = 14


@pytest.fixture(scope="module")
def B():
    import paper_2608_16940_amd as P
    P.lib()
    from paper_2608_16940_amd import batch as B
    return B


def apply_1q(v, q, m, nb):
    t = v.reshape(-1, 2, 1 << q)
    a, b = t[:, 0, :].copy(), t[:, 1, :].copy()
    t[:, 0, :] = m[0, 0] * a + m[0, 1] * b
    t[:, 1, :] = m[1, 0] * a + m[1, 1] * b


def apply_cnot(v, c, t_, nb):
    idx = np.arange(1 << nb)
    sel = ((idx >> c) & 1 == 1) & ((idx >> t_) & 1 == 0)
    x = idx[sel]
    y = x | (1 << t_)
    v[x], v[y] = v[y].copy(), v[x].copy()


def apply_record(v, rec, mat, nb):
    if rec[0] == 3:
        return  # group header: its members follow as single-qubit records on distinct qubits (they commute)
    if rec[0] == 0:
        m = mat.astype(np.float64).view(np.complex128).reshape(2, 2)
        apply_1q(v, int(rec[1]), m, nb)
    elif rec[0] == 1:
        apply_cnot(v, int(rec[1]), int(rec[2]), nb)
    else:
        raise AssertionError("unexpected record kind %d" % rec[0])


def replay(n, recs, mats):
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1
    if n <= SLICE:
        for r, m in zip(recs, mats):
            apply_record(psi, r, m, n)
        return psi, 0
    i, passes = 0, 0
    while i < len(recs):
        assert recs[i][0] == 2, "pass record expected"
        mask, cnt = int(recs[i][1]), int(recs[i][2])
        pos = [q for q in range(n) if (mask >> q) & 1]
        rest = [q for q in range(n) if not (mask >> q) & 1]
        assert len(pos) == SLICE and pos[:3] == [0, 1, 2]
        x = np.arange(1 << SLICE)
        local = np.zeros_like(x)
        for j, q in enumerate(pos):
            local |= ((x >> j) & 1) << q
        for sl in range(1 << len(rest)):
            base = 0
            for r, q in enumerate(rest):
                base |= ((sl >> r) & 1) << q
            v = psi[base + local].copy()
            j = i + 1
            while j < i + 1 + cnt:
                r = recs[j]
                if r[0] == 4:  # a run of CNOTs as one linear map: new[y] = old[f(y)]
                    masks = np.concatenate([mats[j].view(np.int32), mats[j + 1][:6].view(np.int32)])
                    y = np.arange(1 << SLICE)
                    f = np.zeros_like(y)
                    for b in range(SLICE):
                        f ^= np.where((y >> b) & 1, masks[b], 0)
                    v = v[f].copy()
                    j += 2
                    continue
                assert r[0] == 3 or (0 <= r[1] < SLICE and (r[0] != 1 or 0 <= r[2] < SLICE))
                apply_record(v, r, mats[j], SLICE)
                j += 1
            psi[base + local] = v
        i += 1 + cnt
        passes += 1
    return psi, passes


def ladder(n, depth, rng, reverse=False):
    gates = []
    for layer in range(depth):
        for q in range(n):
            gates.append(W.Gate("ry", (q,), W.ry(float(rng.uniform(0, 2 * np.pi)))))
            gates.append(W.Gate("rz", (q,), W.rz(float(rng.uniform(0, 2 * np.pi)))))
        order = range(n - 2, -1, -1) if (reverse and layer % 2) else range(n - 1)
        for q in order:
            gates.append(W.Gate("cnot", (q + 1, q) if (reverse and layer % 2) else (q, q + 1), W.cnot()))
        if reverse:
            gates.append(W.Gate("cnot", (n - 1, 0), W.cnot()))
    return gates


@pytest.mark.parametrize("n,depth,reverse", [(6, 4, False), (14, 3, True), (15, 5, False), (16, 4, True),
                                             (17, 3, True)])
def test_records_replay_equals_oracle(B, n, depth, reverse):
    rng = np.random.default_rng(100 + n)
    gates = ladder(n, depth, rng, reverse)
    b = B.Batch([(n, gates)])
    recs, mats = b.records(0)
    got, passes = replay(n, recs, mats)
    ref = oracle.run(n, gates)
    m = oracle.metrics(ref, got)
    assert m["infidelity"] <= 1e-10 and m["max_abs"] <= 1e-6, m
    ops = [r for r in recs if r[0] in (0, 1)]
    groups = [r for r in recs if r[0] == 3]
    assert groups and all(2 <= g[1] <= 5 for g in groups)  # layers of rotations run as groups
    linear = [r for r in recs if r[0] == 4 and r[1] >= 3]  # runs of CNOTs merged (passes only)
    assert all(r[1] != -1 for r in linear)
    # RY and RZ on the same qubit fuse into one single-qubit record; every CNOT is a record or in a run
    assert len(ops) + sum(int(r[1]) for r in linear) == depth * n + sum(1 for g in gates if g.kind == "cnot")
    if n > SLICE:
        assert linear
    if n > SLICE:
        assert 1 <= passes <= len(ops)
    else:
        assert passes == 0


def test_committed_batch_golden_matches_oracle():
    """The committed sample (written by tests/golden/make_batch_golden.py) equals the oracle now."""
    import oracle
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch4096_seed0_sample.txt")
    circ, amps = {}, {}
    with open(path) as f:
        for ln in f:
            w = ln.split()
            if not w or w[0].startswith("#"):
                continue
            if w[0] == "circ":
                circ[int(w[1])] = (int(w[2]), float(w[3]))
            else:
                amps.setdefault(int(w[1]), []).append((int(w[2]), complex(float(w[3]), float(w[4]))))
    assert len(circ) == 64 and all(len(v) == 16 for v in amps.values())
    circs = W.batch_family(65, seed=0)  # circuit i depends only on (seed, i)
    for i in (0, 64):
        n, gates = circs[i]
        assert n == circ[i][0]
        psi = oracle.run(n, gates)
        assert abs(oracle.expect_z(psi, 0) - circ[i][1]) < 1e-14
        for x, v in amps[i]:
            assert abs(psi[x] - v) < 1e-15


def test_prepare_reports_first_bad_circuit(B):
    """The host pass prepares circuits on several threads; a bad circuit is still reported by the
    lowest failing index, before any device call (the workspace pointer is never touched)."""
    import ctypes
    from types import SimpleNamespace
    import paper_2608_16940_amd as P
    from paper_2608_16940_amd import _native
    x = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    circs = []
    for i in range(600):
        n = 10 + i % 7
        gates = [SimpleNamespace(targets=(q,), matrix=x) for q in range(n)]
        gates += [SimpleNamespace(targets=(q, q + 1), matrix=None, kind="cnot") for q in range(n - 1)]
        circs.append((n, gates))
    b = B.Batch(circs)
    lib = P.lib()

    def prepare():
        prep = ctypes.c_void_p()
        rc = lib.sv_batch_prepare(b.count, b.arr, b.state_bytes,
                                  b.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), None,
                                  ctypes.c_void_p(256), 1 << 20, None, ctypes.byref(prep))
        return rc, lib.sv_last_error().decode()

    # a CNOT on one qubit in circuit 417, then also an unknown kind in circuit 233
    j = circs[417][0]  # the first CNOT of circuit 417
    k417 = b._keep[3 * 417 + 1]
    k417[2 * j + 1] = k417[2 * j]
    rc, msg = prepare()
    assert rc == _native.SV_ERR_ARG and msg == "bad CNOT in batch circuit 417", msg
    b._keep[3 * 233][3] = 7
    rc, msg = prepare()
    assert rc == _native.SV_ERR_ARG and msg == "unknown gate kind in batch circuit 233", msg
