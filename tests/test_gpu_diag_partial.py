"""Partial diagonal sweeps on the GPU: the controlled fast path of the
diagonal lowering, generalised.

Amplitudes whose diagonal entry is exactly 1 stay as they are.  A diagonal
block therefore sweeps only subcubes of the state, with target bits at
physical position 4 or above held fixed, that together hold every entry that
is not 1.  Examples:
- a controlled phase sweeps the half with its control set;
- two CZs on disjoint pairs sweep 6/16 of the state, the amplitudes whose
  sign flips, in four subcubes.
Each case is checked three ways:
- against the oracle (complex128, gate by gate);
- every amplitude whose entry is 1 is bit-for-bit unchanged;
- the 16-byte chunks the sweeps visited, from the handle's statistics,
  against the fraction worked out by hand for that case.
The same holds through a bound plan and its HIP-graph replays.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2608_16940_amd as P
    P.lib()
    return P


def controlled_table(k, ctl, rng, anti=()):
    """Random unit phases, exactly 1 wherever a bit in ctl is 0 or a bit in anti is 1."""
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, 1 << k))
    for r in range(1 << k):
        if any(not (r >> j) & 1 for j in ctl) or any((r >> j) & 1 for j in anti):
            ph[r] = 1.0
    return ph


def cz_pair_table():
    """CZ on block bits (0, 1) times CZ on (2, 3)."""
    return np.array([(-1.0) ** (((r & 3) == 3) + ((r >> 2) == 3)) for r in range(16)], dtype=np.complex128)


# (n, physical = logical targets, table maker, fraction of the state the sweeps visit)
CASES = [
    (14, (6,), lambda rng: controlled_table(1, [0], rng), 1 / 2),                   # phase on one qubit
    (14, (3, 9), lambda rng: controlled_table(2, [0, 1], rng), 1 / 2),              # bit 3 too low to fix
    (15, (4, 12, 7), lambda rng: controlled_table(3, [0, 1, 2], rng), 1 / 8),       # doubly controlled phase
    (16, (2, 5, 11, 14, 0), lambda rng: controlled_table(5, [2], rng), 1 / 2),      # QFT-like block
    (13, (12, 1), lambda rng: controlled_table(2, [], rng), 1.0),                   # generic diagonal
    (20, (19, 4, 8, 0, 13, 6, 2, 10), lambda rng: controlled_table(8, [0, 1], rng), 1 / 4),  # device table
    (9, (8, 7, 6, 5, 4), lambda rng: controlled_table(5, [0, 1, 2, 3, 4], rng), 1 / 32),
    (14, (7, 10), lambda rng: controlled_table(2, [1], rng, anti=[0]), 1 / 4),      # anti-control on bit 7
    (22, (5, 9, 12, 20), lambda rng: cz_pair_table(), 6 / 16),                      # two CZs: four subcubes
    (16, (2, 9, 5, 12), lambda rng: cz_pair_table(), 10 / 16),                      # bit 2 cannot be fixed
    (12, (4, 8), lambda rng: np.ones(4, dtype=np.complex128), 0.0),                 # identity: no sweep
]


@pytest.mark.parametrize("n,targets,table,frac", CASES)
def test_partial_diagonal(P, n, targets, table, frac):
    rng = np.random.default_rng(7 * n + len(targets))
    prep = W.brickwork(n, 2, seed=n)
    d = table(rng)
    g = W.Gate("diag", tuple(targets), np.diag(d), True)
    sv = P.StateVector(n)
    sv.set_relabel(False)
    sv.apply_gates(prep)
    assert list(sv.layout()) == list(range(n))
    before = sv.physical_state().copy()
    st0 = sv.stats()
    sv.apply(g.matrix, g.targets)
    st1 = sv.stats()
    assert st1["diag_chunks"] - st0["diag_chunks"] == round(frac * (1 << (n - 1))), (st1, st0)
    after = sv.physical_state()
    idx = np.arange(1 << n)
    r = np.zeros(1 << n, dtype=np.int64)
    for j, t in enumerate(targets):
        r |= ((idx >> t) & 1) << j
    untouched = d[r] == 1
    np.testing.assert_array_equal(after[untouched], before[untouched])
    ref = oracle.run(n, prep + [g])
    m = oracle.metrics(ref, oracle.decode(after, sv.layout()))
    assert m["infidelity"] < 1e-5 and m["max_abs"] < 1e-5, m
    sv.close()


def test_partial_diagonals_in_bound_plan_and_graph(P):
    """A random start state then QFT16 fused greedily, and a brickwork whose CZ layers fuse into diagonal
    blocks: eager, bound and graph-replayed runs agree bit for bit, visit the same chunks, and match the
    oracle."""
    n = 16
    gates = W.brickwork(n, 2, seed=3) + W.qft(n)
    plan = P.Plan.greedy(n, gates, 5)
    sv = P.StateVector(n)
    sv.set_relabel(False)
    plan.run(sv)
    per_run = sv.stats()["diag_chunks"]
    assert 0 < per_run < sum(1 for b in plan.blocks() if b["diag"]) * (1 << (n - 1))
    eager = sv.physical_state().copy()
    m = oracle.metrics(oracle.run(n, gates), oracle.decode(eager, sv.layout()))
    assert m["infidelity"] < 1e-5 and m["max_abs"] < 1e-5, m
    sv.reset()
    bound = plan.bind(sv)
    bound.run()
    assert sv.stats()["diag_chunks"] == per_run
    np.testing.assert_array_equal(sv.physical_state(), eager)
    for rep in range(3):
        sv.reset()
        sv.norm()  # eager work between replays
        bound.run_graph()
        np.testing.assert_array_equal(sv.physical_state(), eager, err_msg="graph replay %d" % rep)
    bound.close()
    sv.close()


# At 2^30 amplitudes and more, sweeps with three to five fixed bits all at
# physical 13 or below walk their subcube in a different order (two fields of
# the work index exchanged); the others keep the plain order.
LARGE = [
    ((6, 7, 8, 9), lambda rng: controlled_table(4, [0, 1, 2, 3], rng), 1 / 16),   # exchanged order
    ((9, 7, 8), lambda rng: controlled_table(3, [0, 1, 2], rng), 1 / 8),          # exchanged order
    ((5, 9, 12, 13), lambda rng: cz_pair_table(), 6 / 16),                        # four subcubes, 3-4 fixed bits
    ((4, 5, 6, 7, 8), lambda rng: controlled_table(5, [0, 1, 2, 3, 4], rng), 1 / 32),  # five fixed bits
    ((20, 21, 22, 23), lambda rng: controlled_table(4, [0, 1, 2, 3], rng), 1 / 16),    # plain order
    ((8, 9), lambda rng: controlled_table(2, [0, 1], rng), 1 / 4),                # plain order (two bits)
]


@pytest.mark.parametrize("targets,table,frac", LARGE)
def test_partial_diagonal_2e30(P, targets, table, frac):
    """N=30: every amplitude of the subcube is multiplied by its entry exactly once (a traversal that
    visited a chunk twice or skipped one would fail), every other amplitude is bit-for-bit unchanged.
    Checked on the device in slices against torch's complex64 product of the saved state."""
    import torch
    n = 30
    rng = np.random.default_rng(sum(targets))
    d = table(rng)
    sv = P.StateVector(n)
    sv.set_relabel(False)
    for q in range(n):  # a product state whose amplitudes are all different from zero
        a, b = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        nr = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
        a, b = a / nr, b / nr
        sv.apply(np.array([[a, -np.conj(b)], [b, np.conj(a)]]), (q,))
    assert list(sv.layout()) == list(range(n))
    before = sv.amps.clone()
    st0 = sv.stats()
    sv.apply(np.diag(d), targets)
    st1 = sv.stats()
    assert st1["diag_chunks"] - st0["diag_chunks"] == round(frac * (1 << (n - 1)))
    dev = sv.amps.device
    dt = torch.tensor(d.astype(np.complex64), device=dev)
    step = 1 << 26
    for s0 in range(0, 1 << n, step):
        idx = torch.arange(s0, s0 + step, device=dev, dtype=torch.int64)
        r = torch.zeros_like(idx)
        for j, t in enumerate(targets):
            r |= ((idx >> t) & 1) << j
        f = dt[r]
        b = before[s0:s0 + step]
        a = sv.amps[s0:s0 + step]
        one = f == 1
        assert torch.equal(a[one], b[one]), s0
        e = (a[~one] - b[~one] * f[~one]).abs()
        bound = 1e-6 * b[~one].abs() + 1e-12
        assert bool((e <= bound).all()), (s0, float(e.max()))
        assert int((~one).sum()) == int(round(frac * step)), s0
    sv.close()
