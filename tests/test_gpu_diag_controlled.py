"""Controlled diagonal sweeps on the GPU: the controlled fast path of the
diagonal lowering.

Suppose a diagonal block's table is exactly 1 wherever some target bit is 0.
Then that target is a control: the amplitudes with the bit clear stay as they
are, and the sweep visits only the chunks with every such control set.  Only
controls at physical bit 4 or above are used, so that skipped runs are whole
cache lines.  Each case is checked three ways:
- against the oracle (complex128, gate by gate);
- the skipped amplitudes are bit-for-bit unchanged;
- the number of skipped control bits read from the handle's statistics.
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


def controlled_table(k, ctl, rng):
    """Random unit phases, exactly 1 wherever a bit listed in ctl is 0."""
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, 1 << k))
    for r in range(1 << k):
        if any(not (r >> j) & 1 for j in ctl):
            ph[r] = 1.0
    return ph


# (n, physical = logical targets, control block bits, control bits the sweep skips)
CASES = [
    (14, (6,), [0], 1),                               # a phase on one qubit
    (14, (3, 9), [0, 1], 1),                          # controlled phase: bit 3 is too low to skip
    (14, (9, 3), [0, 1], 1),
    (15, (4, 12, 7), [0, 1, 2], 3),                   # doubly controlled phase
    (16, (2, 5, 11, 14, 0), [2], 1),                  # QFT-like block: one common control
    (13, (12, 1), [], 0),                             # generic diagonal
    (20, (19, 4, 8, 0, 13, 6, 2, 10), [0, 1], 2),     # k = 8, table in device memory
    (9, (8, 7, 6, 5, 4), [0, 1, 2, 3, 4], 5),         # every target a control: 2^-5 of the state
]


@pytest.mark.parametrize("n,targets,ctl,skipped", CASES)
def test_controlled_diagonal(P, n, targets, ctl, skipped):
    rng = np.random.default_rng(7 * n + len(targets))
    prep = W.brickwork(n, 2, seed=n)
    g = W.Gate("diag", tuple(targets), np.diag(controlled_table(len(targets), ctl, rng)), True)
    sv = P.StateVector(n)
    sv.set_relabel(False)
    sv.apply_gates(prep)
    assert list(sv.layout()) == list(range(n))
    before = sv.physical_state().copy()
    bits0 = sv.stats()["diag_control_bits"]
    sv.apply(g.matrix, g.targets)
    assert sv.stats()["diag_control_bits"] - bits0 == skipped
    after = sv.physical_state()
    idx = np.arange(1 << n)
    untouched = np.zeros(1 << n, dtype=bool)
    for j in ctl:
        untouched |= ((idx >> targets[j]) & 1) == 0
    np.testing.assert_array_equal(after[untouched], before[untouched])
    ref = oracle.run(n, prep + [g])
    m = oracle.metrics(ref, oracle.decode(after, sv.layout()))
    assert m["infidelity"] < 1e-5 and m["max_abs"] < 1e-5, m
    sv.close()


def test_controlled_diagonals_in_bound_plan_and_graph(P):
    """A random start state then QFT16, fused greedily (its diagonal blocks share the qubit that took
    the Hadamard): eager, bound and graph-replayed runs agree bit for bit and with the oracle."""
    n = 16
    gates = W.brickwork(n, 2, seed=3) + W.qft(n)
    plan = P.Plan.greedy(n, gates, 5)
    sv = P.StateVector(n)
    sv.set_relabel(False)
    b0 = sv.stats()["diag_control_bits"]
    plan.run(sv)
    per_run = sv.stats()["diag_control_bits"] - b0
    assert per_run > 0
    eager = sv.physical_state().copy()
    lay = sv.layout()
    m = oracle.metrics(oracle.run(n, gates), oracle.decode(eager, lay))
    assert m["infidelity"] < 1e-5 and m["max_abs"] < 1e-5, m
    sv.reset()
    bound = plan.bind(sv)
    b1 = sv.stats()["diag_control_bits"]
    bound.run()
    assert sv.stats()["diag_control_bits"] - b1 == per_run
    np.testing.assert_array_equal(sv.physical_state(), eager)
    for rep in range(3):
        sv.reset()
        sv.norm()  # eager work between replays
        bound.run_graph()
        np.testing.assert_array_equal(sv.physical_state(), eager, err_msg="graph replay %d" % rep)
    bound.close()
    sv.close()
