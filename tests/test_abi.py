"""C-ABI and host-logic tests that need no GPU.

* libsv.so loads and exports every function declared in include/*.h;
* host-only entry points validate arguments;
* the greedy planner's FP64 block products and block boundaries agree with
  the oracle (fused blocks applied by the oracle equal the unfused circuit).
"""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import oracle
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(sv_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def P():
    import paper_2608_16940_amd as P
    P.lib()
    return P


def test_header_parse_finds_the_boundary():
    names = header_functions()
    for must in ["sv_alloc", "sv_apply_fused", "sv_permute_layout", "sv_probs", "sv_sample",
                 "sv_sample_probs", "sv_plan_greedy", "sv_run_plan"]:
        assert must in names


def test_library_exports_every_declared_symbol(P):
    lib = P.lib()
    missing = [n for n in header_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2608_16940_amd import _native
    bound = {s[0] for s in _native.SIGNATURES}
    assert set(header_functions()) <= bound | set(), sorted(set(header_functions()) - bound)


def test_workspace_bytes_range(P):
    lib = P.lib()
    assert lib.sv_workspace_bytes(0) == 0
    assert lib.sv_workspace_bytes(36) == 0
    a, b = lib.sv_workspace_bytes(20), lib.sv_workspace_bytes(34)
    assert 0 < a < b
    # CDF block totals: one uint64 per 2^10 amplitudes at N = 34
    assert b - a >= 8 * ((1 << 24) - (1 << 10))


def test_alloc_rejects_bad_arguments(P):
    lib = P.lib()
    h = ctypes.c_void_p()
    assert lib.sv_alloc(ctypes.byref(h), 10, None, 0, None, 0, None) == P._native.SV_ERR_ARG
    buf = ctypes.c_void_p(256)
    assert lib.sv_alloc(ctypes.byref(h), 0, buf, 1 << 20, buf, 1 << 30, None) == P._native.SV_ERR_ARG
    assert lib.sv_alloc(ctypes.byref(h), 10, buf, 100, buf, 1 << 30, None) == P._native.SV_ERR_ARG
    assert b"smaller" in lib.sv_last_error()
    assert lib.sv_alloc(ctypes.byref(h), 10, ctypes.c_void_p(257), 1 << 20, buf, 1 << 30, None) == P._native.SV_ERR_ARG


def test_plan_rejects_bad_arguments(P):
    with pytest.raises(P.SvError):
        P.Plan.greedy(4, W.brickwork(4, 1), k_max=0)
    bad = [W.Gate("x", (1, 1), np.eye(4, dtype=np.complex128))]
    with pytest.raises(P.SvError):
        P.Plan.greedy(4, bad, k_max=3)


@pytest.mark.parametrize("k_max", [1, 2, 3, 4, 5, 6])
def test_greedy_blocks_respect_cap_and_cover_all_gates(P, k_max):
    n = 12
    gates = W.brickwork(n, 4, seed=3) + W.qft(n)
    plan = P.Plan.greedy(n, gates, k_max)
    blocks = plan.blocks()
    assert sum(b["n_gates"] for b in blocks) == len(gates)
    for b in blocks:
        assert b["k"] <= max(k_max, 2)
        assert list(b["targets"]) == sorted(b["targets"])
    # greedy maximality: the next gate could not have been absorbed
    pos = 0
    for i, b in enumerate(blocks):
        pos += b["n_gates"]
        if i + 1 < len(blocks) and b["k"] <= k_max:
            nxt = gates[pos]
            assert len(set(b["targets"]) | set(nxt.targets)) > k_max or nxt.k > k_max


def test_greedy_block_matrices_match_oracle_products(P):
    n = 10
    gates = W.brickwork(n, 3, seed=5) + W.qft(n)
    plan = P.Plan.greedy(n, gates, 5)
    pos = 0
    for b in plan.blocks():
        seg = gates[pos:pos + b["n_gates"]]
        pos += b["n_gates"]
        ref = oracle.block_matrix(seg, b["targets"])
        np.testing.assert_allclose(b["matrix"], ref, atol=1e-13)
        assert b["diag"] == all(g.diag for g in seg)


def test_fused_plan_equals_unfused_on_oracle(P):
    n = 12
    gates = W.brickwork(n, 6, seed=0) + W.qft(n)
    ref = oracle.run(n, gates)
    for k_max in (3, 5, 7):
        plan = P.Plan.greedy(n, gates, k_max)
        psi = oracle.zero_state(n)
        for b in plan.blocks():
            oracle.apply_gate(psi, b["matrix"], b["targets"])
        m = oracle.metrics(ref, psi)
        assert m["infidelity"] < 1e-12 and m["max_abs"] < 1e-12, (k_max, m)


def test_planner_rejects_false_diagonal_marker(P):
    """A gate marked diagonal must have an exactly diagonal matrix."""
    x = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    bad = [W.Gate("x", (0,), x, diag=True)]
    with pytest.raises(RuntimeError):
        P.Plan.greedy(3, bad, 2)
    ok = [W.Gate("rz", (0,), W.rz(0.3), diag=True), W.Gate("cz", (0, 1), W.cz(), diag=True)]
    plan = P.Plan.greedy(3, ok, 2)
    assert [b["diag"] for b in plan.blocks()] == [True]
    # an unmarked diagonal matrix is still found diagonal
    plan = P.Plan.greedy(3, [W.Gate("d", (1,), np.diag([1, 1j]))], 2)
    assert plan.blocks()[0]["diag"]
