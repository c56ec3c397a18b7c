"""Cost model and DP planner, host side (no GPU).

* the host MLP forward equals the FP64 oracle forward on the same weights;
* the windowed DP with the paper's score reaches the brute-force minimum over
  every partition of a window into feasible consecutive blocks
  (Eq. dp-recurrence);
* DP plans (paper score and learned score) applied by the oracle equal the
  unfused circuit;
* the learned score fits held-out measured sweep times better than the
  paper's gamma(k) = 4^k score scaled by least squares.
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W


@pytest.fixture(scope="module")
def P():
    import paper_2608_16940_amd as P
    P.lib()
    return P


@pytest.fixture(scope="module")
def C(P):
    from paper_2608_16940_amd import costmodel as C
    return C


def test_features(C):
    f = C.features(30, [29, 3, 0], diagonal=False)
    np.testing.assert_allclose(f, [30 / 35, 3 / 8, 0, 3 / 35, 29 / 35, -0.25, -0.25, -0.25, -0.25, 0, 1, 1 / 16],
                               rtol=1e-6)
    g = C.features(12, [5, 6], diagonal=True, fraction=0.25, launches=1)
    assert g[9] == 1.0 and g[10] == 0.25 and g[11] == 1 / 16
    with pytest.raises(Exception):
        C.features(12, [5, 6], diagonal=True, fraction=1.5)


def test_diag_sweep_cost_closed_forms(C):
    """The cover the lowering sweeps, in closed form: CZ on positions (10, 20) visits the quarter
    with both bits set (one launch); a controlled phase with one control above bit 3 visits half;
    with both qubits below bit 4 nothing can be skipped (one full sweep); the identity runs nothing;
    two CZs on disjoint high pairs visit 6/16 in four launches or fewer."""
    cz = np.array([1, 1, 1, -1], dtype=np.complex128)
    assert C.diag_sweep_cost(cz, [10, 20]) == (0.25, 1)
    assert C.diag_sweep_cost(cz, [2, 3]) == (1.0, 1)
    cp = np.array([1, 1, 1, np.exp(0.3j)])
    fr, ln = C.diag_sweep_cost(cp, [1, 9])  # only bit 9 can be held fixed
    assert (fr, ln) == (0.5, 1)
    assert C.diag_sweep_cost(np.ones(8, dtype=np.complex128), [4, 5, 6]) == (0.0, 0)
    two = np.array([(-1.0) ** (((x & 1) & ((x >> 1) & 1)) + (((x >> 2) & 1) & ((x >> 3) & 1)))
                    for x in range(16)], dtype=np.complex128)
    fr, ln = C.diag_sweep_cost(two, [10, 11, 20, 21])
    # entries other than 1: exactly one pair set, 6 of 16; an exact cover of them with at most 16 sweeps
    assert abs(fr - 6 / 16) < 1e-12 and 1 <= ln <= 4
    with pytest.raises(Exception):
        C.diag_sweep_cost(cz, [5, 5])


def test_host_forward_matches_oracle(C):
    p = C.init_params(3)
    rng = np.random.default_rng(0)
    X = rng.standard_normal((50, C.NIN)).astype(np.float32)
    y = C.forward_host(p, X)
    ref, _ = oracle.mlp_forward([a.astype(np.float64) for a in C.split_params(p)], X.astype(np.float64))
    np.testing.assert_allclose(y, ref, rtol=1e-9, atol=1e-9)


def paper_score(block):
    return 1 if block["diag"] else 4 ** block["k"]


def brute_force_window(gates, k_max, diag_max):
    h = len(gates)
    best = math.inf
    for cuts in itertools.product([0, 1], repeat=h - 1):
        bounds = [0] + [i + 1 for i, c in enumerate(cuts) if c] + [h]
        total = 0
        ok = True
        for a, b in zip(bounds[:-1], bounds[1:]):
            seg = gates[a:b]
            k = len({q for g in seg for q in g.targets})
            dg = all(g.diag for g in seg)
            cap = diag_max if dg else k_max
            if k > cap and b - a > 1:
                ok = False
                break
            total += 1 if dg else 4 ** k
        if ok:
            best = min(best, total)
    return best


@pytest.mark.parametrize("seed", range(6))
def test_dp_paper_score_is_optimal(P, seed):
    rng = np.random.default_rng(seed)
    n = 5
    gates = []
    for _ in range(10):
        r = rng.random()
        if r < 0.4:
            gates.append(W.Gate("su2", (int(rng.integers(n)),), W.haar_su2(rng)))
        elif r < 0.7:
            a, b = rng.choice(n, 2, replace=False)
            gates.append(W.Gate("cz", (int(a), int(b)), W.cz(), diag=True))
        else:
            gates.append(W.random_dense(n, 2, rng))
    for k_max, diag_max in [(2, 3), (3, 3), (4, 2)]:
        plan = P.Plan.dp(n, gates, k_max=k_max, diag_max=diag_max, window=64)
        got = sum(paper_score(b) for b in plan.blocks())
        assert got == brute_force_window(gates, k_max, diag_max), (seed, k_max, diag_max)


def test_dp_plans_equal_unfused_on_oracle(P, C):
    n = 12
    gates = W.headline(n, 5, seed=2)
    ref = oracle.run(n, gates)
    plans = [P.Plan.dp(n, gates, 5, 6, 64), P.Plan.dp(n, gates, 7, 7, 64, params=C.init_params(5)),
             P.Plan.dp(n, gates, 4, 4, 16)]
    for plan in plans:
        psi = oracle.zero_state(n)
        for b in plan.blocks():
            assert b["k"] <= 7
            oracle.apply_gate(psi, b["matrix"], b["targets"])
        m = oracle.metrics(ref, psi)
        assert m["infidelity"] < 1e-12 and m["max_abs"] < 1e-12
        assert sum(b["n_gates"] for b in plan.blocks()) == len(gates)


def test_learned_score_beats_paper_score_on_held_out_timings(C):
    """Committed timing data: hold out every fifth row, fit, compare errors."""
    path = os.path.join(os.path.dirname(C.WEIGHTS), "costmodel_data.csv")
    if not os.path.exists(C.WEIGHTS) or not os.path.exists(path):
        pytest.skip("no committed cost-model data")
    rows = np.loadtxt(path, delimiter=",", skiprows=1)
    X = rows[:, :C.NIN].astype(np.float32)
    y = rows[:, C.NIN]
    params, meta = C.load()
    test = np.arange(len(y)) % 5 == 0
    # learned: the committed model was trained on the non-held-out rows only
    assert meta.get("holdout") == "every fifth row"
    err_mlp = np.sqrt(np.mean((C.forward_host(params, X[test]) - y[test]) ** 2))
    # paper score: log t = a + b * log(4^k), plus a size term log 2^N, least squares on the training rows
    k = np.rint(X[:, 1] * 8)
    nq = np.rint(X[:, 0] * 35)
    A = np.stack([np.ones_like(k), k * math.log(4), nq * math.log(2)], axis=1)
    coef, *_ = np.linalg.lstsq(A[~test], y[~test], rcond=None)
    err_paper = np.sqrt(np.mean((A[test] @ coef - y[test]) ** 2))
    print("held-out RMSE log-time: learned %.3f, scaled 4^k score %.3f" % (err_mlp, err_paper))
    assert err_mlp < err_paper


def test_reordered_plans_keep_each_qubits_gate_order(P, C):
    """The commute-aware reorder moves gates only across gates on disjoint qubits."""
    n = 10
    gates = W.brickwork(n, 4, 7) + W.qft(n)
    ref = oracle.run(n, gates)
    for plan in [P.Plan.dp(n, gates, 5, 5, 64, reorder=True),
                 P.Plan.learned(n, gates, C.init_params(4)),
                 P.Plan.dp(n, gates, 3, 3, 8, reorder=True)]:
        psi = oracle.zero_state(n)
        for b in plan.blocks():
            if b.get("swap"):
                continue  # a layout swap moves storage, not the logical state
            oracle.apply_gate(psi, b["matrix"], b["targets"])
        m = oracle.metrics(ref, psi)
        assert m["infidelity"] < 1e-12 and m["max_abs"] < 1e-12
        assert sum(b["n_gates"] for b in plan.blocks()) == len(gates)


def test_learned_planner_search_prefers_cheaper_plan(P, C):
    if not os.path.exists(C.WEIGHTS):
        pytest.skip("no committed cost model")
    params, _ = C.load()
    n = 30
    gates = W.brickwork(n, 8, 0)

    def predicted(plan):
        return sum(float(np.exp(C.forward_host(params, C.block_features(n, b)[None])[0]))
                   for b in plan.blocks() if not b.get("swap"))
    best = predicted(P.Plan.learned(n, gates, params))
    for cap in (4, 5, 6, 7):
        assert best <= predicted(P.Plan.dp(n, gates, cap, cap, 64, params=params, reorder=True)) + 1e-9
    assert best < predicted(P.Plan.greedy(n, gates, 5))


def test_repeated_rounds_exact_and_never_worse(P, C):
    """Reorder-and-fuse repeated on the blocks: same state, no more blocks, no higher score."""
    n = 10
    gates = W.brickwork(n, 5, 3) + W.qft(n)
    ref = oracle.run(n, gates)
    once = P.Plan.dp(n, gates, 4, 4, 16, reorder=True)
    again = P.Plan.dp(n, gates, 4, 4, 16, reorder=True, repeat=True)
    assert len(again) <= len(once)
    assert sum(paper_score(b) for b in again.blocks()) <= sum(paper_score(b) for b in once.blocks())
    for plan in (again, P.Plan.paper(n, gates), P.Plan.learned(n, gates, C.init_params(6))):
        psi = oracle.zero_state(n)
        for b in plan.blocks():
            if b.get("swap"):
                continue
            assert b["k"] <= 7
            oracle.apply_gate(psi, b["matrix"], b["targets"])
        m = oracle.metrics(ref, psi)
        assert m["infidelity"] < 1e-12 and m["max_abs"] < 1e-12
        assert sum(b["n_gates"] for b in plan.blocks()) == len(gates)


# ---------------------------------------------------------------- layout swaps chosen by the cost model
def alternating_case(n=30, reps=20, seed=0):
    """Dense 4-qubit gates alternating between qubits 20..23 (slow target bits on MI355X) and 0..3."""
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(reps):
        gates.append(W.random_dense(n, 4, rng, (20, 21, 22, 23)))
        gates.append(W.random_dense(n, 4, rng, (0, 1, 2, 3)))
    return gates


def predicted_with_layout(C, params, n, plan, factor=1.15):
    """Model time of a plan run from the identity layout, swaps priced as the pass prices them."""
    L = list(range(n))
    stream = float(np.exp(C.forward_host(params, C.features(n, [0], True, 1.0, 1)[None])[0]))
    tot = 0.0
    for b in plan.blocks():
        if b.get("swap"):
            for q, d in zip(b["targets"], b["dest"]):
                L[q] = d
            moves = len(b["targets"]) // 2  # each exchange lists two qubits
            tot += stream * factor * ((moves + 4) // 5)
            continue
        tot += float(np.exp(C.forward_host(params, C.block_features(n, b, L)[None])[0]))
    return tot


def test_swap_pass_moves_slow_targets_when_the_model_predicts_a_gain(P, C):
    if not os.path.exists(C.WEIGHTS):
        pytest.skip("no committed cost model")
    params, _ = C.load()
    n = 30
    gates = alternating_case(n)
    base = P.Plan.greedy(n, gates, 4)
    plan = P.Plan.greedy(n, gates, 4)
    assert plan.add_swaps(params) == 1
    blocks = plan.blocks()
    assert len(blocks) == len(base) + 1 and blocks[0].get("swap")
    sw = blocks[0]
    moved = dict(zip(sw["targets"], sw["dest"]))
    # qubits 20..23 leave their bits for a window of four consecutive bits, the occupants take their place
    new = sorted(moved[q] for q in (20, 21, 22, 23))
    assert new == list(range(new[0], new[0] + 4)) and new[0] < 20
    assert sorted(sw["dest"]) == sorted(sw["targets"])
    assert predicted_with_layout(C, params, n, plan) < predicted_with_layout(C, params, n, base)
    # the fused blocks are untouched, so the logical circuit is the same
    for a, b in zip([b for b in blocks if not b.get("swap")], base.blocks()):
        assert a["targets"] == b["targets"] and np.array_equal(a["matrix"], b["matrix"])


def test_swap_pass_inserts_nothing_where_no_gain_is_predicted(P, C):
    if not os.path.exists(C.WEIGHTS):
        pytest.skip("no committed cost model")
    params, _ = C.load()
    plan = P.Plan.learned(30, W.brickwork(30, 6, 0) + W.qft(30), params)
    assert plan.swaps_inserted == 0
    small = P.Plan.greedy(10, W.brickwork(10, 4, 0), 4)
    assert small.add_swaps(params) == 0  # states under 24 qubits get none
    with pytest.raises(P.SvError):
        small.add_swaps(params, margin=-1.0)


def test_swap_blocks_keep_the_logical_state(P, C):
    """Oracle: the fused blocks of a plan with swaps (N=24, the smallest size the pass acts on),
    applied in order, equal the unfused circuit."""
    if not os.path.exists(C.WEIGHTS):
        pytest.skip("no committed cost model")
    params, _ = C.load()
    n = 24
    rng = np.random.default_rng(3)
    gates = []
    for _ in range(6):
        gates.append(W.random_dense(n, 4, rng, (18, 19, 20, 21)))
        gates.append(W.random_dense(n, 3, rng, (0, 1, 2)))
    plan = P.Plan.greedy(n, gates, 4)
    print("swaps at N=24:", plan.add_swaps(params))
    psi = oracle.zero_state(n)
    for b in plan.blocks():
        if not b.get("swap"):
            oracle.apply_gate(psi, b["matrix"], b["targets"])
    m = oracle.metrics(oracle.run(n, gates), psi)
    assert m["infidelity"] < 1e-12 and m["max_abs"] < 1e-12
