"""GPU parity of the HIP path against the CPU oracle (through the C-ABI).

Tolerances: the FP32 paths must reach state fidelity >= 1 - 1e-5 and
max |delta amplitude| <= 1e-5 against the complex128 oracle; the tests also
bound the relative L2 error by 1e-5, which is tighter (1 - F ~ |delta|^2).
Integer work (sampling, layout bookkeeping) is compared bit for bit.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

F_TOL = 1e-5
AMP_TOL = 1e-5
L2_TOL = 1e-5


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2608_16940_amd as P
    P.lib()
    return P


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_logical(sv):
    return oracle.decode(sv.physical_state(), sv.layout())


def check_close(ref, got, f_tol=F_TOL, amp_tol=AMP_TOL, l2_tol=L2_TOL, what=""):
    m = oracle.metrics(ref, got)
    assert m["infidelity"] <= f_tol, (what, m)
    assert m["max_abs"] <= amp_tol, (what, m)
    assert m["rel_l2"] <= l2_tol, (what, m)
    return m


def rand_state_gates(n, rng, count=3):
    """A few Haar single-qubit gates on every qubit: a generic dense start state."""
    gates = []
    for _ in range(count):
        for q in range(n):
            gates.append(W.Gate("su2", (q,), W.haar_su2(rng)))
        for q in range(0, n - 1, 2):
            gates.append(W.Gate("cz", (q, q + 1), W.cz(), True))
    return gates


def target_patterns(n, k, rng):
    lo = list(range(k))
    hi = list(range(n - k, n))
    mixed = sorted(rng.choice(n, size=k, replace=False).tolist())
    rev = list(reversed(lo))
    spread = [int(round(i * (n - 1) / max(1, k - 1))) for i in range(k)] if k > 1 else [n // 2]
    pats = [lo, hi, mixed, rev, spread, rng.permutation(n)[:k].tolist()]
    return [tuple(int(x) for x in p) for p in pats if len(set(p)) == k]


# ---------------------------------------------------------------- every lowering
@pytest.mark.parametrize("variant,ks", [("valu", [1, 2, 3, 4]), ("generic", [1, 2, 3, 5, 8]),
                                        ("mfma", [4, 5, 6, 7])])
@pytest.mark.parametrize("n", [13, 17])
def test_dense_variants_match_oracle(P, variant, ks, n):
    rng = np.random.default_rng(100 + n)
    prep = rand_state_gates(n, rng)
    for k in ks:
        gates = list(prep)
        for tg in target_patterns(n, k, rng):
            gates.append(W.random_dense(n, k, rng, targets=tg))
        say("variant", variant, "n", n, "k", k, "gates", len(gates))
        ref = oracle.run(n, gates)
        sv = P.StateVector(n)
        sv.apply_gates(prep)
        before = sv.stats()["by_variant"][P._native.VARIANT[variant]]
        sv.set_variant(variant)
        sv.apply_gates(gates[len(prep):])
        after = sv.stats()["by_variant"][P._native.VARIANT[variant]]
        assert after - before == len(gates) - len(prep)
        check_close(ref, gpu_logical(sv), what=(variant, n, k))
        sv.close()


@pytest.mark.parametrize("n", [1, 2, 5, 7, 12])
def test_shuffle_single_qubit_every_low_bit(P, n):
    rng = np.random.default_rng(7 + n)
    prep = rand_state_gates(n, rng, 2)
    gates = []
    for b in range(min(n, 7)):
        gates.append(W.Gate("su2", (b,), W.haar_su2(rng)))
    ref = oracle.run(n, prep + gates)
    sv = P.StateVector(n)
    sv.apply_gates(prep)
    sv.set_variant("shuffle")
    sv.apply_gates(gates)
    check_close(ref, gpu_logical(sv), what=("shuffle", n))


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16x3", 2e-4)])
def test_mfma_precisions_deep(P, prec, tol):
    """Many k=5 and k=6 sweeps at n=18; BF16x3 is pinned by tolerance only."""
    n = 18
    rng = np.random.default_rng(55)
    gates = rand_state_gates(n, rng, 1)
    for i in range(12):
        k = 5 + (i % 2)
        gates.append(W.random_dense(n, k, rng))
    ref = oracle.run(n, gates)
    sv = P.StateVector(n)
    sv.set_precision(prec)
    sv.apply_gates(gates)
    m = oracle.metrics(ref, gpu_logical(sv))
    say("precision", prec, m)
    assert m["infidelity"] <= 1e-5 and m["max_abs"] <= 1e-5 and m["rel_l2"] <= tol, m


def test_auto_selector_mixed_widths(P):
    n = 16
    rng = np.random.default_rng(9)
    gates = rand_state_gates(n, rng, 2)
    for k in [1, 2, 3, 4, 5, 6, 7, 8, 1, 5, 4]:
        gates.append(W.random_dense(n, k, rng))
    ref = oracle.run(n, gates)
    sv = P.StateVector(n)
    sv.apply_gates(gates)
    check_close(ref, gpu_logical(sv), what="auto")
    st = sv.stats()
    assert st["by_variant"][P._native.VARIANT["mfma"]] >= 4


def random_diagonal(n, k, rng, targets=None):
    t = tuple(int(q) for q in (targets if targets is not None else rng.choice(n, k, replace=False)))
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, 1 << k))
    return W.Gate("diag%d" % k, t, np.diag(ph), diag=True)


@pytest.mark.parametrize("n", [1, 2, 9, 17])
def test_diagonal_lowering_matches_oracle(P, n):
    """Exactly diagonal matrices take the streaming diagonal kernel (any k <= 8, any target order)."""
    rng = np.random.default_rng(40 + n)
    gates = rand_state_gates(n, rng, 1)
    diag_gates = []
    for k in range(1, min(n, 8) + 1):
        diag_gates.append(random_diagonal(n, k, rng))
    diag_gates.append(random_diagonal(n, 1, rng, [0]))
    diag_gates.append(random_diagonal(n, 1, rng, [n - 1]))
    if n >= 3:
        diag_gates.append(random_diagonal(n, 3, rng, [n - 1, 0, n // 2]))
    gates += diag_gates
    ref = oracle.run(n, gates)
    sv = P.StateVector(n)
    sv.apply_gates(gates[:-len(diag_gates)])
    before = sv.stats()["by_variant"][P._native.VARIANT["diag"]]
    sv.apply_gates(diag_gates)
    after = sv.stats()["by_variant"][P._native.VARIANT["diag"]]
    assert after - before == len(diag_gates)
    check_close(ref, gpu_logical(sv), what="diag n=%d" % n)
    sv.close()


def test_diagonal_forced_and_rejected(P):
    n = 12
    rng = np.random.default_rng(3)
    sv = P.StateVector(n)
    sv.set_variant("diag")
    with pytest.raises(RuntimeError):
        sv.apply(W.random_dense(n, 2, rng).matrix, [1, 2])
    # a diagonal gate forced through the dense MFMA sweep gives the same state
    g = random_diagonal(n, 5, rng, [0, 3, 4, 8, 11])
    prep = rand_state_gates(n, rng, 1)
    ref = oracle.run(n, prep + [g])
    sv.set_variant("auto")
    sv.apply_gates(prep)
    sv.set_variant("mfma")
    sv.apply(g.matrix, g.targets)
    check_close(ref, gpu_logical(sv), what="diag via mfma")
    sv.close()


# ---------------------------------------------------------------- whole circuits
def test_c1_gate_by_gate_n20_and_samples(P):
    """N=20, 20 brickwork layers applied gate by gate; 10^4 samples, fixed seed."""
    n = 20
    gates = W.brickwork(n, 20, seed=0)
    ref = oracle.run(n, gates)
    sv = P.StateVector(n)
    sv.apply_gates(gates)
    got = gpu_logical(sv)
    m = check_close(ref, got, what="C1")
    say("C1 metrics", m)
    seed = 0x5EED
    shots = sv.sample(seed, 10_000)
    # bit-exact against the oracle sampler on the GPU's own probabilities, decoded
    p_phys = sv.probs(logical=False).cpu().numpy()
    ys = oracle.sample(p_phys, seed, 10_000)
    xs = oracle.decode_index(ys, sv.layout())
    np.testing.assert_array_equal(shots, xs)
    # GPU probabilities in logical order equal |amplitude|^2 of the decoded state (computed in FP64)
    p_log = sv.probs(logical=True).cpu().numpy()
    np.testing.assert_array_equal(p_log, oracle.decode(sv.physical_state(), sv.layout()).real ** 2
                                  + oracle.decode(sv.physical_state(), sv.layout()).imag ** 2)


@pytest.mark.parametrize("n,k_max", [(14, 5), (18, 5), (16, 4), (20, 7)])
def test_greedy_plan_brickwork_plus_qft(P, n, k_max):
    gates = W.headline(n, 6)
    ref = oracle.run(n, gates)
    sv = P.StateVector(n)
    plan = P.Plan.greedy(n, gates, k_max)
    plan.run(sv)
    check_close(ref, gpu_logical(sv), what=("plan", n, k_max))
    st = sv.stats()
    assert st["gate_sweeps"] + st["layout_only"] == len(plan)
    assert st["layout_only"] >= 1  # the QFT's closing swaps need no sweep


def test_ghz_and_qft_closed_forms(P):
    n = 16
    sv = P.StateVector(n)
    sv.apply_gates(W.ghz(n))
    got = gpu_logical(sv)
    ref = np.zeros(1 << n, dtype=np.complex128)
    ref[0] = ref[-1] = 1 / math.sqrt(2)
    check_close(ref, got, what="ghz")
    x = 12345
    sv.reset()
    plan = P.Plan.greedy(n, W.basis_prep(n, x) + W.qft(n), 5)
    plan.run(sv)
    y = np.arange(1 << n)
    ref = np.exp(2j * np.pi * x * y / (1 << n)) / math.sqrt(1 << n)
    check_close(ref, gpu_logical(sv), what="qft")


# ---------------------------------------------------------------- layout
def test_permute_layout_and_canonicalize(P):
    n = 15
    rng = np.random.default_rng(21)
    gates = rand_state_gates(n, rng, 2)
    ref = oracle.run(n, gates)
    sv = P.StateVector(n)
    sv.apply_gates(gates)
    for _ in range(3):
        L = rng.permutation(n)
        sv.permute_layout(L)
        np.testing.assert_array_equal(sv.layout(), L)
        check_close(ref, gpu_logical(sv), what="permuted")
    # keep applying gates in a scrambled layout: targets resolve through L
    more = [W.random_dense(n, k, rng) for k in (1, 2, 3, 5, 6)]
    ref2 = oracle.run(n, more, ref.copy())
    sv.apply_gates(more)
    check_close(ref2, gpu_logical(sv), what="gates after permute")
    sv.canonicalize()
    np.testing.assert_array_equal(sv.layout(), np.arange(n))
    check_close(ref2, sv.physical_state(), what="canonical")


def test_bad_layout_rejected(P):
    sv = P.StateVector(6)
    with pytest.raises(P.SvError):
        sv.permute_layout([0, 1, 2, 3, 4, 4])
    with pytest.raises(P.SvError):
        sv.apply(np.eye(4), [2, 2])
    with pytest.raises(P.SvError):
        sv.apply(np.eye(2), [6])


# ---------------------------------------------------------------- sampler
@pytest.mark.parametrize("n", [3, 10, 12, 17, 21])
def test_sampler_bit_exact_fixed_probabilities(P, n):
    import torch
    rng = np.random.default_rng(n)
    p = rng.random(1 << n) ** 3
    p[rng.random(1 << n) < 0.3] = 0.0
    p /= p.sum()
    pd = torch.from_numpy(p).cuda()
    # the same values 8 bytes into an allocation: the block totals read entry by entry
    shifted = torch.zeros((1 << n) + 1, dtype=torch.float64, device=pd.device)
    shifted[1:] = pd
    pu = shifted[1:]
    assert pu.data_ptr() % 16 == 8
    for seed in (0, 1, 0xDEADBEEFCAFE):
        got = P.sample_probs(pd, seed, 20_000)
        ref = oracle.sample(p, seed, 20_000)
        np.testing.assert_array_equal(got, ref)
        assert np.all(p[got.astype(np.int64)] > 0)
        np.testing.assert_array_equal(P.sample_probs(pu, seed, 20_000), ref)


def test_sampler_delta_and_state_decode(P):
    n = 12
    sv = P.StateVector(n)
    x = 0b101100111001
    sv.apply_gates(W.basis_prep(n, x))
    L = np.random.default_rng(3).permutation(n)
    sv.permute_layout(L)
    s = sv.sample(7, 1000)
    assert np.all(s == x)
    assert abs(sv.norm() - 1.0) < 1e-12


def test_norm_and_probs(P):
    n = 19
    rng = np.random.default_rng(4)
    sv = P.StateVector(n)
    gates = rand_state_gates(n, rng, 2)
    sv.apply_gates(gates)
    ref = oracle.run(n, gates)
    p = sv.probs(logical=True).cpu().numpy()
    np.testing.assert_allclose(p, np.abs(ref) ** 2, atol=1e-9)
    assert abs(sv.norm() - 1.0) < 1e-5


# ---------------------------------------------------------------- lazy relabel (on-demand moves of high targets)
@pytest.mark.parametrize("policy", ["belady", "first_free", "lru"])
def test_relabel_keeps_logical_state(P, policy):
    n = 17
    gates = W.headline(n, 5, seed=3)
    ref = oracle.run(n, gates)
    sv = P.StateVector(n)
    sv.set_relabel(True, low_bits=9, policy=policy)
    plan = P.Plan.greedy(n, gates, 5)
    plan.run(sv)
    st = sv.stats()
    say("relabel", policy, st)
    assert st["relabels"] > 0
    assert sorted(sv.layout().tolist()) == list(range(n))
    check_close(ref, gpu_logical(sv), what=("relabel", policy))
    # samples decode through the relabelled layout
    s = sv.sample(5, 2000)
    p_phys = sv.probs(logical=False).cpu().numpy()
    np.testing.assert_array_equal(s, oracle.decode_index(oracle.sample(p_phys, 5, 2000), sv.layout()))
    sv.canonicalize()
    check_close(ref, sv.physical_state(), what=("relabel canonical", policy))


def test_relabel_plain_calls_lru(P):
    n = 16
    rng = np.random.default_rng(31)
    gates = rand_state_gates(n, rng, 1) + [W.random_dense(n, k, rng) for k in (4, 5, 6, 7, 5, 4, 5)]
    ref = oracle.run(n, gates)
    sv = P.StateVector(n)
    sv.set_relabel(True, low_bits=8)
    sv.apply_gates(gates)
    check_close(ref, gpu_logical(sv), what="relabel plain")


@pytest.mark.parametrize("n", [3, 8, 11, 12, 20])
def test_permute_layout_small_and_tile_paths(P, n):
    rng = np.random.default_rng(40 + n)
    gates = rand_state_gates(n, rng, 2)
    ref = oracle.run(n, gates)
    sv = P.StateVector(n)
    sv.apply_gates(gates)
    for _ in range(2):
        L = rng.permutation(n)
        sv.permute_layout(L)
        np.testing.assert_array_equal(sv.layout(), L)
        check_close(ref, gpu_logical(sv), what=("perm", n))
    st = sv.stats()
    if n >= 12:
        assert st["permute_sweeps"] > 0 and st["swap_half_sweeps"] == 0
    else:
        assert st["permute_sweeps"] == 0


# ---------------------------------------------------------------- bound plans and HIP graphs
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_bound_plan_and_graph_replays(P, prec):
    """A bound plan launches the same kernels with the same operands as plan.run (bit-identical);
    its HIP-graph replays, with eager work between them, reproduce it bit for bit."""
    n = 16
    rng = np.random.default_rng(21)
    gates = rand_state_gates(n, rng, 2) + W.brickwork(n, 4, 3) + W.qft(n)
    gates += [W.random_dense(n, 7, rng), W.random_dense(n, 8, rng), W.random_dense(n, 1, rng, (12,)),
              W.random_dense(n, 1, rng, (3,))]
    plan = P.Plan.greedy(n, gates, 6)
    ref_sv = P.StateVector(n)
    ref_sv.set_precision(prec)
    plan.run(ref_sv)
    ref = ref_sv.physical_state()
    variants = ref_sv.stats()["by_variant"]
    assert variants[P._native.VARIANT["diag"]] > 0 and variants[P._native.VARIANT["mfma"]] > 0
    assert variants[P._native.VARIANT["generic"]] > 0
    sv = P.StateVector(n)
    sv.set_precision(prec)
    bound = plan.bind(sv)
    bound.run()
    np.testing.assert_array_equal(sv.physical_state(), ref)
    for rep in range(3):
        sv.reset()
        bound.run_graph()
        got = sv.physical_state()
        np.testing.assert_array_equal(got, ref)
        assert abs(sv.norm() - 1) < 2e-4  # eager work between replays
        sv.sample(rep, 100)
    st = sv.stats()  # counters restart at each reset; a replay adds one run
    assert st["gate_sweeps"] + st["layout_only"] == len(plan) and st["layout_only"] >= 1
    if prec == "fp32":
        check_close(oracle.run(n, gates), oracle.decode(ref, sv.layout()), what="bound plan")
    bound.close()
    sv.close()
    ref_sv.close()


def test_bound_plan_guards(P):
    n = 12
    rng = np.random.default_rng(5)
    plan = P.Plan.greedy(n, [W.random_dense(n, 5, rng), W.random_dense(n, 2, rng)], 5)
    sv = P.StateVector(n)
    sv.set_relabel(True)
    with pytest.raises(RuntimeError):
        plan.bind(sv)
    sv.set_relabel(False)
    bound = plan.bind(sv)
    bound.run()
    layout = list(range(n))
    layout[0], layout[n - 1] = layout[n - 1], layout[0]
    sv.permute_layout(layout)
    with pytest.raises(RuntimeError):
        bound.run()
    with pytest.raises(RuntimeError):
        bound.run_graph()
    bound.close()
    sv.close()


def perm_matrix(k, perm):
    """|c> -> |pi(c)>, bit j of c moving to bit perm[j]."""
    d = 1 << k
    m = np.zeros((d, d), dtype=np.complex128)
    for c in range(d):
        r = sum(((c >> j) & 1) << perm[j] for j in range(k))
        m[r, c] = 1
    return m


def test_qubit_permutations_go_to_the_layout_map(P):
    """Blocks that only permute their qubits move no data: the layout map absorbs them."""
    n = 12
    rng = np.random.default_rng(17)
    gates = rand_state_gates(n, rng, 1)
    swaps = [W.Gate("swap", (2, 9), perm_matrix(2, [1, 0])),
             W.Gate("cyc", (0, 5, 11), perm_matrix(3, [1, 2, 0])),
             W.Gate("net", (1, 3, 7, 10), perm_matrix(4, [3, 2, 1, 0])),
             W.Gate("id", (4, 6), np.eye(4, dtype=np.complex128)),
             W.random_dense(n, 2, rng, (9, 2))]
    gates += swaps
    ref = oracle.run(n, gates)
    sv = P.StateVector(n)
    sv.apply_gates(gates[:-len(swaps)])
    before = sv.stats()
    sv.apply_gates(swaps)
    after = sv.stats()
    assert after["layout_only"] - before["layout_only"] == 4
    assert after["gate_sweeps"] - before["gate_sweeps"] == 1
    assert list(sv.layout()) != list(range(n))
    check_close(ref, gpu_logical(sv), what="layout-only permutations")
    # a forced variant still sweeps
    sv.set_variant("valu")
    s0 = sv.stats()["gate_sweeps"]
    sv.apply(perm_matrix(2, [1, 0]), [2, 9])
    assert sv.stats()["gate_sweeps"] == s0 + 1
    sv.close()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16x3", 2e-4)])
def test_every_mfma_operand_placement(P, prec, tol):
    """Each MFMA sweep instance (operand in registers, LDS or read through the caches; k = 4..7)."""
    n = 14
    rng = np.random.default_rng(31)
    prep = rand_state_gates(n, rng, 1)
    for opsrc in ("regs", "lds", "global", "auto"):
        gates = prep + [W.random_dense(n, k, rng) for k in (4, 5, 6, 7)]
        ref = oracle.run(n, gates)
        sv = P.StateVector(n)
        sv.apply_gates(prep)
        sv.set_precision(prec)
        sv.set_variant("mfma")
        sv.set_option(P._native.OPT_MFMA_OPERAND, P._native.MFMA_OPERAND[opsrc])
        sv.apply_gates(gates[len(prep):])
        m = oracle.metrics(ref, gpu_logical(sv))
        say("operand", opsrc, prec, m["rel_l2"])
        assert m["infidelity"] <= 1e-5 and m["max_abs"] <= 1e-5 and m["rel_l2"] <= tol, (opsrc, m)
        sv.close()
