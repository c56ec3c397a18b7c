"""Pins for the CPU oracle (run without a GPU).

Each test checks the oracle against something other than itself: closed
forms (GHZ, QFT of a basis state, Hadamard layer), textbook special cases
(X permutes, Kronecker products for single-qubit and adjacent two-qubit
gates), brute force on small inputs (full 2^n x 2^n operators built with
numpy's tensordot on the rank-n tensor view, an independent lowering),
invariants (norm, circuit times inverse), published known-answer vectors
(Philox4x32-10), and the statistical check of Section V-B (all-zero GHZ
marginal within binomial standard errors).
"""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- independent references
def tensordot_apply(psi, G, targets):
    """Apply G on ordered targets through the rank-n tensor view (numpy tensordot)."""
    n = int(psi.size).bit_length() - 1
    k = len(targets)
    T = psi.reshape([2] * n)                # axis a <-> qubit n-1-a
    Gt = G.reshape([2] * (2 * k))           # axes: out bits k-1..0, in bits k-1..0
    in_axes = list(range(k, 2 * k))
    st_axes = [n - 1 - targets[k - 1 - i] for i in range(k)]
    R = np.tensordot(Gt, T, axes=(in_axes, st_axes))
    # result axes: out bits (k-1..0), then the remaining state axes in order
    rest = [a for a in range(n) if a not in st_axes]
    order = st_axes + rest
    out = np.empty_like(T)
    out = np.moveaxis(R, list(range(n)), order)
    return np.ascontiguousarray(out).reshape(-1)


def kron_1q(n, G, q):
    return np.kron(np.kron(np.eye(1 << (n - 1 - q)), G), np.eye(1 << q))


def rand_state(n, rng):
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return (v / np.linalg.norm(v)).astype(np.complex128)


# ---------------------------------------------------------------- gate application
@pytest.mark.parametrize("n", [1, 3, 6])
def test_single_qubit_matches_kronecker(n):
    rng = np.random.default_rng(1)
    for q in range(n):
        G = W.haar_su2(rng)
        psi = rand_state(n, rng)
        ref = kron_1q(n, G, q) @ psi
        got = psi.copy()
        oracle.apply_gate(got, G, [q])
        np.testing.assert_allclose(got, ref, atol=1e-13)


def test_adjacent_two_qubit_kronecker_both_orders():
    rng = np.random.default_rng(2)
    n = 5
    G = W.random_dense(n, 2, rng, targets=(0, 1)).matrix
    S = W.swap()
    for q in range(n - 1):
        psi = rand_state(n, rng)
        U = np.kron(np.kron(np.eye(1 << (n - 2 - q)), G), np.eye(1 << q))
        got = psi.copy()
        oracle.apply_gate(got, G, [q, q + 1])
        np.testing.assert_allclose(got, U @ psi, atol=1e-13)
        # reversed target order: q_0 = q+1 is the low bit of G's index
        got2 = psi.copy()
        oracle.apply_gate(got2, G, [q + 1, q])
        U2 = np.kron(np.kron(np.eye(1 << (n - 2 - q)), S @ G @ S), np.eye(1 << q))
        np.testing.assert_allclose(got2, U2 @ psi, atol=1e-13)


@pytest.mark.parametrize("n,k", [(4, 1), (5, 2), (6, 3), (7, 4), (8, 5), (8, 7)])
def test_dense_gate_brute_force(n, k):
    """Random targets in random order vs the tensordot lowering and vs the full operator."""
    rng = np.random.default_rng(10 * n + k)
    for _ in range(3):
        g = W.random_dense(n, k, rng)
        psi = rand_state(n, rng)
        ref = tensordot_apply(psi, g.matrix, list(g.targets))
        got = psi.copy()
        oracle.apply_gate(got, g.matrix, g.targets)
        np.testing.assert_allclose(got, ref, atol=1e-12)
    if n <= 6:
        # full 2^n x 2^n operator, one column per basis state
        U = np.stack([tensordot_apply(np.eye(1 << n, dtype=np.complex128)[:, c].copy(), g.matrix,
                                      list(g.targets)) for c in range(1 << n)], axis=1)
        assert np.allclose(U.conj().T @ U, np.eye(1 << n), atol=1e-12)
        got = psi.copy()
        oracle.apply_gate(got, g.matrix, g.targets)
        np.testing.assert_allclose(got, U @ psi, atol=1e-12)


def test_x_permutes_basis():
    n = 6
    X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    rng = np.random.default_rng(3)
    psi = rand_state(n, rng)
    for q in range(n):
        got = psi.copy()
        oracle.apply_gate(got, X, [q])
        idx = np.arange(1 << n) ^ (1 << q)
        np.testing.assert_array_equal(got, psi[idx])


def test_hadamard_layer_uniform():
    n = 10
    H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2)
    psi = oracle.zero_state(n)
    for q in range(n):
        oracle.apply_gate(psi, H, [q])
    np.testing.assert_allclose(psi, np.full(1 << n, 2 ** (-n / 2)), atol=1e-14)


def test_bad_gates_rejected():
    psi = oracle.zero_state(3)
    with pytest.raises(ValueError):
        oracle.apply_gate(psi, np.eye(4), [1, 1])
    with pytest.raises(ValueError):
        oracle.apply_gate(psi, np.eye(2), [3])


# ---------------------------------------------------------------- whole circuits
@pytest.mark.parametrize("n", [2, 5, 12])
def test_ghz(n):
    psi = oracle.run(n, W.ghz(n))
    ref = np.zeros(1 << n, dtype=np.complex128)
    ref[0] = ref[-1] = 1 / math.sqrt(2)
    np.testing.assert_allclose(psi, ref, atol=1e-14)


@pytest.mark.parametrize("n,x", [(3, 5), (6, 0), (6, 37), (9, 300), (11, 1234)])
def test_qft_of_basis_state(n, x):
    psi = oracle.run(n, W.basis_prep(n, x) + W.qft(n))
    y = np.arange(1 << n)
    ref = np.exp(2j * np.pi * x * y / (1 << n)) / math.sqrt(1 << n)
    np.testing.assert_allclose(psi, ref, atol=1e-12)


def test_circuit_times_inverse_is_identity():
    n = 10
    c = W.brickwork(n, 6, seed=4) + W.qft(n)
    psi = oracle.run(n, c + W.inverse(c))
    ref = np.zeros(1 << n, dtype=np.complex128)
    ref[0] = 1
    np.testing.assert_allclose(psi, ref, atol=1e-12)


def test_norm_preserved_and_brickwork_structure():
    n = 12
    c = W.brickwork(n, 8, seed=0)
    assert len(c) == 8 * n + 4 * (n // 2) + 4 * ((n - 1) // 2)
    psi = oracle.run(n, c)
    assert abs(np.vdot(psi, psi).real - 1) < 1e-12


def test_expect_z_closed_forms():
    n = 4
    for th in [0.0, 0.3, 1.7, 3.1]:
        psi = oracle.zero_state(n)
        oracle.apply_gate(psi, W.ry(th), [0])
        oracle.apply_gate(psi, W.rz(0.77), [0])
        oracle.apply_gate(psi, W.haar_su2(np.random.default_rng(0)), [2])
        assert abs(oracle.expect_z(psi, 0) - math.cos(th)) < 1e-13
    psi = oracle.zero_state(n)
    for q in range(n):
        oracle.apply_gate(psi, W.rz(0.1 + q), [q])
    assert abs(oracle.expect_z(psi, 0) - 1.0) < 1e-14


# ---------------------------------------------------------------- layout decode
def test_decode_matches_tensor_transpose():
    n = 7
    rng = np.random.default_rng(5)
    for _ in range(4):
        logical = rand_state(n, rng)
        L = rng.permutation(n)
        # physical tensor: logical qubit q sits at physical bit L[q]; built by transposing axes
        T = logical.reshape([2] * n)         # axis a <-> logical qubit n-1-a
        perm = [0] * n                        # physical axis b' = n-1-L[q] takes logical axis n-1-q
        for q in range(n):
            perm[n - 1 - L[q]] = n - 1 - q
        phys = np.ascontiguousarray(np.transpose(T, perm)).reshape(-1)
        np.testing.assert_array_equal(oracle.decode(phys, L), logical)
        # index decode agrees with amplitude decode
        y = np.arange(1 << n, dtype=np.uint64)
        x = oracle.decode_index(y, L)
        np.testing.assert_array_equal(logical[x.astype(np.int64)], phys)


def test_paper_worked_example_axis_order():
    """Lazy TTGT worked example (Fig. 3): identity layout, V=(2,4).

    Moving q_j to position n-k+j and keeping the other axes in relative
    order gives the row-major axis order (4,2,n-1,...,5,3,1,0).  The layout
    map that records it, L'(q) = physical bit of q, decodes the permuted
    tensor back to the original state.
    """
    n = 8
    V = (2, 4)
    k = len(V)
    rest = [q for q in range(n) if q not in V]
    Lp = {}
    for j, q in enumerate(V):
        Lp[q] = n - k + j
    for i, q in enumerate(rest):
        Lp[q] = i
    axis_order_msb_first = sorted(range(n), key=lambda q: -Lp[q])
    assert axis_order_msb_first == [4, 2, 7, 6, 5, 3, 1, 0]
    rng = np.random.default_rng(6)
    logical = rand_state(n, rng)
    T = logical.reshape([2] * n)
    phys = np.ascontiguousarray(np.transpose(T, [n - 1 - q for q in axis_order_msb_first])).reshape(-1)
    L = [Lp[q] for q in range(n)]
    np.testing.assert_array_equal(oracle.decode(phys, L), logical)


# ---------------------------------------------------------------- sampler
def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        assert oracle.philox4x32_10(v[0:4], v[4:6]) == v[6:10]


def test_sampler_never_draws_zero_bins_and_delta():
    n = 8
    rng = np.random.default_rng(7)
    p = rng.random(1 << n)
    p[rng.random(1 << n) < 0.6] = 0.0
    p /= p.sum()
    s = oracle.sample(p, seed=11, shots=20000)
    assert np.all(p[s.astype(np.int64)] > 0)
    d = np.zeros(1 << n)
    d[77] = 1.0
    assert np.all(oracle.sample(d, seed=3, shots=1000) == 77)
    # a tiny but non-zero bin next to zero bins is still reachable in principle, never the zeros
    e = np.zeros(1 << n)
    e[5] = 1e-3
    e[200] = 1 - 1e-3
    s = oracle.sample(e, seed=5, shots=5000)
    assert set(np.unique(s).tolist()) <= {5, 200}


def test_sampler_chi_square():
    n = 6
    rng = np.random.default_rng(8)
    p = rng.dirichlet(np.ones(1 << n))
    shots = 200000
    s = oracle.sample(p, seed=123, shots=shots)
    cnt = np.bincount(s.astype(np.int64), minlength=1 << n)
    exp = p * shots
    chi2 = float(np.sum((cnt - exp) ** 2 / exp))
    # 63 degrees of freedom: mean 63, sd ~ 11.2; 6 sd bound
    assert chi2 < 63 + 6 * math.sqrt(2 * 63)


def test_sampler_deterministic_and_seed_sensitive():
    p = np.full(1 << 10, 1.0 / (1 << 10))
    a = oracle.sample(p, seed=99, shots=1000)
    b = oracle.sample(p, seed=99, shots=1000)
    c = oracle.sample(p, seed=100, shots=1000)
    np.testing.assert_array_equal(a, b)
    assert np.mean(a == c) < 0.05


def test_ghz_all_zero_marginal_binomial():
    """Section V-B check: the all-zero GHZ frequency lies within a few binomial SEs of 1/2."""
    n = 10
    psi = oracle.run(n, W.ghz(n))
    S = 1000
    s = oracle.sample(oracle.probs(psi), seed=2024, shots=S)
    assert set(np.unique(s).tolist()) <= {0, (1 << n) - 1}
    f0 = np.mean(s == 0)
    se = math.sqrt(0.25 / S)
    assert abs(f0 - 0.5) <= 4 * se


# ---------------------------------------------------------------- fusion reference
def test_block_matrix_special_cases():
    rng = np.random.default_rng(9)
    A, B = W.haar_su2(rng), W.haar_su2(rng)
    ga = W.Gate("a", (3,), A)
    gb = W.Gate("b", (7,), B)
    # disjoint single-qubit gates on tuple (3, 7): q_0 = 3 is the low bit
    np.testing.assert_allclose(oracle.block_matrix([ga, gb], (3, 7)), np.kron(B, A), atol=1e-14)
    np.testing.assert_allclose(oracle.block_matrix([ga, gb], (7, 3)), np.kron(A, B), atol=1e-14)
    # two gates on one qubit: later gate on the left
    gc = W.Gate("c", (3,), B)
    np.testing.assert_allclose(oracle.block_matrix([ga, gc], (3,)), B @ A, atol=1e-14)


def test_block_matrix_equals_unfused_application():
    n = 9
    rng = np.random.default_rng(10)
    gates = W.brickwork(n, 3, seed=1)[:14]
    tup = sorted({q for g in gates for q in g.targets})
    if len(tup) > 7:
        gates = [g for g in gates if all(q in tup[:7] for q in g.targets)]
        tup = sorted({q for g in gates for q in g.targets})
    psi = rand_state(n, rng)
    ref = oracle.run(n, gates, psi.copy())
    M = oracle.block_matrix(gates, tup)
    got = psi.copy()
    oracle.apply_gate(got, M, tup)
    m = oracle.metrics(ref, got)
    assert m["infidelity"] < 1e-12 and m["max_abs"] < 1e-12


def test_metrics_definitions():
    o = np.array([1, 0, 0, 0], dtype=np.complex128)
    g = np.array([math.cos(0.1), math.sin(0.1), 0, 0], dtype=np.complex128)
    m = oracle.metrics(o, g)
    assert abs(m["fidelity"] - math.cos(0.1) ** 2) < 1e-15
    assert abs(m["max_abs"] - max(1 - math.cos(0.1), math.sin(0.1))) < 1e-15
    assert abs(m["rel_l2"] - math.hypot(1 - math.cos(0.1), math.sin(0.1))) < 1e-15
    # a global phase does not change the fidelity
    assert abs(oracle.metrics(o, 1j * o)["fidelity"] - 1) < 1e-15


# ---------------------------------------------------------------- MLP reference
def _mlp_params(rng, nin=10, h=8):
    return [rng.standard_normal((nin, h)) * 0.5, rng.standard_normal(h) * 0.1,
            rng.standard_normal((h, h)) * 0.5, rng.standard_normal(h) * 0.1,
            rng.standard_normal((h, 1)) * 0.5, rng.standard_normal(1) * 0.1]


def test_mlp_gradient_finite_differences():
    rng = np.random.default_rng(11)
    P = _mlp_params(rng)
    x = rng.standard_normal((16, 10))
    t = rng.standard_normal(16)
    loss, grads = oracle.mlp_loss_grad(P, x, t)
    h = 1e-6
    for pi, p in enumerate(P):
        flat = p.reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = oracle.mlp_loss_grad(P, x, t)
            flat[idx] = old - h
            lm, _ = oracle.mlp_loss_grad(P, x, t)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = grads[pi].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (pi, idx, fd, an)


def test_mlp_forward_small_closed_form():
    # one input, identity-like weights: y = relu(relu(x) ) summed
    P = [np.eye(2), np.zeros(2), np.eye(2), np.zeros(2), np.ones((2, 1)), np.array([0.5])]
    y, _ = oracle.mlp_forward(P, np.array([[1.0, -2.0], [3.0, 4.0]]))
    np.testing.assert_allclose(y, [1.5, 7.5])


def test_adam_first_step_is_lr_times_sign():
    p = [np.array([1.0, -2.0, 0.5])]
    g = [np.array([0.3, -4.0, 1e-3])]
    m = [np.zeros(3)]
    v = [np.zeros(3)]
    newp, newm, newv = oracle.adam_step(p, g, m, v, t=1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(newp[0], p[0] - 0.01 * np.sign(g[0]), atol=1e-15)
    np.testing.assert_allclose(newm[0], 0.1 * g[0])
    np.testing.assert_allclose(newv[0], 0.001 * g[0] ** 2)


def _ry_rz_product_state(thetas, phis):
    """Closed form of RY(theta_q) then RZ(phi_q) on every qubit of |0...0>, written out per qubit:
    qubit q is (cos(theta/2) e^{-i phi/2}, sin(theta/2) e^{+i phi/2}); index bit q = qubit q."""
    psi = np.ones(1, dtype=np.complex128)
    for th, ph in zip(thetas, phis):
        one = np.array([math.cos(th / 2) * np.exp(-0.5j * ph), math.sin(th / 2) * np.exp(0.5j * ph)])
        psi = np.kron(one, psi)  # the new qubit is the next higher index bit
    return psi


@pytest.mark.parametrize("n", [1, 3, 6])
def test_probs_of_complex_product_state_closed_form(n):
    """p_x = |psi_x|^2 (Section IV-E) on amplitudes with nonzero imaginary parts: for the RY-RZ product
    state, p_x = prod_q cos^2(theta_q/2) or sin^2(theta_q/2) by bit x_q, independent of the phases.
    Re^2 alone, |psi| or a dropped imaginary part all miss it."""
    rng = np.random.default_rng(40 + n)
    th = rng.uniform(0.2, 2.9, n)
    ph = rng.uniform(0.3, 2.8, n)
    psi = _ry_rz_product_state(th, ph)
    assert np.abs(psi.imag).max() > 0.05  # the pin needs complex amplitudes
    want = np.ones(1 << n)
    for x in range(1 << n):
        for q in range(n):
            want[x] *= math.sin(th[q] / 2) ** 2 if (x >> q) & 1 else math.cos(th[q] / 2) ** 2
    got = oracle.probs(psi)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)
    assert abs(got.sum() - 1.0) < 1e-14
    # the same state from the gate-by-gate oracle (RY then RZ as 2x2 gates)
    gates = []
    for q in range(n):
        c, s = math.cos(th[q] / 2), math.sin(th[q] / 2)
        gates.append(W.Gate("ry", (q,), np.array([[c, -s], [s, c]], dtype=np.complex128)))
        gates.append(W.Gate("rz", (q,), np.diag([np.exp(-0.5j * ph[q]), np.exp(0.5j * ph[q])]), True))
    np.testing.assert_allclose(oracle.probs(oracle.run(n, gates)), want, rtol=0, atol=1e-14)


def test_probs_single_amplitude_values():
    """p = re^2 + im^2 entry by entry on hand-picked amplitudes (3+4i -> 25, -2i -> 4, 0.5-0.5i -> 0.5)."""
    psi = np.array([3 + 4j, -2j, 0.5 - 0.5j, 0.0], dtype=np.complex128)
    np.testing.assert_array_equal(oracle.probs(psi), [25.0, 4.0, 0.5, 0.0])
