"""Edge cases of the C-ABI on the GPU: bad arguments on a live handle, empty
plans, gates over every qubit of the state (k = N), single-qubit states and
zero shots.  Results are checked against the oracle as in the parity tests."""
import ctypes

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


def test_apply_rejects_bad_arguments(P):
    import paper_2608_16940_amd._native as N
    lib = P.lib()
    n = 6
    sv = P.StateVector(n)
    m = np.eye(4, dtype=np.complex128)
    cases = [(m, (0, 0)),            # duplicate target
             (m, (0, n)),            # target outside the state
             (m, (-1, 2)),           # negative target
             (np.eye(1 << 9, dtype=np.complex128), tuple(range(9)))]  # wider than the state and SV_MAX_K
    for mat, t in cases:
        with pytest.raises(P.SvError) as e:
            sv.apply(mat, t)
        assert e.value.code == N.SV_ERR_ARG, t
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    t0 = np.zeros(1, dtype=np.int32)
    assert lib.sv_apply_fused(sv._h, m.view(np.float64).ctypes.data_as(dp), t0.ctypes.data_as(ip), 0) == N.SV_ERR_ARG
    assert lib.sv_apply_fused(sv._h, None, t0.ctypes.data_as(ip), 1) == N.SV_ERR_ARG
    assert lib.sv_apply_fused(None, m.view(np.float64).ctypes.data_as(dp), t0.ctypes.data_as(ip), 1) == N.SV_ERR_ARG
    # the state is untouched by rejected calls
    assert abs(sv.amps[0].item() - 1) == 0 and abs(sv.norm() - 1) < 1e-12
    sv.close()


def test_empty_plan_and_zero_shots(P):
    n = 12
    plan = P.Plan.greedy(n, [], 5)
    assert len(plan) == 0
    sv = P.StateVector(n)
    plan.run(sv)
    assert sv.sample(7, 0).size == 0
    s = sv.sample(7, 100)
    assert np.all(s == 0)
    assert abs(sv.amps[0].item() - 1) == 0
    sv.close()


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_gate_over_every_qubit(P, n):
    """k = N: one dense gate on all qubits (targets in a shuffled order), then a diagonal one."""
    rng = np.random.default_rng(n)
    t = tuple(int(x) for x in rng.permutation(n))
    g = W.random_dense(n, n, rng, t)
    d = np.diag(np.exp(1j * rng.uniform(0, 2 * np.pi, 1 << n)))
    sv = P.StateVector(n)
    sv.apply(g.matrix, g.targets)
    sv.apply(d, t[::-1])
    ref = oracle.zero_state(n)
    oracle.apply_gate(ref, g.matrix, list(g.targets))
    oracle.apply_gate(ref, d, list(t[::-1]))
    got = oracle.decode(sv.physical_state(), sv.layout())
    m = oracle.metrics(ref, got)
    assert m["infidelity"] < 1e-5 and m["max_abs"] < 1e-5, (n, m)
    p = sv.probs().cpu().numpy()
    assert np.abs(p - oracle.probs(ref)).max() < 1e-6
    shots = sv.sample(11, 500)
    np.testing.assert_array_equal(shots, oracle.sample(p, 11, 500))
    sv.close()


@pytest.mark.parametrize("n", [14, 23])
def test_copy_out_physical_and_logical(P, n):
    """sv_copy_out: physical order is the stored state; logical order decodes y_{L(q)} = x_q on the host
    (n = 23: two passes through the 2^22-amplitude staging buffer) and leaves the layout and the
    device state unchanged."""
    rng = np.random.default_rng(n)
    gates = [W.random_dense(n, k, rng) for k in (1, 2, 3, 5, 2)]
    sv = P.StateVector(n)
    for g in gates:
        sv.apply(g.matrix, g.targets)
    perm = rng.permutation(n).astype(np.int32)
    sv.permute_layout(perm)
    phys = sv.copy_out(logical=False)
    np.testing.assert_array_equal(phys, sv.amps.cpu().numpy())
    log = sv.copy_out(logical=True)
    np.testing.assert_array_equal(log.astype(np.complex128), oracle.decode(phys.astype(np.complex128), perm))
    assert list(sv.layout()) == list(perm)
    m = oracle.metrics(oracle.run(n, gates), log.astype(np.complex128))
    assert m["infidelity"] < 1e-5 and m["max_abs"] < 1e-5
    sv.close()


def test_sampler_rejects_bad_probabilities(P):
    """sv_sample_probs: entries must be finite and in [0, 4) and sum to less than 4 (the fixed-point
    total floor(p * 2^62) summed must fit in 64 bits); the check runs on the GPU during the CDF build."""
    import torch
    import paper_2608_16940_amd._native as N
    n = 11
    p = np.full(1 << n, 1.0 / (1 << n))
    for i, v in [(3, -1e-300), (7, np.nan), (0, np.inf), (1, 4.0)]:
        q = p.copy()
        q[i] = v
        with pytest.raises(P.SvError) as e:
            P.sample_probs(torch.from_numpy(q).cuda(), 1, 10)
        assert e.value.code == N.SV_ERR_ARG, (i, v)
    # two entries of 2.0: each is 2^63 in fixed point, the total is exactly 2^64 and wraps
    q = np.zeros(1 << n)
    q[[5, 900]] = 2.0
    with pytest.raises(P.SvError) as e:
        P.sample_probs(torch.from_numpy(q).cuda(), 1, 10)
    assert e.value.code == N.SV_ERR_ARG
    # just under the bound: valid, and only the two nonzero indices are drawn
    q[900] = np.nextafter(2.0, 0.0)
    s = P.sample_probs(torch.from_numpy(q).cuda(), 1, 1000)
    assert set(np.unique(s).tolist()) <= {5, 900}
    np.testing.assert_array_equal(s, oracle.sample(q, 1, 1000))
    # unnormalised but valid input samples as the oracle does
    q = np.random.default_rng(3).random(1 << n) * 3.9 / (1 << n)
    np.testing.assert_array_equal(P.sample_probs(torch.from_numpy(q).cuda(), 9, 777), oracle.sample(q, 9, 777))


def test_sample_rejects_state_outside_the_fixed_point_range(P):
    """sv_sample on a state whose norm is 4 or more, or with a NaN amplitude, is SV_ERR_STATE
    (unitarity is not checked by the gate calls, so the sampler guards its fixed-point total)."""
    import torch
    import paper_2608_16940_amd._native as N
    n = 10
    sv = P.StateVector(n)
    sv.amps[0] = 2.0  # ||psi||^2 = 4
    torch.cuda.synchronize()
    with pytest.raises(P.SvError) as e:
        sv.sample(1, 10)
    assert e.value.code == N.SV_ERR_STATE
    sv.amps[0] = complex(1.0, float("nan"))
    torch.cuda.synchronize()
    with pytest.raises(P.SvError) as e:
        sv.sample(1, 10)
    assert e.value.code == N.SV_ERR_STATE
    sv.amps[0] = 1.9
    torch.cuda.synchronize()
    assert np.all(sv.sample(1, 50) == 0)
    sv.close()
