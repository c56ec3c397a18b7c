"""GPU parity of the density-matrix path (Section IV-B) against the oracle.

The GPU applies each channel as the 2k-target superoperator on vec(rho)
through the same kernels as state vectors; the oracle applies
sum_i E_i rho E_i^dagger with dense matrices.  Bars: max |delta rho_ij| and
max |delta p_x| <= 1e-5 (the FP32 amplitude bar of the state-vector path),
trace and purity within 1e-5; sampling bit for bit on the same FP64
probabilities.  Full-size cases (N = 15, 8 GiB, and the maximum N = 17,
128 GiB) are checked on sampled entries against closed-form product states,
and by invariants that hold at any size.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import density as D
import workloads as W
from workloads import noise as Nz

pytestmark = pytest.mark.gpu

TOL = 1e-5


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


def random_channels(n, count, rng):
    out = []
    for i in range(count):
        kind = i % 8
        if kind == 0:
            k = min(n, 1 + i % 3)
            out.append(Nz.unitary(W.random_dense(n, k, rng)))
        elif kind == 1:
            k = min(n, 1 + (i // 8) % 2)
            t = tuple(int(q) for q in rng.choice(n, k, replace=False))
            out.append(Nz.random_channel(t, 2 + i % 3, rng))
        elif kind == 2:
            out.append(Nz.amplitude_damping(int(rng.integers(n)), float(rng.uniform(0.05, 0.6))))
        elif kind == 3:
            out.append(Nz.dephasing(int(rng.integers(n)), float(rng.uniform(0.05, 0.5))))
        elif kind == 4 and n >= 2:
            t = tuple(int(q) for q in rng.choice(n, 2, replace=False))
            out.append(Nz.depolarizing(t, float(rng.uniform(0.01, 0.2))))
        elif kind == 5 and n >= 2:
            t = tuple(int(q) for q in rng.choice(n, 2, replace=False))
            out.append(Nz.unitary(W.Gate("cz", t, W.cz(), diag=True)))
        elif kind == 6 and n >= 2:
            t = tuple(int(q) for q in rng.choice(n, 2, replace=False))
            out.append(Nz.unitary(W.Gate("swap", t, W.swap())))
        else:
            out.append(Nz.unitary(W.Gate("su2", (int(rng.integers(n)),), W.haar_su2(rng))))
    return out


def compare(dm, ref, what):
    got = dm.matrix().cpu().numpy().astype(np.complex128)
    err = np.abs(got - ref).max()
    p = dm.probs().cpu().numpy()
    perr = np.abs(p - np.clip(D.probs(ref), 0, None)).max()
    tr, pur = dm.trace(), dm.purity()
    say(what, "max|drho| %.2e max|dp| %.2e trace %.9f purity %.6f (oracle %.6f)" % (err, perr, tr, pur, D.purity(ref)))
    assert err <= TOL and perr <= TOL
    assert abs(tr - D.trace(ref)) <= TOL and abs(pur - D.purity(ref)) <= TOL


@pytest.mark.parametrize("n,count", [(2, 16), (3, 24), (5, 32), (7, 24)])
def test_channels_match_oracle(P, n, count):
    rng = np.random.default_rng(100 + n)
    chans = random_channels(n, count, rng)
    dm = P.DensityMatrix(n)
    dm.apply_channels(chans)
    compare(dm, D.run(n, chans), "n=%d channels=%d" % (n, count))
    st = dm.stats()
    assert st["layout_only"] >= 1  # the SWAP channels only relabel vector qubits
    dm.close()


def test_initial_state_and_reset(P):
    dm = P.DensityMatrix(4)
    compare(dm, D.zero(4), "initial")
    dm.apply_channel(Nz.depolarizing((1,), 0.5).kraus, (1,))
    dm.reset()
    compare(dm, D.zero(4), "reset")
    dm.close()


@pytest.mark.parametrize("planner", ["greedy", "dp", "paper", "learned"])
def test_fused_superoperator_plans(P, planner):
    n = 5
    chans = Nz.noisy_brickwork(n, 3, 0.05, seed=7)
    gates = P.superop_gates(n, chans)
    if planner == "greedy":
        plan = P.Plan.greedy(2 * n, gates, 6)
    elif planner == "dp":
        plan = P.Plan.dp(2 * n, gates, 6, 8, 64, reorder=True)
    elif planner == "learned":
        from paper_2608_16940_amd import costmodel as C
        plan = P.Plan.learned(2 * n, gates, C.load()[0])
    else:
        plan = P.Plan.paper(2 * n, gates)
    assert len(plan) < len(gates)
    dm = P.DensityMatrix(n)
    plan.run(dm)
    compare(dm, D.run(n, chans), "plan %s: %d blocks for %d channels" % (planner, len(plan), len(chans)))
    dm.close()


def test_layout_permutation_and_probs_through_layout(P):
    n = 6
    rng = np.random.default_rng(5)
    chans = random_channels(n, 16, rng)
    dm = P.DensityMatrix(n)
    dm.apply_channels(chans)
    ref = D.run(n, chans)
    perm = rng.permutation(2 * n).astype(np.int32)
    dm.permute_layout(perm)
    assert list(dm.layout()) == list(perm)
    p = dm.probs().cpu().numpy()
    assert np.abs(p - np.clip(D.probs(ref), 0, None)).max() <= TOL
    assert abs(dm.trace() - 1.0) <= TOL
    compare(dm, ref, "after permute")  # matrix() moves the layout back to identity
    dm.close()


def test_sampling_bit_exact(P):
    n = 6
    rng = np.random.default_rng(9)
    chans = random_channels(n, 20, rng)
    dm = P.DensityMatrix(n)
    dm.apply_channels(chans)
    dm.permute_layout(rng.permutation(2 * n).astype(np.int32))
    p = dm.probs().cpu().numpy()
    for seed, shots in [(1, 1000), (0x5EED, 4097)]:
        got = dm.sample(seed, shots)
        want = oracle.sample(p, seed, shots)
        np.testing.assert_array_equal(got, want)
    assert (got < (1 << n)).all()
    dm.close()


def test_operator_sums_that_are_not_trace_preserving(P):
    import paper_2608_16940_amd._native as N
    n = 3
    dm = P.DensityMatrix(n)
    proj1 = np.diag([0, 1]).astype(np.complex128)
    dm.apply_channel([proj1], (2,))  # project |0..0> onto qubit 2 = 1: rho = 0
    assert dm.trace() == 0.0
    with pytest.raises(P.SvError) as e:
        dm.sample(1, 10)
    assert e.value.code == N.SV_ERR_STATE
    dm.close()


def test_argument_errors(P):
    import ctypes
    import paper_2608_16940_amd._native as N
    lib = P.lib()
    dm = P.DensityMatrix(3)
    eye = [np.eye(2)]
    for kraus, targets in [([np.eye(32)], (0, 1, 2, 0, 1)), (eye, (3,)), (eye, (-1,)), ([np.eye(4)], (1, 1))]:
        with pytest.raises(P.SvError) as e:
            dm.apply_channel(kraus, targets)
        assert e.value.code == N.SV_ERR_ARG
    sv = P.StateVector(6)
    out = ctypes.c_double()
    assert lib.sv_dm_trace(sv._h, ctypes.byref(out)) == N.SV_ERR_ARG
    assert lib.sv_dm_qubits(sv._h) == 0 and lib.sv_dm_qubits(dm._h) == 3
    assert lib.sv_dm_state_bytes(1) == 0 and lib.sv_dm_state_bytes(18) == 0
    h = ctypes.c_void_p()
    assert lib.sv_dm_alloc(ctypes.byref(h), 18, ctypes.c_void_p(sv.amps.data_ptr()), 8 << 12,
                           ctypes.c_void_p(sv.ws.data_ptr()), sv.ws.numel(), None) == N.SV_ERR_ARG
    sv.close()
    dm.close()


def product_channels(n, rng):
    """Per qubit: a Haar SU(2), amplitude damping, depolarizing; rho is the tensor product of the qubits' rho_q."""
    chans, per_qubit = [], []
    for q in range(n):
        u = W.haar_su2(rng)
        ad = float(rng.uniform(0.05, 0.5))
        dp = float(rng.uniform(0.01, 0.2))
        cq = [Nz.unitary(W.Gate("su2", (q,), u)), Nz.amplitude_damping(q, ad), Nz.depolarizing((q,), dp)]
        chans += cq
        local = [Nz.unitary(W.Gate("su2", (0,), u)), Nz.amplitude_damping(0, ad), Nz.depolarizing((0,), dp)]
        per_qubit.append(D.run(1, local))
    return chans, per_qubit


def product_entry(per_qubit, r, c):
    v = 1.0 + 0j
    for q, rq in enumerate(per_qubit):
        v *= rq[(r >> q) & 1, (c >> q) & 1]
    return v


@pytest.mark.parametrize("n", [15, 17])
def test_full_size_product_state(P, n):
    """N = 15 (8 GiB vec) and the maximum N = 17 (128 GiB): sampled entries against the product form."""
    import torch
    torch.cuda.empty_cache()
    rng = np.random.default_rng(n)
    chans, per_qubit = product_channels(n, rng)
    dm = P.DensityMatrix(n)
    say("full-size density matrix n=%d, %d channels" % (n, len(chans)))
    dm.apply_channels(chans)
    d = 1 << n
    rows = rng.integers(0, d, 4096)
    cols = rng.integers(0, d, 4096)
    rows[:16] = cols[:16] = rng.integers(0, d, 16)  # some diagonal entries
    idx = torch.as_tensor(rows + d * cols, device=dm.amps.device)
    dm.sync()
    got = dm.amps[idx].cpu().numpy().astype(np.complex128)  # identity layout: no relabel in this circuit
    assert list(dm.layout()) == list(range(2 * n))
    want = np.array([product_entry(per_qubit, int(r), int(c)) for r, c in zip(rows, cols)])
    err = np.abs(got - want).max()
    tr, pur = dm.trace(), dm.purity()
    want_pur = float(np.prod([D.purity(r) for r in per_qubit]))
    say("n=%d max|drho| %.2e on 4096 sampled entries, trace %.8f, purity %.3e (product %.3e)" %
        (n, err, tr, pur, want_pur))
    assert err <= TOL and abs(tr - 1.0) <= TOL and abs(pur - want_pur) <= TOL
    p = dm.probs()
    xs = rng.integers(0, d, 512)
    pw = np.array([product_entry(per_qubit, int(x), int(x)).real for x in xs])
    assert np.abs(p[torch.as_tensor(xs, device=p.device)].cpu().numpy() - pw).max() <= TOL
    shots = dm.sample(3, 2000)
    np.testing.assert_array_equal(shots, oracle.sample(p.cpu().numpy(), 3, 2000))
    dm.close()


def test_full_size_entangling_channels_invariants(P):
    """N = 15 with two-qubit random channels and CZ: trace, Hermiticity and purity <= 1 on sampled entries."""
    import torch
    n = 15
    rng = np.random.default_rng(33)
    chans = []
    for q in range(n - 1):
        chans.append(Nz.unitary(W.Gate("su2", (q,), W.haar_su2(rng))))
        chans.append(Nz.random_channel((q, q + 1), 2, rng))
        chans.append(Nz.unitary(W.Gate("cz", (q + 1, q), W.cz(), diag=True)))
    dm = P.DensityMatrix(n)
    dm.apply_channels(chans)
    say("n=15 entangling: %d channels, stats %s" % (len(chans), dm.stats()))
    tr, pur = dm.trace(), dm.purity()
    assert abs(tr - 1.0) <= TOL and 0 < pur <= 1 + TOL
    rho = dm.matrix()
    d = 1 << n
    r = torch.as_tensor(rng.integers(0, d, 4096), device=rho.device)
    c = torch.as_tensor(rng.integers(0, d, 4096), device=rho.device)
    a = rho[r, c].cpu().numpy()
    b = rho[c, r].cpu().numpy()
    assert np.abs(a - b.conj()).max() <= 1e-6
    diag = rho[r, r].cpu().numpy()
    assert np.abs(diag.imag).max() <= 1e-6 and diag.real.min() >= -1e-6
    dm.close()


def test_bound_superoperator_plan_and_graph_replays(P):
    """A plan over superoperators bound to a density handle: eager run, bound run and HIP-graph
    replays (with eager work between them) give bit-identical vec(rho), equal to the oracle."""
    from paper_2608_16940_amd import costmodel as C
    n = 6
    rng = np.random.default_rng(77)
    chans = Nz.noisy_brickwork(n, 3, 0.02, seed=11) + random_channels(n, 12, rng)
    plan = P.Plan.learned(2 * n, P.superop_gates(n, chans), C.load()[0])
    ref_dm = P.DensityMatrix(n)
    plan.run(ref_dm)
    ref = ref_dm.physical_state()
    dm = P.DensityMatrix(n)
    bound = plan.bind(dm)
    bound.run()
    np.testing.assert_array_equal(dm.physical_state(), ref)
    for rep in range(3):
        dm.reset()
        bound.run_graph()
        np.testing.assert_array_equal(dm.physical_state(), ref)
        assert abs(dm.trace() - 1.0) <= TOL  # eager work between replays
        dm.sample(rep, 50)
    assert list(dm.layout()) == list(ref_dm.layout())
    compare(dm, D.run(n, chans), "bound learned plan, %d blocks" % len(plan))
    bound.close()
    dm.close()
    ref_dm.close()


@pytest.mark.parametrize("p_noise", [0.0, 1e-3])
def test_bench_configuration_n15(P, p_noise):
    """The density bench's configuration (N=15, noisy brickwork depth 8, learned plan over
    superoperators).  With p = 0 the result is |psi><psi| with psi from the state-vector oracle
    (compared at 4096 sampled entries); with the bench's p = 1e-3: trace, Hermiticity, purity."""
    import torch
    from paper_2608_16940_amd import costmodel as C
    n = 15
    chans = Nz.noisy_brickwork(n, 8, p_noise, 0)
    plan = P.Plan.learned(2 * n, P.superop_gates(n, chans), C.load()[0])
    dm = P.DensityMatrix(n)
    plan.run(dm)
    rho = dm.matrix()
    rng = np.random.default_rng(15)
    d = 1 << n
    r = rng.integers(0, d, 4096)
    c = rng.integers(0, d, 4096)
    got = rho[torch.as_tensor(r, device=rho.device), torch.as_tensor(c, device=rho.device)].cpu().numpy()
    tr, pur = dm.trace(), dm.purity()
    if p_noise == 0.0:
        psi = oracle.run(n, W.brickwork(n, 8, 0))
        want = psi[r] * psi[c].conj()
        err = np.abs(got - want).max()
        say("n=15 p=0 learned plan (%d blocks): max|drho| %.2e, trace %.8f, purity %.8f" % (len(plan), err, tr, pur))
        assert err <= TOL and abs(pur - 1) <= TOL
    else:
        back = rho[torch.as_tensor(c, device=rho.device), torch.as_tensor(r, device=rho.device)].cpu().numpy()
        say("n=15 p=1e-3 learned plan (%d blocks): trace %.8f, purity %.6f" % (len(plan), tr, pur))
        assert np.abs(got - back.conj()).max() <= 1e-6 and 0 < pur < 1
    assert abs(tr - 1) <= TOL
    dm.close()


@pytest.mark.parametrize("q,frac", [(4, 0.5), (1, 1.0)])
def test_dephasing_sweeps_only_the_off_diagonal_half(P, q, frac):
    """Dephasing's superoperator on (q, q + N) is diagonal and exactly 1 where the row and column bits
    agree, so the partial diagonal sweep visits only the half of vec(rho) where they differ, provided both
    positions can be held fixed (from bit 4 up); with q = 1 it sweeps the whole state.  Checked against
    the oracle and by the chunks the sweep visited."""
    n = 6
    rng = np.random.default_rng(40 + q)
    chans = [Nz.unitary(W.Gate("su2", (j,), W.haar_su2(rng))) for j in range(n)]
    chans += [Nz.depolarizing((0, 1), 0.1), Nz.amplitude_damping(2, 0.2), Nz.depolarizing((3, 5), 0.05)]
    dm = P.DensityMatrix(n)
    dm.set_relabel(False)
    dm.apply_channels(chans)
    assert list(dm.layout()) == list(range(2 * n))
    ch = Nz.dephasing(q, 0.3)
    c0 = dm.stats()["diag_chunks"]
    dm.apply_channel(ch.kraus, ch.targets)
    assert dm.stats()["diag_chunks"] - c0 == round(frac * (1 << (2 * n - 1)))
    compare(dm, D.run(n, chans + [ch]), "dephasing on %d after %d channels" % (q, len(chans)))
    dm.close()
