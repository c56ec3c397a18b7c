"""Full-size (N=30) checks in the launch configuration bench.py times.

* the headline circuit (brickwork depth 24 + QFT30, greedy fusion k<=5)
  against complex128 oracle amplitudes stored by
  tests/golden/make_headline_n30_golden.py at 2050 seeded indices;
* QFT30 of a basis state against its closed form at sampled indices;
* echo: the fused circuit followed by its fused inverse returns |0...0>.
"""
import math
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

N = 30
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "headline_n30_amplitudes.txt")


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


def logical_to_physical(x, layout):
    x = np.asarray(x, dtype=np.int64)
    y = np.zeros_like(x)
    for q, pos in enumerate(layout):
        y |= ((x >> q) & 1) << int(pos)
    return y


def gather(sv, logical_idx):
    import torch
    phys = logical_to_physical(logical_idx, sv.layout())
    sv.sync()
    return sv.amps[torch.from_numpy(phys).to(sv.amps.device)].cpu().numpy().astype(np.complex128)


def read_golden():
    idx, vals, norm = [], [], None
    with open(GOLDEN) as f:
        for ln in f:
            if ln.startswith("# norm"):
                norm = float(ln.split()[2])
            if ln.startswith("#") or not ln.strip():
                continue
            i, re, im = ln.split()
            idx.append(int(i))
            vals.append(complex(float(re), float(im)))
    return np.array(idx, dtype=np.int64), np.array(vals, dtype=np.complex128), norm


def test_headline_n30_against_oracle_samples(P):
    idx, ref, onorm = read_golden()
    assert abs(onorm - 1) < 1e-10
    gates = W.headline(N, 24, 0)
    plan = P.Plan.greedy(N, gates, 5)
    sv = P.StateVector(N)
    say("headline plan blocks", len(plan))
    plan.run(sv)
    got = gather(sv, idx)
    d = np.abs(got - ref)
    rel = float(np.sqrt(np.sum(d ** 2) / np.sum(np.abs(ref) ** 2)))
    say("headline n30: max|d| %.3e  rel_l2(sample) %.3e  typical |amp| %.3e" % (d.max(), rel, np.abs(ref).mean()))
    assert d.max() <= 1e-5
    # the absolute bar says little for amplitudes of size ~3e-5: every sampled
    # amplitude is also held to 1e-5 of the largest one (measured ~1e-6)
    assert d.max() <= 1e-5 * np.abs(ref).max()
    assert rel <= 1e-5
    nrm = sv.norm()
    assert abs(nrm - 1) <= 1e-5
    sv.close()


def test_qft30_basis_state_closed_form(P):
    x = 0x2A5F1C3D & ((1 << N) - 1)
    plan = P.Plan.greedy(N, W.basis_prep(N, x) + W.qft(N), 5)
    sv = P.StateVector(N)
    plan.run(sv)
    rng = np.random.default_rng(7)
    ys = np.unique(np.concatenate([rng.integers(0, 1 << N, 4096), [0, 1, (1 << N) - 1]]))
    got = gather(sv, ys)
    # phase = 2 pi x y / 2^N, reduced exactly in integers before the float conversion
    ph = (np.uint64(x) * ys.astype(np.uint64)) & np.uint64((1 << N) - 1)
    ref = np.exp(2j * np.pi * ph.astype(np.float64) / (1 << N)) / math.sqrt(1 << N)
    d = np.abs(got - ref)
    say("qft30: max|d| %.3e rel %.3e" % (d.max(), d.max() * math.sqrt(1 << N)))
    assert d.max() <= 1e-5
    assert d.max() * math.sqrt(1 << N) <= 1e-3  # relative to the amplitude magnitude
    sv.close()


def test_echo_n30(P):
    gates = W.headline(N, 24, 0)
    fwd = P.Plan.greedy(N, gates, 5)
    inv = P.Plan.greedy(N, W.inverse(gates), 5)
    sv = P.StateVector(N)
    fwd.run(sv)
    inv.run(sv)
    a0 = gather(sv, np.array([0]))[0]
    f0 = abs(a0) ** 2
    say("echo n30: |<0|psi>|^2 = %.9f" % f0)
    assert f0 >= 1 - 1e-5
    s = sv.sample(99, 1000)
    assert np.all(s == 0)
    sv.close()


@pytest.mark.parametrize("n", [33, 34])
def test_largest_states_dispatch_limits(P, n):
    """N=33/34: grids past 2^32 work-items are capped (shuffle, CDF block totals, MFMA tiles, diagonal)."""
    import torch
    sv = P.StateVector(n)
    H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2)
    sv.apply(H, [0])          # shuffle lowering, bit 0
    sv.apply(H, [5])          # shuffle lowering, bit 5
    sv.apply(W.cnot(), [0, n - 1])
    # MFMA sweep with more tiles than workgroups (k=4: 2^(n-11) tiles) and a
    # grid-strided diagonal sweep, each undone by its inverse
    rng = np.random.default_rng(n)
    u = W.random_dense(n, 4, rng, (1, 2, 3, n - 1)).matrix
    d = np.diag(np.exp(1j * rng.uniform(0, 2 * np.pi, 8)))
    for m, t in ((u, [1, 2, 3, n - 1]), (d, [0, 17, n - 1])):
        sv.apply(m, t)
        sv.apply(m.conj().T, t)
    assert sv.stats()["by_variant"][P._native.VARIANT["mfma"]] >= 2
    assert sv.stats()["by_variant"][P._native.VARIANT["diag"]] >= 2
    nrm = sv.norm()
    assert abs(nrm - 1) < 1e-5
    s = sv.sample(3, 4000)
    bit0 = (s & 1).astype(np.int64)
    top = ((s >> np.uint64(n - 1)) & np.uint64(1)).astype(np.int64)
    assert np.all(bit0 == top)
    assert np.all((s & ~np.uint64(1 | 32 | (1 << (n - 1)))) == 0)
    assert 0.4 < bit0.mean() < 0.6 and 0.4 < ((s >> np.uint64(5)) & np.uint64(1)).astype(np.int64).mean() < 0.6
    amps = gather(sv, np.array([0, 1 | (1 << (n - 1)), 32, 1]))
    np.testing.assert_allclose(amps, [0.5, 0.5, 0.5, 0.0], atol=2e-6)
    sv.close()
    del sv
    torch.cuda.empty_cache()


def test_probs_large_state_exact(P):
    """FP64 probabilities at N=26 (the large-state streaming order), physical and logical."""
    import torch
    n = 26
    rng = np.random.default_rng(26)
    sv = P.StateVector(n)
    for q in (0, 3, 9, 17, 25):
        sv.apply(W.haar_su2(rng), [q])
    sv.apply(W.cnot(), [3, 24])
    layout = list(range(n))
    layout[1], layout[20] = layout[20], layout[1]
    sv.permute_layout(layout)
    a = sv.amps
    want = a.real.double() ** 2 + a.imag.double() ** 2
    p_phys = sv.probs(logical=False)
    assert torch.equal(p_phys, want)
    p_log = sv.probs(logical=True)
    idx = torch.arange(1 << n, device=a.device, dtype=torch.int64)
    phys = torch.zeros_like(idx)
    for q, pos in enumerate(sv.layout()):
        phys |= ((idx >> q) & 1) << int(pos)
    assert torch.equal(p_log, want[phys])
    assert abs(float(p_phys.sum()) - 1) < 1e-5
    sv.close()


def test_maximum_state_n35_closed_form(P):
    """N=35, the largest state the interface accepts (256 GiB): a k=5 MFMA sweep on the top five
    qubits, a shuffle sweep on qubit 0 and a diagonal CZ give a state whose 64 nonzero amplitudes
    have a closed form; the FP64 norm and the sampler's support are checked too."""
    import torch
    n = 35
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    need = (8 << n) + (1 << 30)
    if free < need:
        pytest.skip("N=35 needs %.0f GiB of free device memory, %.0f GiB free" % (need / 2**30, free / 2**30))
    say("n=35: %.0f GiB free" % (free / 2**30))
    rng = np.random.default_rng(35)
    top = (30, 31, 32, 33, 34)
    G = W.random_dense(n, 5, rng, top).matrix
    H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2)
    sv = P.StateVector(n)
    sv.apply(G, list(top))    # MFMA tile sweep, targets on the five highest bits
    sv.apply(H, [0])          # wave-shuffle sweep on bit 0
    sv.apply(W.cz(), [0, 30])  # streaming diagonal sweep
    st = sv.stats()["by_variant"]
    assert st[P._native.VARIANT["mfma"]] == 1 and st[P._native.VARIANT["shuffle"]] == 1
    assert st[P._native.VARIANT["diag"]] == 1
    xs, want = [], []
    for r in range(32):
        for b0 in range(2):
            x = b0 | (r << 30)
            sign = -1.0 if (b0 and (r & 1)) else 1.0
            xs.append(x)
            want.append(sign * G[r, 0] / math.sqrt(2))
    got = gather(sv, np.array(xs, dtype=np.int64))
    err = np.abs(got - np.array(want)).max()
    nrm = sv.norm()
    say("n=35 max|damp| %.2e on the 64 nonzero amplitudes, norm - 1 = %.2e" % (err, nrm - 1))
    assert err < 1e-6 and abs(nrm - 1) < 1e-5
    s = sv.sample(35, 2000)
    support = np.uint64(1 | (31 << 30))
    assert np.all((s & ~support) == 0)
    sv.close()
    del sv
    torch.cuda.empty_cache()
