"""Batched persistent kernel against the oracle, per circuit."""
import math

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2608_16940_amd import batch as B
    return B


def test_batch_matches_oracle_every_circuit(B):
    circs = W.batch_family(96, seed=5, n_lo=3, n_hi=17, d_lo=1, d_hi=12)
    # two equal-structure circuits per size so packs of several circuits form
    circs += W.batch_family(40, seed=6, n_lo=10, n_hi=11, d_lo=4, d_hi=4)
    b = B.Batch(circs).allocate()
    z0 = b.run()
    worst = 0.0
    for i, (n, gates) in enumerate(circs):
        ref = oracle.run(n, gates)
        got = b.state(i)
        m = oracle.metrics(ref, got)
        worst = max(worst, m["max_abs"])
        assert m["infidelity"] <= 1e-5 and m["max_abs"] <= 1e-5 and m["rel_l2"] <= 1e-5, (i, n, m)
        assert abs(z0[i] - oracle.expect_z(ref, 0)) <= 1e-5, (i, z0[i])
    print("batch worst max|d|", worst, flush=True)


def test_batch_multi_pass_states(B):
    """States above 2^14 amplitudes run as LDS slice passes; reversed ladders and
    long-range CNOTs force many passes with changing slice qubit sets."""
    rng = np.random.default_rng(77)
    circs = []
    for n in (15, 16, 17, 18):
        gates = []
        for layer in range(5):
            for q in rng.permutation(n):
                gates.append(W.Gate("ry", (int(q),), W.ry(float(rng.uniform(0, 2 * np.pi)))))
            order = range(n - 2, -1, -1) if layer % 2 else range(n - 1)
            for q in order:
                gates.append(W.Gate("cnot", (q + 1, q) if layer % 2 else (q, q + 1), W.cnot()))
            gates.append(W.Gate("cnot", (0, n - 1), W.cnot()))
            gates.append(W.Gate("cnot", (n - 1, 3), W.cnot()))
            gates.append(W.Gate("rz", (n - 1,), W.rz(float(rng.uniform(0, 2 * np.pi)))))
        circs.append((n, gates))
    b = B.Batch(circs).allocate()
    z0 = b.run()
    for i, (n, gates) in enumerate(circs):
        ref = oracle.run(n, gates)
        m = oracle.metrics(ref, b.state(i))
        assert m["infidelity"] <= 1e-5 and m["max_abs"] <= 1e-5 and m["rel_l2"] <= 1e-5, (n, m)
        assert abs(z0[i] - oracle.expect_z(ref, 0)) <= 1e-5


def test_batch_configs_agree_and_autotune(B):
    circs = W.batch_family(64, seed=9, n_lo=10, n_hi=14, d_lo=6, d_hi=6)
    b = B.Batch(circs).allocate()
    z_def = b.run()
    s_def = [b.state(i) for i in range(len(circs))]
    cfg = np.ones(19, dtype=np.int32)
    z_one = b.run(cfg)
    np.testing.assert_allclose(z_one, z_def, atol=1e-6)
    for i in range(len(circs)):
        np.testing.assert_allclose(b.state(i), s_def[i], atol=1e-6)
    best, times = b.autotune(sample_per_size=8)
    assert all(best[n] >= 1 for n in range(1, 19))
    for n in range(10, 15):
        assert times[n] > 0 and best[n] & (best[n] - 1) == 0
        assert best[n] * (1 << n) <= (1 << 14) or best[n] == 1
    z_best = b.run(best)
    np.testing.assert_allclose(z_best, z_def, atol=1e-6)


def test_batch_closed_forms(B):
    # RY(theta) on qubit 0 then RZ on everything: <Z_0> = cos(theta)
    thetas = [0.0, 0.4, 1.3, 2.9, math.pi]
    circs = []
    for th in thetas:
        n = 9
        g = [W.Gate("ry", (0,), W.ry(th))] + [W.Gate("rz", (q,), W.rz(0.3 * q + 0.1)) for q in range(n)]
        circs.append((n, g))
    b = B.Batch(circs).allocate()
    z0 = b.run()
    np.testing.assert_allclose(z0, np.cos(thetas), atol=1e-6)


def test_batch_rejects_bad_input(B):
    from paper_2608_16940_amd import SvError
    with pytest.raises(SvError):
        B.Batch([(19, [])]).allocate().run()
    bad = [(4, [W.Gate("cnot", (1, 1), W.cnot())])]
    with pytest.raises(SvError):
        B.Batch(bad).allocate().run()


def test_batch_prepare_launch_matches_run(B):
    """Prepared once (records resident), launched twice: identical states and <Z_0> to sv_batch_run."""
    circs = W.batch_family(48, seed=11, n_lo=8, n_hi=16, d_lo=3, d_hi=9)
    b = B.Batch(circs).allocate()
    z_run = b.run()
    s_run = [b.state(i) for i in range(len(circs))]
    b.prepare()
    for _ in range(2):
        b.states.zero_()
        z = b.launch()
        np.testing.assert_array_equal(z, z_run)
        for i in range(len(circs)):
            np.testing.assert_array_equal(b.state(i), s_run[i])
    b.close_prepared()
