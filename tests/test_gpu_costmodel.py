"""Cost-model kernels on the GPU against the FP64 oracle, and the learned planner."""
import os
import sys
import time

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    import torch
    assert torch.cuda.is_available()
    from paper_2608_16940_amd import costmodel as C
    return C


def _data(B=300, seed=0):
    rng = np.random.default_rng(seed)
    from paper_2608_16940_amd import costmodel as C
    X = rng.standard_normal((B, C.NIN)).astype(np.float32)
    t = (np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2]).astype(np.float32)
    return X, t


def test_forward_backward_match_oracle(C):
    import torch
    X, t = _data()
    p = C.init_params(7)
    net = C.DeviceMLP(p, X.shape[0])
    Xd, td = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    y = net.forward(Xd).cpu().numpy()
    P64 = [a.astype(np.float64) for a in C.split_params(p)]
    yref, _ = oracle.mlp_forward(P64, X.astype(np.float64))
    np.testing.assert_allclose(y, yref, rtol=1e-4, atol=1e-5)
    g = net.backward(Xd, td).cpu().numpy()
    loss_ref, gref = oracle.mlp_loss_grad(P64, X.astype(np.float64), t.astype(np.float64))
    assert abs(net.loss.item() - loss_ref) <= 1e-4 * max(1.0, loss_ref)
    gflat = np.concatenate([a.reshape(-1) for a in gref])
    for name, a, b in zip(["W1", "b1", "W2", "b2", "W3", "b3"], C.split_params(g), gref):
        a = np.asarray(a, dtype=np.float64).reshape(-1)
        b = b.reshape(-1)
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-12)
        assert rel <= 1e-3, (name, rel)
    assert np.linalg.norm(g - gflat) / np.linalg.norm(gflat) <= 1e-3


def test_adam_matches_oracle(C):
    import torch
    X, t = _data(64, 1)
    p = C.init_params(2)
    net = C.DeviceMLP(p, X.shape[0])
    Xd, td = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    P = [a.astype(np.float64) for a in C.split_params(p)]
    m = [np.zeros_like(a) for a in P]
    v = [np.zeros_like(a) for a in P]
    for step in range(1, 4):
        net.forward(Xd)
        g = net.backward(Xd, td).cpu().numpy().astype(np.float64)
        net.adam(lr=1e-2)
        G = [np.asarray(a) for a in C.split_params(g)]
        P, m, v = oracle.adam_step(P, G, m, v, t=step, lr=1e-2)
        got = [np.asarray(a, dtype=np.float64) for a in C.split_params(net.params())]
        for a, b in zip(got, P):
            np.testing.assert_allclose(a, b, rtol=1e-4, atol=1e-6)


def test_training_reduces_loss(C):
    X, t = _data(512, 3)
    params, hist = C.train(X, t, steps=600, lr=3e-3, log_every=100)
    print("loss", hist, flush=True)
    assert hist[-1][1] < 0.1 * hist[0][1]


def test_learned_plan_parity(C):
    import paper_2608_16940_amd as P
    params = C.load()[0] if os.path.exists(C.WEIGHTS) else C.init_params(0)
    n = 18
    gates = W.headline(n, 6, 1)
    plan = P.Plan.learned(n, gates, params)
    sv = P.StateVector(n)
    plan.run(sv)
    got = oracle.decode(sv.physical_state(), sv.layout())
    m = oracle.metrics(oracle.run(n, gates), got)
    assert m["infidelity"] <= 1e-5 and m["max_abs"] <= 1e-5 and m["rel_l2"] <= 1e-5, m


def test_learned_plan_not_slower_than_greedy(C):
    """The learned planner (reorder, DP on predicted times, cap search) against greedy k<=5 in circuit
    order: execute time at N=27.  Most of this gain comes from wider blocks and the reorder; the
    network's own share is measured against the analytic score below."""
    import torch

    import paper_2608_16940_amd as P
    if not os.path.exists(C.WEIGHTS):
        pytest.skip("no trained cost model committed")
    params = C.load()[0]
    n = 27
    gates = W.brickwork(n, 12, 0)
    plans = {"greedy": P.Plan.greedy(n, gates, 5), "learned": P.Plan.learned(n, gates, params)}
    sv = P.StateVector(n)
    res = {}
    for name, plan in plans.items():
        plan.run(sv)
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            sv.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.run(sv)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        res[name] = (min(ts), len(plan))
    print("greedy %.4f s (%d blocks), learned %.4f s (%d blocks), gain %.1f%%"
          % (res["greedy"][0], res["greedy"][1], res["learned"][0], res["learned"][1],
             100 * (1 - res["learned"][0] / res["greedy"][0])), flush=True)
    assert res["learned"][0] < res["greedy"][0]


def test_layout_swap_from_the_model_runs_and_pays(C):
    """N=30, dense 4-qubit gates alternating between qubits 20..23 and 0..3: the swap pass moves
    20..23 down once; the run keeps the logical state (echo with the inverse plan back to |0...0>)
    and takes less time than the plan without the swap.  Binding a plan with swaps is refused."""
    import torch
    import paper_2608_16940_amd as P
    import paper_2608_16940_amd._native as N
    params, _ = C.load()
    n = 30
    rng = np.random.default_rng(0)
    gates = []
    for _ in range(20):
        gates.append(W.random_dense(n, 4, rng, (20, 21, 22, 23)))
        gates.append(W.random_dense(n, 4, rng, (0, 1, 2, 3)))
    base = P.Plan.greedy(n, gates, 4)
    swp = P.Plan.greedy(n, gates, 4)
    assert swp.add_swaps(params) == 1
    sv = P.StateVector(n)

    def timed(plan):
        sv.reset()
        plan.run(sv)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2):
            sv.reset()
            plan.run(sv)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / 2
    t_base, t_swap = timed(base), timed(swp)
    print("alternating case: %.1f ms without swap, %.1f ms with the model's swap" % (t_base * 1e3, t_swap * 1e3),
          flush=True)
    assert t_swap < t_base
    st = sv.stats()
    assert st["permute_sweeps"] == 1
    assert not np.array_equal(sv.layout(), np.arange(n))  # 20..23 now sit on the chosen window
    inv = P.Plan.greedy(n, W.inverse(gates), 4)
    inv.run(sv)
    sv.sync()
    f0 = abs(sv.amps[0].item()) ** 2 / sv.norm()
    assert f0 >= 1 - 1e-5
    with pytest.raises(P.SvError) as e:
        swp.bind(sv)
    assert e.value.code == N.SV_ERR_UNSUPPORTED
    sv.close()


def test_network_vs_analytic_score_same_pipeline(C):
    """Ablation of the cost model: the same reorder, windowed DP, cross-window merge, cap search and
    four rounds with Gamma = the MLP's predicted sweep time or Gamma = the analytic roofline time
    (SV_SCORE_ROOFLINE).  At N=28 (brickwork depth 16, seed 0) both plans are checked against the
    oracle amplitudes and timed.  The measured margin is reported; the test requires both to beat
    greedy k<=5 by 2x and to lie within 10% of each other (at N=30 and N=34 the analytic score's
    plans were 0.8% and 2.0% faster, so the trained network shows no gain over it here)."""
    import torch

    import paper_2608_16940_amd as P
    n = 28
    params, _ = C.load()
    gates = W.brickwork(n, 16, 0)
    golden = os.path.join(os.path.dirname(__file__), "golden", "brickwork_n28_amplitudes.txt")
    idx, ref = [], []
    with open(golden) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            i, re, im = ln.split()
            idx.append(int(i))
            ref.append(complex(float(re), float(im)))
    idx, ref = np.array(idx, dtype=np.int64), np.array(ref)
    plans = {"greedy": P.Plan.greedy(n, gates, 5), "network": P.Plan.learned(n, gates, params, swaps=False),
             "analytic": P.Plan.roofline(n, gates)}
    sv = P.StateVector(n)
    t = {}
    for name, plan in plans.items():
        ts = []
        for _ in range(3):
            sv.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.run(sv)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        t[name] = sorted(ts)[1]
        lay = sv.layout()
        y = np.zeros_like(idx)
        for q, pos in enumerate(lay):
            y |= ((idx >> q) & 1) << int(pos)
        got = sv.amps[torch.from_numpy(y).to(sv.amps.device)].cpu().numpy().astype(np.complex128)
        d = np.abs(got - ref)
        rel = float(np.sqrt(np.sum(d ** 2) / np.sum(np.abs(ref) ** 2)))
        print("N=28 %s: %d blocks, %.1f ms, rel_l2(sample) %.2e" % (name, len(plan), t[name] * 1e3, rel), flush=True)
        assert d.max() <= 1e-5 and rel <= 1e-5
    margin = 1 - t["network"] / t["analytic"]
    print("network margin over the analytic score: %+.1f%%" % (100 * margin), flush=True)
    assert t["network"] < 0.5 * t["greedy"] and t["analytic"] < 0.5 * t["greedy"]
    assert abs(margin) <= 0.10
    sv.close()
