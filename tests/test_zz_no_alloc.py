"""The allocation-free sampler (sv_sample_probs_noalloc) against the sampler with a
caller workspace (sv_sample_probs), through the C ABI: outcomes must be
bit-identical (integer work), on consecutive calls that shrink the input, at
the maximum size, across the shot-chunk boundary, and with the same errors."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2608_16940_amd as P
    from paper_2608_16940_amd import _native as N
    P.lib()
    return torch, P, N


def _probs(torch, n, seed, zero_frac=0.25):
    rng = np.random.default_rng(seed)
    p = rng.random(1 << n)
    p[rng.random(1 << n) < zero_frac] = 0.0
    p /= p.sum()
    return torch.from_numpy(p).to("cuda:0")


def _call_noalloc(torch, P, N, probs_dev, n, seed, shots):
    out = np.empty(int(shots), dtype=np.uint64)
    rc = P.lib().sv_sample_probs_noalloc(ctypes.c_void_p(probs_dev.data_ptr()), n, ctypes.c_uint64(seed), int(shots),
                                         out.ctypes.data_as(N._u64p),
                                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, out


def _call_ws(torch, P, N, probs_dev, n, seed, shots):
    ws = torch.empty(P.workspace_bytes(n), dtype=torch.uint8, device="cuda:0")
    out = np.empty(int(shots), dtype=np.uint64)
    rc = P.lib().sv_sample_probs(ctypes.c_void_p(probs_dev.data_ptr()), n, ctypes.c_uint64(seed), int(shots),
                                 out.ctypes.data_as(N._u64p), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, out


@pytest.mark.parametrize("sizes", [(20, 13), (26, 3), (11, 10)])
def test_noalloc_matches_workspace_sampler_on_consecutive_calls(env, sizes):
    torch, P, N = env
    for i, n in enumerate(sizes):
        probs = _probs(torch, n, 100 * n + i)
        shots = 150_000 if i == 0 else 5_000  # the first call crosses the 65536-shot chunk
        seed = 0x5EED + i
        rc_a, a = _call_noalloc(torch, P, N, probs, n, seed, shots)
        rc_b, b = _call_ws(torch, P, N, probs, n, seed, shots)
        assert rc_a == N.SV_OK and rc_b == N.SV_OK, (n, P.lib().sv_last_error())
        np.testing.assert_array_equal(a, b)
        # every outcome is a valid index with nonzero probability
        pc = probs.cpu().numpy()
        assert int(a.max()) < (1 << n) and np.all(pc[a.astype(np.int64)] > 0)


def test_noalloc_rejects_what_the_workspace_sampler_rejects(env):
    torch, P, N = env
    n = 12
    base = _probs(torch, n, 7).cpu().numpy()
    bad = []
    neg = base.copy()
    neg[5] = -1e-3
    bad.append(neg)
    nan = base.copy()
    nan[9] = np.nan
    bad.append(nan)
    big = base * 5.0  # sums to 5: the fixed-point total would wrap
    bad.append(big)
    inf = base.copy()
    inf[0] = np.inf
    bad.append(inf)
    for arr in bad:
        d = torch.from_numpy(arr).to("cuda:0")
        assert _call_noalloc(torch, P, N, d, n, 1, 10)[0] == N.SV_ERR_ARG
        assert _call_ws(torch, P, N, d, n, 1, 10)[0] == N.SV_ERR_ARG
    zero = torch.zeros(1 << n, dtype=torch.float64, device="cuda:0")
    assert _call_noalloc(torch, P, N, zero, n, 1, 10)[0] == N.SV_ERR_STATE
    # beyond the scratch array's capacity
    d = torch.zeros(1 << (N.NOALLOC_MAX_QUBITS + 1), dtype=torch.float64, device="cuda:0")
    d[0] = 1.0
    rc, _ = _call_noalloc(torch, P, N, d, N.NOALLOC_MAX_QUBITS + 1, 1, 10)
    assert rc == N.SV_ERR_ARG and b"NOALLOC" in P.lib().sv_last_error()
    # a valid call after the rejected ones still matches
    good = torch.from_numpy(base).to("cuda:0")
    np.testing.assert_array_equal(_call_noalloc(torch, P, N, good, n, 3, 2000)[1],
                                  _call_ws(torch, P, N, good, n, 3, 2000)[1])
