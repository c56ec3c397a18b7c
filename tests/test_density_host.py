"""Host side of the density-matrix wrapper (no GPU).

* sv_dm_superop builds sum_i conj(E_i) (x) E_i with E_i on the low (row) bits,
  as the vectorised form of Section IV-B fixes; compared with numpy's
  Kronecker product and, through the oracle, with sum E rho E^dagger;
* size queries and argument errors;
* superop_gates: targets (V, V + N) and the diagonal marker.
"""
import ctypes

import numpy as np
import pytest

import oracle
from oracle import density as D
from workloads import noise as Nz


@pytest.fixture(scope="module")
def P():
    import paper_2608_16940_amd as P
    P.lib()
    return P


@pytest.mark.parametrize("k,r", [(1, 1), (1, 4), (2, 3), (3, 2), (4, 2)])
def test_superop_is_conj_kron(P, k, r):
    rng = np.random.default_rng(10 * k + r)
    ch = Nz.random_channel(tuple(range(k)), r, rng)
    S = P.superop(ch.kraus)
    np.testing.assert_allclose(S, sum(np.kron(e.conj(), e) for e in ch.kraus), atol=1e-15)


def test_superop_acts_as_the_channel_on_vec(P):
    rng = np.random.default_rng(2)
    n = 3
    rho = D.run(n, [Nz.random_channel((0, 1, 2), 3, rng)])
    ch = Nz.random_channel((2, 0), 2, rng)
    v = D.vec(rho).copy()
    oracle.apply_gate(v, P.superop(ch.kraus), [2, 0, 2 + n, 0 + n])
    np.testing.assert_allclose(v, D.vec(D.apply_channel(rho, ch.kraus, (2, 0))), atol=1e-13)


def test_sizes_and_errors(P):
    import paper_2608_16940_amd._native as N
    lib = P.lib()
    assert lib.sv_dm_state_bytes(2) == 8 * 16 and lib.sv_dm_state_bytes(17) == 8 << 34
    assert lib.sv_dm_state_bytes(1) == 0 and lib.sv_dm_state_bytes(18) == 0
    assert lib.sv_dm_workspace_bytes(10) == lib.sv_workspace_bytes(20)
    out = np.zeros(2 * 16, dtype=np.float64)
    e = np.eye(2, dtype=np.complex128)
    dp = ctypes.POINTER(ctypes.c_double)
    for nk, k in [(0, 1), (1, 0), (1, 5)]:
        assert lib.sv_dm_superop(e.view(np.float64).ctypes.data_as(dp), nk, k, out.ctypes.data_as(dp)) == N.SV_ERR_ARG
    assert lib.sv_dm_qubits(None) == N.SV_ERR_ARG
    with pytest.raises(ValueError):
        P.superop([np.ones((2, 3))])


def test_superop_gates_targets_and_diag(P):
    n = 4
    chans = [Nz.dephasing(3, 0.2), Nz.depolarizing((1, 2), 0.1), Nz.amplitude_damping(0, 0.3)]
    g = P.superop_gates(n, chans)
    assert [x.targets for x in g] == [(3, 7), (1, 2, 5, 6), (0, 4)]
    assert [x.diag for x in g] == [True, False, False]
    assert all(np.count_nonzero(x.matrix - np.diag(np.diag(x.matrix))) == 0 for x in g if x.diag)
