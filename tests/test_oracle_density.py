"""Pins for the density-matrix oracle (no GPU).

The oracle applies rho -> sum_i E_i rho E_i^dagger with embedded operators.
It is checked against what does not come from that code:

* a unitary circuit on |0><0| gives |psi><psi| with psi from the pinned
  state-vector oracle (catches E rho E^T, conj(E) rho E^T and swapped factors);
* closed forms of textbook channels: one- and two-qubit depolarizing,
  amplitude damping on a state with a complex phase (target on a high qubit
  too), dephasing, and complete depolarization of every qubit;
* the vectorised form of Section IV-B: sum_i conj(E_i) kron E_i applied by
  the state-vector oracle to vec(rho) on the 2k targets (V, V + N) equals
  vec of the oracle's result (column-major vec, row copies first);
* trace, Hermiticity and positivity for random CPTP channels.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import density as D
import workloads as W
from workloads import noise as Nz


def random_mixed(n, rng, r=3):
    d = 1 << n
    rho = np.zeros((d, d), dtype=np.complex128)
    w = rng.random(r)
    w /= w.sum()
    for wi in w:
        v = rng.standard_normal(d) + 1j * rng.standard_normal(d)
        v /= np.linalg.norm(v)
        rho += wi * np.outer(v, v.conj())
    return rho


def test_unitary_circuit_is_outer_product_of_pure_state():
    n = 4
    gates = W.brickwork(n, 3, seed=5) + W.qft(n)
    psi = oracle.run(n, gates)
    rho = D.run(n, [Nz.unitary(g) for g in gates])
    np.testing.assert_allclose(rho, np.outer(psi, psi.conj()), atol=1e-12)


@pytest.mark.parametrize("p", [0.0, 0.3, 0.75])
def test_one_qubit_depolarizing_closed_form(p):
    # |0><0| on qubit 1 of two: populations 1 - 2p/3 and 2p/3 at indices 0 and 2
    rho = D.apply_channel(D.zero(2), Nz.depolarizing((1,), p).kraus, (1,))
    want = np.zeros((4, 4), dtype=np.complex128)
    want[0, 0] = 1 - 2 * p / 3
    want[2, 2] = 2 * p / 3
    np.testing.assert_allclose(rho, want, atol=1e-14)
    # |+><+|: the coherence shrinks by 1 - 4p/3
    plus = np.full((2, 2), 0.5, dtype=np.complex128)
    out = D.apply_channel(plus, Nz.depolarizing((0,), p).kraus, (0,))
    np.testing.assert_allclose(out, [[0.5, 0.5 * (1 - 4 * p / 3)], [0.5 * (1 - 4 * p / 3), 0.5]], atol=1e-14)


def test_two_qubit_depolarizing_closed_form():
    rng = np.random.default_rng(1)
    p = 0.2
    rho = random_mixed(2, rng)
    out = D.apply_channel(rho, Nz.depolarizing((1, 0), p).kraus, (1, 0))
    want = (1 - p - p / 15) * rho + (4 * p / 15) * np.eye(4)
    np.testing.assert_allclose(out, want, atol=1e-14)


@pytest.mark.parametrize("gamma,phi", [(0.3, 0.7), (1.0, 2.0)])
def test_amplitude_damping_closed_form(gamma, phi):
    e = complex(math.cos(phi), math.sin(phi))
    psi = np.array([1, e]) / math.sqrt(2)
    rho = np.outer(psi, psi.conj())
    out = D.apply_channel(rho, Nz.amplitude_damping(0, gamma).kraus, (0,))
    s = math.sqrt(1 - gamma)
    want = np.array([[1 - (1 - gamma) / 2, s * e.conjugate() / 2], [s * e / 2, (1 - gamma) / 2]])
    np.testing.assert_allclose(out, want, atol=1e-14)
    # the same one-qubit state as qubit 2 of three (others |0>): entries at bit 2
    big = np.zeros((8, 8), dtype=np.complex128)
    for a in range(2):
        for b in range(2):
            big[a << 2, b << 2] = rho[a, b]
    out3 = D.apply_channel(big, Nz.amplitude_damping(2, gamma).kraus, (2,))
    for a in range(2):
        for b in range(2):
            assert abs(out3[a << 2, b << 2] - want[a, b]) < 1e-14
    assert np.count_nonzero(np.abs(out3) > 1e-15) == np.count_nonzero(np.abs(want) > 1e-15)


def test_dephasing_and_complete_depolarization():
    rng = np.random.default_rng(2)
    n = 3
    rho = random_mixed(n, rng)
    out = D.apply_channel(rho, Nz.dephasing(1, 0.5).kraus, (1,))
    for r in range(8):
        for c in range(8):
            want = rho[r, c] if ((r >> 1) & 1) == ((c >> 1) & 1) else 0
            assert abs(out[r, c] - want) < 1e-14
    full = rho
    for q in range(n):
        full = D.apply_channel(full, Nz.depolarizing((q,), 0.75).kraus, (q,))
    np.testing.assert_allclose(full, np.eye(8) / 8, atol=1e-14)


@pytest.mark.parametrize("targets,r", [((2, 0), 3), ((0, 1), 2), ((1,), 4), ((2, 0, 1), 2)])
def test_vectorised_superoperator_form(targets, r):
    """Section IV-B: vec(sum E rho E^dag) = (sum conj(E) kron E) vec(rho) on targets (V, V + N)."""
    rng = np.random.default_rng(len(targets) * 10 + r)
    n = 3
    rho = random_mixed(n, rng)
    ch = Nz.random_channel(targets, r, rng)
    want = D.vec(D.apply_channel(rho, ch.kraus, targets))
    S = sum(np.kron(e.conj(), e) for e in ch.kraus)
    v = D.vec(rho).copy()
    oracle.apply_gate(v, S, list(targets) + [t + n for t in targets])
    np.testing.assert_allclose(v, want, atol=1e-13)
    # the column-major convention: vec index = row + 2^N column
    assert D.vec(rho)[3 + 8 * 5] == rho[3, 5]
    np.testing.assert_array_equal(D.unvec(D.vec(rho)), rho)


def test_random_channels_keep_a_density_matrix():
    rng = np.random.default_rng(3)
    n = 4
    rho = D.zero(n)
    for i in range(6):
        k = 1 + i % 2
        t = tuple(int(x) for x in rng.choice(n, k, replace=False))
        rho = D.apply_channel(rho, Nz.random_channel(t, 2 + i % 3, rng).kraus, t)
    assert abs(D.trace(rho) - 1) < 1e-13
    np.testing.assert_allclose(rho, rho.conj().T, atol=1e-14)
    assert np.linalg.eigvalsh(rho).min() > -1e-13
    assert D.purity(rho) <= 1 + 1e-13
    np.testing.assert_allclose(D.probs(rho).sum(), 1.0, atol=1e-13)


def test_kraus_sets_are_complete():
    rng = np.random.default_rng(4)
    for ch in [Nz.depolarizing((0, 1), 0.1), Nz.amplitude_damping(0, 0.4), Nz.dephasing(0, 0.2),
               Nz.random_channel((0, 1, 2), 3, rng)]:
        d = 1 << ch.k
        np.testing.assert_allclose(sum(e.conj().T @ e for e in ch.kraus), np.eye(d), atol=1e-13)


def test_purity_closed_forms():
    """purity = Tr(rho^2) = sum_ij |rho_ij|^2 on density matrices written out by hand: a pure state
    (1), the maximally mixed state on n qubits (2^-n), a dephased superposition with a complex
    coherence (1/2 + (1-2p)^2/2) and a diagonal mixture.  Tr(rho) (always 1), the diagonal alone,
    or Re(rho_ij)^2 all fail one of them."""
    rng = np.random.default_rng(11)
    v = rng.standard_normal(8) + 1j * rng.standard_normal(8)
    v /= np.linalg.norm(v)
    assert abs(D.purity(np.outer(v, v.conj())) - 1.0) < 1e-14
    for n in (1, 2, 4):
        assert abs(D.purity(np.eye(1 << n, dtype=np.complex128) / (1 << n)) - 2.0 ** -n) < 1e-15
    for p, phi in [(0.0, 0.7), (0.2, 1.3), (0.5, 2.0)]:
        c = 0.5 * (1 - 2 * p) * np.exp(-1j * phi)
        rho = np.array([[0.5, c], [np.conj(c), 0.5]], dtype=np.complex128)
        assert abs(D.purity(rho) - (0.5 + 0.5 * (1 - 2 * p) ** 2)) < 1e-15
    w = np.array([0.5, 0.25, 0.125, 0.125])
    assert abs(D.purity(np.diag(w).astype(np.complex128)) - float((w ** 2).sum())) < 1e-15


@pytest.mark.parametrize("p", [0.1, 0.4, 0.75])
def test_purity_after_depolarizing_closed_form(p):
    """One-qubit depolarizing of |0><0| through the oracle's channel application: populations
    1 - 2p/3 and 2p/3, so purity (1 + (1 - 4p/3)^2) / 2; on |+><+| the coherence shrinks by
    1 - 4p/3 and the purity is the same."""
    want = (1 + (1 - 4 * p / 3) ** 2) / 2
    rho = D.apply_channel(D.zero(1), Nz.depolarizing((0,), p).kraus, (0,))
    assert abs(D.purity(rho) - want) < 1e-14
    plus = np.full((2, 2), 0.5, dtype=np.complex128)
    rho = D.apply_channel(plus, Nz.depolarizing((0,), p).kraus, (0,))
    assert abs(D.purity(rho) - want) < 1e-14
    assert abs(D.trace(rho) - 1.0) < 1e-14
