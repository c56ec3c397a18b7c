"""The stored oracle values under tests/golden belong to the oracle and to the
circuit family they name (no GPU): a cheap subset of each file is recomputed
with the oracle and compared."""
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def batch_circuits():
    return W.batch_family(4096, seed=0)


def test_batch_z0_file_matches_the_oracle(batch_circuits):
    rows = {}
    with open(os.path.join(GOLDEN, "batch4096_seed0_z0.txt")) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            i, n, ng, z = ln.split()
            rows[int(i)] = (int(n), int(ng), float(z))
    assert sorted(rows) == list(range(4096))
    for i, (n, gates) in enumerate(batch_circuits):
        assert rows[i][:2] == (n, len(gates))
    # every circuit of up to 11 qubits among the first 512 (a few seconds of oracle work)
    small = [i for i in range(512) if batch_circuits[i][0] <= 11]
    assert len(small) >= 20
    for i in small:
        n, gates = batch_circuits[i]
        z = oracle.expect_z(oracle.run(n, gates), 0)
        assert abs(z - rows[i][2]) <= 1e-12, (i, z, rows[i][2])


def test_batch_sample_file_agrees_with_the_z0_file():
    z0 = {}
    with open(os.path.join(GOLDEN, "batch4096_seed0_z0.txt")) as f:
        for ln in f:
            if not ln.startswith("#") and ln.strip():
                i, _, _, z = ln.split()
                z0[int(i)] = float(z)
    seen = 0
    with open(os.path.join(GOLDEN, "batch4096_seed0_sample.txt")) as f:
        for ln in f:
            w = ln.split()
            if w and w[0] == "circ":
                assert abs(float(w[3]) - z0[int(w[1])]) <= 1e-12
                seen += 1
    assert seen == 64
