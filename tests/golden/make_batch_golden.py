"""Write oracle results for a sample of the 4096-circuit batch family (seed 0).

Circuits 0, 64, ..., 4032 of batch_family(4096, seed=0) are applied gate by
gate by the complex128 CPU oracle.  For each: <Z_0> and the amplitudes at
index 0 and 15 indices drawn with numpy's default generator seeded 20262 + i.
Used by the batch bench to report fidelity per result without running the
oracle at measurement time.  Calls only oracle/ and workloads/.

usage: python tests/golden/make_batch_golden.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch4096_seed0_sample.txt")


def main():
    circs = W.batch_family(4096, seed=0)
    with open(OUT, "w") as f:
        f.write("# batch_family(4096, seed=0): complex128 oracle, gate by gate\n")
        f.write("# circ <index> <n_qubits> <Z0>   then   amp <index> <basis index> <re> <im>\n")
        for i in range(0, 4096, 64):
            n, gates = circs[i]
            psi = oracle.run(n, gates)
            f.write("circ %d %d %.17g\n" % (i, n, oracle.expect_z(psi, 0)))
            rng = np.random.default_rng(20262 + i)
            idx = [0] + sorted(int(x) for x in rng.choice(1 << n, 15, replace=False))
            for x in idx:
                f.write("amp %d %d %.17g %.17g\n" % (i, x, psi[x].real, psi[x].imag))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
