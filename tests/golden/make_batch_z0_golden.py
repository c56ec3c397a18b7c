"""Write the oracle's <Z_0> for every circuit of the 4096-circuit batch family (seed 0).

Each circuit of batch_family(4096, seed=0) is applied gate by gate by the
complex128 CPU oracle; <Z_0> = sum_x |psi_x|^2 (1 - 2 x_0) in FP64.  The
full-batch GPU test compares the batched kernel's <Z_0> for all 4096
circuits against this file.  Calls only oracle/ and workloads/.

usage: python tests/golden/make_batch_z0_golden.py
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch4096_seed0_z0.txt")


def main():
    circs = W.batch_family(4096, seed=0)
    with open(OUT, "w") as f:
        f.write("# batch_family(4096, seed=0): complex128 oracle, gate by gate\n")
        f.write("# <index> <n_qubits> <gates> <Z0>\n")
        for i, (n, gates) in enumerate(circs):
            psi = oracle.run(n, gates)
            f.write("%d %d %d %.17g\n" % (i, n, len(gates), oracle.expect_z(psi, 0)))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
