"""Write oracle amplitudes of brickwork(28, depth 16, seed 0) at seeded sample indices.

Used by the precision tests (k=6/7 fused sweeps in FP32 and BF16x3) and the
learned-planner parity test.  Applied gate by gate by the complex128 CPU
oracle; stores 2048 indices drawn with numpy's default generator seeded
20261 plus 0 and 2^28-1, and the oracle's squared norm.  Calls only oracle/
and workloads/.

usage: python tests/golden/make_brickwork_n28_golden.py   (4 GiB of host memory)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "brickwork_n28_amplitudes.txt")


def main():
    n = 28
    gates = W.brickwork(n, 16, 0)
    t0 = time.time()
    psi = oracle.run(n, gates)
    el = time.time() - t0
    rng = np.random.default_rng(20261)
    idx = np.unique(np.concatenate([rng.integers(0, 1 << n, 2048), [0, (1 << n) - 1]]))
    norm = float(np.vdot(psi, psi).real)
    with open(OUT, "w") as f:
        f.write("# oracle amplitudes, N=28 brickwork depth 16 (seed 0), complex128 gate by gate\n")
        f.write("# written by tests/golden/make_brickwork_n28_golden.py (%d gates, %.0f s on %d threads)\n"
                % (len(gates), el, oracle.threads()))
        f.write("# norm %.17g\n" % norm)
        f.write("# index re im\n")
        for i in idx:
            a = psi[i]
            f.write("%d %.17g %.17g\n" % (int(i), a.real, a.imag))
    print("wrote", OUT, len(idx), "samples, norm", norm, "time", el)


if __name__ == "__main__":
    main()
