"""Write oracle amplitudes of the N=30 headline circuit at seeded sample indices.

Circuit: random brickwork depth 24 (seed 0) followed by QFT30, the workload
bench.py times, applied gate by gate by the complex128 CPU oracle.  The file
stores the logical basis index and the amplitude (re, im) at 2048 indices
drawn with numpy's default generator seeded 20260, plus indices 0 and 2^30-1,
and the oracle's squared norm.  Calls only oracle/ and workloads/.

usage: python tests/golden/make_headline_n30_golden.py  (16 GiB of host memory, minutes on many cores)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "headline_n30_amplitudes.txt")


def main():
    n = 30
    gates = W.headline(n, 24, 0)
    t0 = time.time()
    psi = oracle.run(n, gates)
    el = time.time() - t0
    rng = np.random.default_rng(20260)
    idx = np.unique(np.concatenate([rng.integers(0, 1 << n, 2048), [0, (1 << n) - 1]]))
    norm = float(np.vdot(psi, psi).real)
    with open(OUT, "w") as f:
        f.write("# oracle amplitudes, N=30 brickwork depth 24 (seed 0) + QFT30, complex128 gate by gate\n")
        f.write("# written by tests/golden/make_headline_n30_golden.py (%d gates, %.0f s on %d threads)\n"
                % (len(gates), el, oracle.threads()))
        f.write("# norm %.17g\n" % norm)
        f.write("# index re im\n")
        for i in idx:
            a = psi[i]
            f.write("%d %.17g %.17g\n" % (int(i), a.real, a.imag))
    print("wrote", OUT, len(idx), "samples, norm", norm, "time", el)


if __name__ == "__main__":
    main()
