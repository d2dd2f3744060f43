"""Writes the exact fixed-dtau expectations used as pins by the GPU tests.

Calls only the oracle.  Each fixture is the exact Boltzmann average over all
2^L Hubbard-Stratonovich fields (enumeration, no Monte Carlo) for the
half-filled Bethe-lattice impurity at a fixed Trotter step, so a Monte Carlo
run at the same parameters must agree with it within its statistical error.

  python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import bath as B  # noqa: E402
from oracle import hfqmc as H  # noqa: E402

CASES = {
    # name: (beta, U, L, t, n_iw)
    "bethe_b10_u4_L12": (10.0, 4.0, 12, 1.0, 20000),
    "bethe_b10_u4_L20": (10.0, 4.0, 20, 1.0, 20000),
}


def main():
    for name, (beta, U, L, t, n_iw) in CASES.items():
        g_tau = B.bath_to_tau(B.semicircle_iw(beta, t, n_iw), t * t, beta, L)
        g, D, wmin = H.brute_force(g_tau, U, beta)
        path = os.path.join(HERE, name + ".txt")
        with open(path, "w") as f:
            f.write("# exact enumeration over 2^L HS fields, half-filled Bethe lattice (t=%g, W=4t)\n" % t)
            f.write("# semi-elliptic DOS as in the Benchmark results section; written by make_golden.py (oracle only)\n")
            f.write("# beta=%r U=%r L=%d n_iw=%d\n" % (beta, U, L, n_iw))
            f.write("# min relative weight %.3e\n" % wmin)
            f.write("D %.17g\n" % D)
            for k, v in enumerate(g):
                f.write("G %d %.17g\n" % (k, v))
        print("wrote", path)


if __name__ == "__main__":
    main()
