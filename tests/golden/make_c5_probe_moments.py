"""Writes c5_probe_moments.txt: the oracle's per-probe Chebyshev moments of
the large workload at its full degree, for the FP32 path's parity test.

Workload: 3D Anderson model on a 128^3 periodic grid (uniform[-8, 8]
diagonal, seed 1005) plus 2 random N(0, 0.1^2) long-range pairs per row
(seed 1105), values rounded to FP32 as the FP32 path reads them.  Bounds:
the oracle's 20-step Lanczos bounds (section 3.1.1) from start-vector seed
3005 with a 1 % margin.  Moments: probes 254 and 255 of seed 2005 (the last
probe block of the 256), degree 1000, plain three-term recurrence of
section 3.1.1 in FP64 (no doubling), normalised by n.  Calls only the
oracle and the input generators; takes a few minutes on two cores.

    python tests/golden/make_c5_probe_moments.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "c5_probe_moments.txt")
M, PROBES, SEED, LZ_SEED = 1000, (254, 255), 2005, 3005


def main():
    A = synth.config_matrix("c5").rounded_f32()
    b = oracle.lanczos_bounds(A, 20, LZ_SEED, 0.01)
    lb, ub = float(b["lb"]), float(b["ub"])
    c, d = oracle.rescale(lb, ub)
    z = oracle.moments_per_vector(A, c, d, M, len(PROBES), SEED, vec0=PROBES[0], nthreads=len(PROBES)) / A.n
    with open(OUT, "w") as f:
        f.write("# Oracle per-probe moments of the 128^3 + long-range workload; written by\n")
        f.write("# make_c5_probe_moments.py (see its docstring for the recipe).\n")
        f.write(f"# n {A.n} nnz {A.nnz} M {M} seed {SEED} probes {PROBES[0]} {PROBES[1]}\n")
        f.write(f"lb {lb!r}\nub {ub!r}\n")
        for k in range(M + 1):
            f.write(f"{k} {float(z[0, k])!r} {float(z[1, k])!r}\n")
    print(f"wrote {OUT}: lb {lb} ub {ub}")


if __name__ == "__main__":
    main()
