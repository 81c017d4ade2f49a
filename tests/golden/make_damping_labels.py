"""Writes damping_labels.npz: exact blurred densities of a labelled subset of
the damping network's training family, for the learned-damping tests.

Matrices (generators in synth/, no method arithmetic):
  family 0: synth.damping_training_matrix(i), i < 8,192 -- random sparse
            symmetric, n = 2,048; training i = 0..1,791, held out
            i = 8,000..8,191;
  family 1: synth.damping_training_matrix(8,192 + j) -- 2D Anderson 32 x 64;
            training j = 0..255, held out j = 992..1,023;
  family 2: synth.anderson3d_family_matrix(j) -- 3D Anderson 12^3;
            training j = 0..255, held out j = 256..287;
  family 3: synth.lattice_family_matrix(j) -- nearly clean 3D periodic and
            2D Dirichlet Laplacians (W < 2, spectra of a few high peaks);
            training j = 0..255, held out j = 256..287.
Values are rounded to FP32, as the FP32 path reads them.

Per matrix (oracle only): eigenvalues by dense eigh; bounds lb, ub with
c = (lambda_min + lambda_max)/2 and d = (lambda_max - lambda_min)/(2 * 0.98)
(the spectrum maps into [-0.98, 0.98]); label = the Gaussian-blurred exact
density phi_sigma(t) = (1/n) sum_j g_sigma(t - s_j) of eq. (blurphi) (with
the 1/n) at the 200 midpoints of [-1, 1], sigma = 0.02, s_j = (lambda_j - c)/d.

    python tests/golden/make_damping_labels.py      (a few minutes on 8 cores)
"""
import os
import sys

os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import multiprocessing as mp  # noqa: E402

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "damping_labels.npz")
SIGMA = 0.02
SPLITS = [  # (family, indices, split: 0 = training, 1 = held out)
    (0, range(0, 1792), 0), (0, range(8000, 8192), 1),
    (1, range(0, 256), 0), (1, range(992, 1024), 1),
    (2, range(0, 256), 0), (2, range(256, 288), 1),
    (3, range(0, 256), 0), (3, range(256, 288), 1),
]


def matrix(family: int, i: int):
    if family == 0:
        return synth.damping_training_matrix(i)
    if family == 1:
        return synth.damping_training_matrix(synth.DAMPING_N_RANDOM + i)
    if family == 2:
        return synth.anderson3d_family_matrix(i)
    return synth.lattice_family_matrix(i)


def label(job):
    family, i = job
    A = matrix(family, i).rounded_f32()
    lam = np.linalg.eigvalsh(A.dense())
    c, d = 0.5 * (lam[0] + lam[-1]), 0.5 * (lam[-1] - lam[0]) / 0.98
    phi = oracle.blurred_exact((lam - c) / d, oracle.midpoints(200), SIGMA)
    return c - d, c + d, phi


def main():
    jobs, fam, idx, split = [], [], [], []
    for f, rng, s in SPLITS:
        for i in rng:
            jobs.append((f, i))
            fam.append(f)
            idx.append(i)
            split.append(s)
    with mp.Pool(min(8, os.cpu_count() or 1)) as pool:
        res = pool.map(label, jobs, chunksize=8)
    np.savez_compressed(OUT, family=np.array(fam, dtype=np.int8), index=np.array(idx, dtype=np.int32),
                        split=np.array(split, dtype=np.int8), lb=np.array([r[0] for r in res]),
                        ub=np.array([r[1] for r in res]),
                        label=np.array([r[2] for r in res], dtype=np.float32), sigma=np.float64(SIGMA))
    print(f"wrote {OUT}: {len(jobs)} matrices")


if __name__ == "__main__":
    main()
