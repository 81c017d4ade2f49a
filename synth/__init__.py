"""Seeded synthetic sparse symmetric matrices shaped like the paper's workloads.

This module builds inputs only: CSR arrays of test matrices.  It holds no step
of the kernel polynomial method (no rescaling, no recurrence, no moments), so
both the CPU oracle and the GPU library may consume what it produces.

The paper's own test matrices (a modified 2D Laplacian, and the pe3k / shwater
matrices of the Florida sparse collection, section 4) are not available here;
the generators below stand in for them with matrices of the same families:
finite-difference Laplacians, Anderson-type random diagonal disorder, random
sparse symmetric matrices and random long-range hoppings.

Every generator returns a :class:`CSR` with int32 ``row_ptr``/``col_idx``
(columns sorted within each row, no duplicates) and float64 ``val``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp

__all__ = [
    "CSR",
    "laplacian2d_dirichlet",
    "laplacian3d_periodic",
    "laplacian2d_periodic",
    "add_diagonal_disorder",
    "random_sparse_symmetric",
    "add_long_range",
    "diagonal_matrix",
    "batched_uneven_set",
    "lattice_family_matrix",
    "damping_training_set",
    "config_matrix",
    "CONFIGS",
]


@dataclasses.dataclass
class CSR:
    """Compressed sparse row matrix (square, symmetric by construction)."""

    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col_idx: np.ndarray  # int32 [nnz]
    val: np.ndarray      # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.n, self.n))

    def dense(self) -> np.ndarray:
        return self.to_scipy().toarray()

    def rounded_f32(self) -> "CSR":
        """Same pattern with values rounded to float32 and held back in float64.

        The rounded values are exactly representable in both precisions, so an
        FP32 consumer and an FP64 consumer see the same matrix.
        """
        return CSR(self.n, self.row_ptr, self.col_idx,
                   self.val.astype(np.float32).astype(np.float64))


def _from_scipy(m: sp.spmatrix) -> CSR:
    m = sp.csr_matrix(m)
    m.sum_duplicates()
    m.sort_indices()
    m.eliminate_zeros()
    n = m.shape[0]
    return CSR(n, m.indptr.astype(np.int32), m.indices.astype(np.int32),
               m.data.astype(np.float64))


def _lap1d(N: int, periodic: bool) -> sp.csr_matrix:
    main = 2.0 * np.ones(N)
    off = -np.ones(N - 1)
    T = sp.diags([off, main, off], [-1, 0, 1], shape=(N, N), format="lil")
    if periodic and N > 2:
        T[0, N - 1] = -1.0
        T[N - 1, 0] = -1.0
    return sp.csr_matrix(T)


def laplacian2d_dirichlet(N: int) -> CSR:
    """5-point Laplacian on an N x N grid with zero Dirichlet boundary.

    Diagonal 4, nearest neighbours -1 (grid spacing 1), n = N^2.
    """
    T = _lap1d(N, False)
    I = sp.identity(N, format="csr")
    return _from_scipy(sp.kron(I, T) + sp.kron(T, I))


def laplacian2d_periodic(Lx: int, Ly: int) -> CSR:
    """5-point Laplacian on an Lx x Ly periodic grid (diagonal 4, off -1)."""
    Tx, Ty = _lap1d(Lx, True), _lap1d(Ly, True)
    return _from_scipy(sp.kron(sp.identity(Ly), Tx) + sp.kron(Ty, sp.identity(Lx)))


def laplacian3d_periodic(L: int) -> CSR:
    """7-point Laplacian on an L^3 periodic grid (diagonal 6, off -1), n = L^3."""
    T = _lap1d(L, True)
    I = sp.identity(L, format="csr")
    A = sp.kron(sp.kron(I, I), T) + sp.kron(sp.kron(I, T), I) + sp.kron(sp.kron(T, I), I)
    return _from_scipy(A)


def add_diagonal_disorder(A: CSR, W: float, seed: int) -> CSR:
    """Anderson-type disorder: add an independent uniform[-W/2, W/2] value to each diagonal entry."""
    rng = np.random.default_rng(seed)
    eps = rng.uniform(-W / 2.0, W / 2.0, size=A.n)
    return _from_scipy(A.to_scipy() + sp.diags(eps))


def diagonal_matrix(d: np.ndarray) -> CSR:
    """Diagonal matrix with the given entries (one stored entry per row, zeros kept)."""
    n = len(d)
    return CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
               np.asarray(d, dtype=np.float64).copy())


def random_sparse_symmetric(n: int, pairs_per_row: float, seed: int,
                            diag_range: tuple[float, float] = (-1.0, 1.0),
                            off_scale: float = 1.0) -> CSR:
    """Random sparse symmetric matrix.

    ``round(pairs_per_row * n)`` random off-diagonal positions (i < j) get
    N(0, off_scale^2) values mirrored to (j, i); the diagonal is uniform in
    ``diag_range``.  With pairs_per_row = 4.5 a row holds about 10 entries.
    """
    rng = np.random.default_rng(seed)
    m = int(round(pairs_per_row * n))
    i = rng.integers(0, n, size=m)
    j = rng.integers(0, n, size=m)
    keep = i != j
    i, j = i[keep], j[keep]
    lo, hi = np.minimum(i, j), np.maximum(i, j)
    v = rng.normal(0.0, off_scale, size=lo.size)
    U = sp.coo_matrix((v, (lo, hi)), shape=(n, n)).tocsr()
    U.sum_duplicates()
    D = sp.diags(rng.uniform(diag_range[0], diag_range[1], size=n))
    return _from_scipy(U + U.T + D)


def add_long_range(A: CSR, pairs_per_row: float, sigma: float, seed: int) -> CSR:
    """Add random long-range symmetric hoppings: about pairs_per_row * n random
    (i, j) pairs with N(0, sigma^2) values, mirrored."""
    rng = np.random.default_rng(seed)
    n = A.n
    m = int(round(pairs_per_row * n))
    i = rng.integers(0, n, size=m)
    j = rng.integers(0, n, size=m)
    keep = i != j
    i, j = i[keep], j[keep]
    v = rng.normal(0.0, sigma, size=i.size)
    U = sp.coo_matrix((v, (i, j)), shape=(n, n)).tocsr()
    return _from_scipy(A.to_scipy() + U + U.T)


def batched_uneven_set(count: int = 48, seed_base: int = 3000) -> list[CSR]:
    """The uneven batch: half 2D 5-point Dirichlet Laplacians (side 64..512),
    half 3D 7-point periodic Laplacians (side 16..64), each with uniform
    diagonal disorder of width W cycling through {2, 8, 16}."""
    half = count // 2
    mats = []
    widths = (2.0, 8.0, 16.0)
    for i in range(half):
        L = int(round(64 * 2 ** (3.0 * i / max(half - 1, 1))))
        W = widths[i % 3]
        mats.append(add_diagonal_disorder(laplacian2d_dirichlet(L), W, seed_base + i))
    for i in range(count - half):
        L = int(round(16 * 2 ** (2.0 * i / max(count - half - 1, 1))))
        W = widths[(half + i) % 3]
        mats.append(add_diagonal_disorder(laplacian3d_periodic(L), W, seed_base + half + i))
    return mats


GOLDEN_RATIO_FRAC = 0.6180339887498949
DAMPING_N_RANDOM, DAMPING_N_ANDERSON2D = 8192, 1024


def damping_training_matrix(i: int, seed_base: int = 4000) -> CSR:
    """Matrix i of the damping network's training family: i < 8,192 a random
    sparse symmetric matrix (n = 2,048, 4.5 n mirrored N(0, 1) pairs,
    uniform [-1, 1] diagonal, about 10 entries per row); 8,192 <= i < 9,216
    a 2D Anderson matrix (32 x 64 periodic lattice, diagonal disorder of
    width W = 1 + 15 frac(j * golden ratio), j = i - 8,192).  Seed seed_base + i."""
    if i < DAMPING_N_RANDOM:
        return random_sparse_symmetric(2048, 4.5, seed_base + i)
    j = i - DAMPING_N_RANDOM
    W = 1.0 + 15.0 * ((j * GOLDEN_RATIO_FRAC) % 1.0)
    return add_diagonal_disorder(laplacian2d_periodic(32, 64), W, seed_base + i)


def anderson3d_family_matrix(j: int, L: int = 12, seed_base: int = 14000) -> CSR:
    """Member j of a small 3D Anderson family (L^3 periodic 7-point
    Laplacian, diagonal disorder of width W = 1 + 15 frac(j * golden ratio)),
    the family of the 3D workloads at a size whose spectrum dense eigh
    resolves in well under a second.  Seed seed_base + j."""
    W = 1.0 + 15.0 * ((j * GOLDEN_RATIO_FRAC) % 1.0)
    return add_diagonal_disorder(laplacian3d_periodic(L), W, seed_base + j)


def lattice_family_matrix(j: int, seed_base: int = 15000) -> CSR:
    """Member j of a family of nearly clean lattice Laplacians, whose spectra
    are a few high peaks: even j a 3D periodic 7-point Laplacian of side
    12 + (j/2 mod 5), odd j a 2D Dirichlet 5-point Laplacian of side
    40 + (j/2 mod 25), both with uniform diagonal disorder of width
    W = 2 frac(j * golden ratio) in [0, 2).  Seed seed_base + j."""
    W = 2.0 * ((j * GOLDEN_RATIO_FRAC) % 1.0)
    if j % 2 == 0:
        return add_diagonal_disorder(laplacian3d_periodic(12 + (j // 2) % 5), W, seed_base + j)
    return add_diagonal_disorder(laplacian2d_dirichlet(40 + (j // 2) % 25), W, seed_base + j)


def damping_training_set(n_random: int = 8192, n_anderson: int = 1024, seed_base: int = 4000) -> list[CSR]:
    """The damping network's training family at full size: ``n_random``
    random sparse symmetric matrices followed by ``n_anderson`` 2D Anderson
    matrices, as damping_training_matrix describes (with the default counts
    matrix i of the list is damping_training_matrix(i))."""
    mats = [random_sparse_symmetric(2048, 4.5, seed_base + i) for i in range(n_random)]
    for i in range(n_anderson):
        W = 1.0 + 15.0 * ((i * GOLDEN_RATIO_FRAC) % 1.0)
        mats.append(add_diagonal_disorder(laplacian2d_periodic(32, 64), W, seed_base + n_random + i))
    return mats


# Workload registry.  Seeds: matrix 1000+cfg, probe vectors 2000+cfg, Lanczos 3000+cfg.
CONFIGS = {
    "c1": dict(name="lap2d_dirichlet_32x32", M=100, nvec=20, block=20, precision="f64",
               vec_seed=2001, lanczos_seed=3001),
    "c2": dict(name="anderson3d_64cubed_W16", M=256, nvec=64, block=64, precision="f32",
               vec_seed=2002, lanczos_seed=3002),
    "c3": dict(name="batched_uneven_48", M=200, nvec=32, block=32, precision="f32",
               vec_seed=2003, lanczos_seed=3003),
    "c4": dict(name="damping_training_set_8192_random_1024_anderson2d", M=127, nvec=256, block=64,
               precision="f32", vec_seed=2004, lanczos_seed=3004),
    "c5": dict(name="anderson3d_128cubed_longrange", M=1000, nvec=256, block=64,
               precision="f32", vec_seed=2005, lanczos_seed=3005),
}


def config_matrix(cfg: str, scale: int | None = None) -> CSR:
    """Matrix of a registered workload; ``scale`` overrides the grid side for
    reduced-size variants of the same family."""
    if cfg == "c1":
        return laplacian2d_dirichlet(scale or 32)
    if cfg == "c2":
        return add_diagonal_disorder(laplacian3d_periodic(scale or 64), 16.0, 1002)
    if cfg == "c5":
        base = add_diagonal_disorder(laplacian3d_periodic(scale or 128), 16.0, 1005)
        return add_long_range(base, 2.0, 0.1, 1105)
    raise KeyError(cfg)


def grid_side_for(n: int, dim: int) -> int:
    return int(round(n ** (1.0 / dim)))


if __name__ == "__main__":  # pragma: no cover
    A = config_matrix("c2")
    print(A.n, A.nnz, math.isclose(A.nnz / A.n, 7.0))
