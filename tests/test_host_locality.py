"""kpm_locality_order (host-only): the grid it finds behind a
lexicographically numbered matrix and the Morton row order it returns.

The order is checked against an independent Morton construction from the
grid coordinates; matrices without a grid (random sparse, diagonal, 1D
chain) keep the identity.  No GPU.
"""
import numpy as np
import pytest

import paper_1308_5467_amd as kpm
import synth


def morton_order(dims):
    """Rows of an nx x ny x nz grid (x fastest) sorted by interleaved bits."""
    nx, ny, nz = dims
    i = np.arange(nx * ny * nz, dtype=np.int64)
    x, y, z = i % nx, (i // nx) % ny, i // (nx * ny)
    key = np.zeros_like(i)
    for b in range(21):
        key |= ((x >> b) & 1) << (3 * b) | ((y >> b) & 1) << (3 * b + 1) | ((z >> b) & 1) << (3 * b + 2)
    return np.argsort(key, kind="stable")


@pytest.mark.parametrize("A,dims", [
    (synth.add_long_range(synth.add_diagonal_disorder(synth.laplacian3d_periodic(20), 16.0, 1), 2.0, 0.1, 2),
     (20, 20, 20)),
    (synth.laplacian2d_dirichlet(37), (37, 37, 1)),
    (synth.laplacian2d_periodic(24, 40), (24, 40, 1)),
])
def test_grid_found_and_morton_order(A, dims):
    perm, got = kpm.kpm_locality_order(A.row_ptr, A.col_idx)
    assert got == dims
    assert np.array_equal(perm, morton_order(dims))


def test_locality_of_the_order():
    """On a 32^3 stencil the renumbered neighbours are close: most entries
    within a few hundred rows of the diagonal instead of a plane (1,024 rows)."""
    A = synth.laplacian3d_periodic(32)
    perm, dims = kpm.kpm_locality_order(A.row_ptr, A.col_idx)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(A.n, dtype=np.int32)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    d_nat = np.abs(A.col_idx - rows)
    d_new = np.abs(inv[A.col_idx] - inv[rows])
    assert np.median(d_new[d_new > 0]) < 0.1 * np.median(d_nat[d_nat > 0]) + 8
    assert np.mean(d_new > 1024) < 0.5 * np.mean(d_nat >= 1024)


@pytest.mark.parametrize("A", [synth.random_sparse_symmetric(500, 4.5, 3), synth.diagonal_matrix(np.arange(7.0)),
                               synth.CSR(5, np.array([0, 2, 5, 8, 11, 13], np.int32),
                                         np.array([0, 1, 0, 1, 2, 1, 2, 3, 2, 3, 4, 3, 4], np.int32),
                                         np.ones(13))])
def test_no_grid_identity(A):
    perm, dims = kpm.kpm_locality_order(A.row_ptr, A.col_idx)
    assert dims == (0, 0, 0) and np.array_equal(perm, np.arange(A.n))


def test_bad_arguments():
    with pytest.raises(kpm.KpmError):
        kpm.kpm_locality_order(np.array([1, 2], np.int32), np.array([0], np.int32))  # row_ptr[0] != 0
    with pytest.raises(kpm.KpmError):
        kpm.kpm_locality_order(np.array([0, 3], np.int32), np.array([0], np.int32))  # row_ptr[n] != nnz
