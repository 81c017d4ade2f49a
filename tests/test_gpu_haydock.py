"""GPU parity of Haydock's method (section 3.2.2) through the C ABI against
the CPU oracle (``oracle.haydock_dos``, dense complex solves from the
definition), on the same seeded probes and the same (lb, ub).

Tolerances: the device evaluates the continued fraction of eq. (cfHaydock)
in FP64, the oracle solves (z - T) w = e_1 by LU: both are backward stable
with eta > 0, so the densities agree to ~1e-13 relative on the oracle's own
coefficients (bar 1e-11 of the maximum).  End to end, the GPU's Lanczos
coefficients differ from the oracle's by < 1e-11 (the Lanczos parity bar),
so the densities are compared at 1e-9 of their maximum with eta no smaller
than a tenth of the spectral half-width's 1 %.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import paper_1308_5467_amd as kpm
import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = kpm.Context(0)
    yield c
    c.close()


def dev(A, dtype):
    vals = A.val if dtype == "f64" else A.val.astype(np.float32)
    return kpm.DeviceCSR.from_host(A.n, A.row_ptr, A.col_idx, vals, dtype)


@pytest.mark.parametrize("M,npts,eta", [(1, 7, 0.5), (40, 150, 0.05), (530, 33, 0.02), (513, 9, 0.3)])
def test_kernel_on_oracle_coefficients(ctx, M, npts, eta):
    """Several point tiles with a ragged last one; M > 512 crosses the
    kernel's LDS chunks."""
    _say(f"haydock kernel M={M} npts={npts} eta={eta}")
    A = synth.random_sparse_symmetric(3001, 4.5, 17)
    b = oracle.lanczos_bounds(A, 20, 4)
    c, d = oracle.rescale(b["lb"], b["ub"])
    al, be = oracle.lanczos_tridiag(A, c, d, M, 5, 9)
    m = oracle.lanczos_steps_used(al, be)
    x = np.linspace(b["lb"] - 0.5, b["ub"] + 0.5, npts)
    ref = oracle.haydock_dos(al, be, m, x, eta, c, d)
    phi = kpm.kpm_haydock_dos(ctx, al, be, m, b["lb"], b["ub"], eta, x)
    assert np.max(np.abs(phi - ref)) < 1e-11 * np.max(ref)
    assert np.all(phi > 0.0)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_end_to_end_anderson3d(ctx, dtype):
    _say(f"haydock end to end anderson3d {dtype}")
    A = synth.add_diagonal_disorder(synth.laplacian3d_periodic(13), 16.0, 83)
    Ao = A if dtype == "f64" else A.rounded_f32()
    b = oracle.lanczos_bounds(Ao, 20, 3)
    c, d = oracle.rescale(b["lb"], b["ub"])
    M, nvec, seed = 60, 10, 123
    _, _, used, al, be = kpm.kpm_slq(ctx, dev(A, dtype), b["lb"], b["ub"], M, nvec, seed, coefficients=True)
    used2, al2, be2 = kpm.kpm_slq(ctx, dev(A, dtype), b["lb"], b["ub"], M, nvec, seed, coefficients=True,
                                  nodes=False)  # coefficients only: the same bits
    assert np.array_equal(used, used2) and np.array_equal(al, al2) and np.array_equal(be, be2)
    ra, rb = oracle.lanczos_tridiag(Ao, c, d, M, nvec, seed)
    rm = oracle.lanczos_steps_used(ra, rb)
    assert np.array_equal(used, rm)
    x = np.linspace(b["lb"], b["ub"], 200)
    eta = 0.01 * d
    phi = kpm.kpm_haydock_dos(ctx, al, be, used, b["lb"], b["ub"], eta, x)
    ref = oracle.haydock_dos(ra, rb, rm, x, eta, c, d)
    assert np.max(np.abs(phi - ref)) < 1e-9 * np.max(ref)


def test_breakdown_exact_density(ctx):
    vals = np.array([-0.5] * 50 + [0.1] * 30 + [0.7] * 40)
    A = synth.diagonal_matrix(np.random.default_rng(2).permutation(vals))
    _, _, used, al, be = kpm.kpm_slq(ctx, dev(A, "f64"), -1.0, 1.0, 8, 3, 4, coefficients=True)
    assert np.all(used == 3)
    x = np.linspace(-1.0, 1.0, 101)
    eta = 0.02
    ref = (50 * oracle.lorentz(x + 0.5, eta) + 30 * oracle.lorentz(x - 0.1, eta)
           + 40 * oracle.lorentz(x - 0.7, eta)) / 120.0
    phi = kpm.kpm_haydock_dos(ctx, al, be, used, -1.0, 1.0, eta, x)
    assert np.max(np.abs(phi - ref)) < 1e-12 * np.max(ref)


def test_unit_mass_and_errors(ctx):
    A = synth.add_diagonal_disorder(synth.laplacian2d_dirichlet(20), 4.0, 8)
    lb, ub = -2.5, 10.5
    _, _, used, al, be = kpm.kpm_slq(ctx, dev(A, "f64"), lb, ub, 30, 4, 8, coefficients=True)
    c, d = 0.5 * (lb + ub), 0.5 * (ub - lb)
    eta, R = 0.1, 40.0
    x = np.arange(c - R, c + R + 1e-9, eta / 10.0)
    phi = kpm.kpm_haydock_dos(ctx, al, be, used, lb, ub, eta, x)
    assert np.all(phi > 0.0)
    mass = np.trapezoid(phi, x)
    assert 1.0 - 2.0 / math.pi * eta / (R - d) - 1e-5 < mass < 1.0 - 2.0 / math.pi * eta / (R + d) + 1e-5
    assert kpm.kpm_haydock_dos(ctx, al, be, used, lb, ub, eta, np.zeros(0)).size == 0
    bad = used.copy()
    bad[1] = 0
    for args in ((al, be, used, lb, ub, 0.0), (al, be, used, ub, lb, 0.1), (al, be, bad, lb, ub, 0.1)):
        with pytest.raises(kpm.KpmError) as e:
            kpm.kpm_haydock_dos(ctx, *args, x[:5])
        assert e.value.status == -1
    nan = al.copy()
    nan[2, 3] = np.nan
    with pytest.raises(kpm.KpmError):
        kpm.kpm_haydock_dos(ctx, nan, be, used, lb, ub, 0.1, x[:5])


def test_c2_full_size_sampled(ctx):
    """64^3 Anderson (n = 262,144), 100 steps, 64 probes, FP32 values; the
    oracle runs probes 0, 31 and 63 and their densities are compared one by
    one."""
    _say("haydock c2 full size")
    A = synth.config_matrix("c2")
    D = dev(A, "f32")
    lb, ub = kpm.kpm_bounds(ctx, D, 20, 3002, 0.01)
    c, d = oracle.rescale(lb, ub)
    _, _, used, al, be = kpm.kpm_slq(ctx, D, lb, ub, 100, 64, 2002, coefficients=True)
    x = np.linspace(lb, ub, 200)
    eta = 0.02 * d
    full = kpm.kpm_haydock_dos(ctx, al, be, used, lb, ub, eta, x)
    assert np.all(full > 0.0)
    Ao = A.rounded_f32()
    for l in (0, 31, 63):
        ra, rb = oracle.lanczos_tridiag(Ao, c, d, 100, 1, 2002, vec0=l)
        rm = oracle.lanczos_steps_used(ra, rb)
        ref = oracle.haydock_dos(ra, rb, rm, x, eta, c, d)
        phi = kpm.kpm_haydock_dos(ctx, al[l:l + 1], be[l:l + 1], used[l:l + 1], lb, ub, eta, x)
        assert np.max(np.abs(phi - ref)) < 1e-9 * np.max(ref), l
