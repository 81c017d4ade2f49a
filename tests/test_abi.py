"""The C-ABI library loads and exports every symbol include/kpm.h declares.

No compute calls: these run without a GPU.
"""
import ctypes
import os
import re

import pytest

import paper_1308_5467_amd as kpm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "kpm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kpm_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    assert _declared() == sorted(kpm.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = kpm.load_library()
    for name in _declared():
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_mlp_param_count():
    assert kpm.kpm_mlp_param_count() == 128 * 256 + 256 + 256 * 256 + 256 + 256 * 128 + 128


def test_status_codes_match_header():
    src = open(os.path.join(ROOT, "include", "kpm.h")).read()
    for name, val in re.findall(r"(KPM_(?:OK|ERR_[A-Z]+))\s*=\s*(-?\d+)", src):
        assert kpm.STATUS[int(val)] == name


def test_null_context_is_rejected_without_gpu():
    lib = kpm.load_library()
    assert lib.kpm_destroy(None) == -1
    assert lib.kpm_last_error(None) == b"context is NULL"
    assert lib.kpm_profile_enable(None, 1) == -1


def test_functional_nodes_are_gauss_chebyshev():
    """kpm_functional_nodes is host-only.  Mapped back to t = (x - c)/d, its
    Q nodes integrate T_k exactly against the Chebyshev weight: the mean of
    T_k(t_q) is 1 for k = 0 and 0 for 0 < k < 2Q (Gauss-Chebyshev rule), and
    the nodes are distinct, decreasing and inside (lb, ub)."""
    import numpy as np
    lb, ub, Q = -3.5, 9.25, 37
    x = kpm.kpm_functional_nodes(Q, lb, ub)
    c, d = 0.5 * (lb + ub), 0.5 * (ub - lb)
    t = (x - c) / d
    assert np.all(np.diff(x) < 0) and lb < x.min() and x.max() < ub
    for k in range(0, 2 * Q):
        mean = np.mean(np.polynomial.chebyshev.chebval(t, [0] * k + [1]))
        assert abs(mean - (1.0 if k == 0 else 0.0)) < 1e-12, k
    assert abs(np.mean(np.polynomial.chebyshev.chebval(t, [0] * (2 * Q) + [1])) + 1.0) < 1e-12
    with pytest.raises(kpm.KpmError):
        kpm.kpm_functional_nodes(0, lb, ub)
    with pytest.raises(kpm.KpmError):
        kpm.kpm_functional_nodes(4, 1.0, 1.0)
