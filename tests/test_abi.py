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
