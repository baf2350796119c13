"""C-ABI library: loads, exports every declared symbol, host-only defaults.
No device work is done here."""
import ctypes
import json
import os
import re

import pytest

from oracle import mfipm_ref as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mfipm.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mfipm_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1208_5435_amd import mfipm
    return mfipm.load_library()


def test_header_declares_expected_entry_points():
    decl = _declared()
    for name in ("mfipm_create", "mfipm_solve", "mfipm_solve_batched", "mfipm_backward", "mfipm_destroy"):
        assert name in decl
    from paper_1208_5435_amd import mfipm
    assert sorted(mfipm.EXPORTS) == decl


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_param_defaults_match_paper_and_oracle(lib):
    from paper_1208_5435_amd import mfipm
    p = mfipm.Params()
    assert lib.mfipm_params_default(ctypes.byref(p)) == 0
    with open(os.path.join(ROOT, "tests", "golden", "paper_params.json")) as f:
        gold = json.load(f)["values"]
    for k, e in gold.items():
        assert getattr(p, k) == e["value"], k
    o = R.Params()
    for k, _ in mfipm.Params._fields_:
        assert getattr(p, k) == getattr(o, k), k


def test_params_default_rejects_null(lib):
    assert lib.mfipm_params_default(None) == -1


def test_status_strings(lib):
    for code in range(-6, 8):
        s = lib.mfipm_status_string(code)
        assert s and s != b"unknown", code
    assert lib.mfipm_status_string(99) == b"unknown"


def test_create_rejects_bad_params(lib):
    """Parameter checks happen before any device query."""
    from paper_1208_5435_amd import mfipm
    p = mfipm.Params()
    lib.mfipm_params_default(ctypes.byref(p))
    p.tol = -1.0
    h = ctypes.c_void_p()
    assert lib.mfipm_create(ctypes.byref(h), ctypes.byref(p), None) == -1
    assert lib.mfipm_create(None, ctypes.byref(p), None) == -1
