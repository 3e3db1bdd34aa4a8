"""The C-ABI library loads and exports every entry point include/osmpm.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "osmpm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(osmpm_[A-Za-z0-9_]+)\s*\(", src)))


def test_header_declares_binding_symbols():
    from paper_2605_09097_amd import binding

    assert _declared() == sorted(binding.ABI_SYMBOLS)


def test_library_exports_every_declared_symbol():
    from paper_2605_09097_amd import binding

    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(binding.LIB_PATH)
    missing = [s for s in _declared() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_declares_signatures():
    from paper_2605_09097_amd import binding

    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    L = binding.lib()
    for s in binding.ABI_SYMBOLS:
        assert getattr(L, s).restype is not None or s in ("osmpm_ctx_destroy", "osmpm_domain_destroy", "osmpm_batch_destroy")
