"""The C-ABI library loads on the CPU and exports every function declared
in include/ppcg.h (no compute call without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1407_7506_amd", "libppcg.so")


def declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(ppcg_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_declares_entry_points():
    d = declared()
    for must in ("ppcg_create", "ppcg_solve", "ppcg_destroy", "ppcg_last_error", "ppcg_apply_h"):
        assert must in d


@pytest.mark.skipif(not os.path.exists(LIB), reason="libppcg.so not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_refuses_missing_library(monkeypatch):
    from paper_1407_7506_amd import binding
    monkeypatch.setattr(binding, "LIB_PATH", "/nonexistent/libppcg.so")
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(RuntimeError):
        binding.lib()


def test_autograd_module_imports_without_gpu():
    from paper_1407_7506_amd import autograd
    assert hasattr(autograd, "EigDensity") and hasattr(autograd, "EigConfig")
