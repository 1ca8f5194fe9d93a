"""The C-ABI library loads and exports every symbol the public header declares.

No compute calls: this runs without a GPU.
"""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kry.h")
LIB = os.path.join(ROOT, "paper_1707_00023_amd", "libkry.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kry_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    syms = declared_symbols()
    for name in ("kry_create", "kry_destroy", "kry_expv", "kry_solve_multifreq",
                 "kry_last_error", "kry_apply", "kry_arnoldi", "kry_stationary"):
        assert name in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="libkry.so not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [s for s in declared_symbols() if s not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(LIB)
    for s in declared_symbols():
        assert hasattr(lib, s)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libkry.so not built")
def test_binding_declares_the_same_symbols():
    import paper_1707_00023_amd as kry
    assert sorted(kry.EXPORTED) == declared_symbols()


def test_binding_fails_loudly_without_library(tmp_path):
    import paper_1707_00023_amd as kry
    with pytest.raises(RuntimeError, match="not found"):
        kry._lib = None
        kry.load_library(str(tmp_path / "missing.so"))
    kry._lib = None
