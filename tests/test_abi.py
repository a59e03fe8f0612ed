"""CPU checks of the C ABI library: it loads, exports every declared entry
point, and the product package never reaches the oracle."""
import ast
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dcsched.h")
PKG = os.path.join(ROOT, "paper_1909_07673_amd")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dc_[a-z_]+)\s*\(", txt)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ("dc_create", "dc_submit_request", "dc_schedule", "dc_release", "dc_destroy", "dc_strerror"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1909_07673_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    L = ctypes.CDLL(binding.LIB_PATH)          # loads without touching a GPU
    for n in _declared():
        assert hasattr(L, n)
    L.dc_strerror.restype = ctypes.c_char_p
    assert L.dc_strerror(-1) == b"invalid argument"


def test_product_never_imports_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            path = os.path.join(dirpath, f)
            if f.endswith(".py"):
                tree = ast.parse(open(path).read())
                for node in ast.walk(tree):
                    if isinstance(node, ast.Import):
                        assert all(not a.name.startswith("oracle") for a in node.names), path
                    if isinstance(node, ast.ImportFrom):
                        assert not (node.module or "").startswith("oracle"), path
            if f.endswith((".hip", ".hpp", ".cpp", ".h")):
                assert "oracle" not in open(path).read().lower(), path


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1909_07673_amd import binding
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        binding.lib()
