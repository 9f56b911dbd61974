"""The C-ABI library loads and exports every function include/rpfeti.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rpfeti.h")
LIB = os.path.join(ROOT, "paper_1208_6387_amd", "librpfeti.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "for")))


def test_header_declares_the_four_calls():
    names = declared_functions()
    for n in ("pattern_factor", "pattern_condense", "feti_apply", "block_krylov_solve"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_signature_table_matches_header():
    from paper_1208_6387_amd import _lib
    assert sorted(_lib.EXPORTS) == declared_functions()
    lib = _lib.load()
    assert lib.rpf_version() >= 100


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1208_6387_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        _lib.load()
