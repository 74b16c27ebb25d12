"""CPU-side checks of the C-ABI library: it loads and exports every symbol the
header declares, and the binding declares exactly those symbols.  No compute
calls (no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "laph.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(laph_[A-Za-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for need in ["laph_create", "laph_apply_dslash", "laph_apply_clover", "laph_solve", "laph_perambulator"]:
        assert need in names


def test_library_exports_every_declared_symbol():
    from paper_2510_26313_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("liblaph.so not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(_lib.EXPORTED) == _declared()


def test_binding_refuses_to_run_without_library(tmp_path):
    from paper_2510_26313_amd import _lib
    with pytest.raises(RuntimeError):
        _lib.load(str(tmp_path / "nonexistent.so"))


def test_param_struct_layout_matches_header():
    from paper_2510_26313_amd import _lib
    src = open(HEADER).read()
    body = re.search(r"typedef struct \{([^{}]*)\} laph_solve_params;", src, re.S).group(1)
    fields = re.findall(r"\b(int|double)\s+([a-z0-9_]+);", body)
    assert [f[1] for f in fields] == [f[0] for f in _lib.SolveParams._fields_]
    body = re.search(r"typedef struct \{([^{}]*)\} laph_rhs_stats;", src, re.S).group(1)
    fields = re.findall(r"\b(int|double)\s+([a-z0-9_]+);", body)
    assert [f[1] for f in fields] == [f[0] for f in _lib.RhsStats._fields_]
