"""The C ABI library loads without a GPU and exports every function that
include/rs.h declares; the binding's signature table covers the same set."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rs_[a-z0-9_]+)\s*\(", text)))


def test_header_parses():
    names = declared_functions()
    assert "rs_run" in names and "rs_graph_create" in names and len(names) >= 20


def test_library_exports_all_declared():
    import paper_2010_08423_amd as R

    if not os.path.exists(R.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(R.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    import paper_2010_08423_amd as R

    assert sorted(R._SIGNATURES) == declared_functions()


def test_status_strings_without_gpu():
    import paper_2010_08423_amd as R

    if not os.path.exists(R.LIB_PATH):
        pytest.skip("library not built")
    assert R.status_str(R.RS_EINVAL).startswith("RS_EINVAL")
    assert b"gfx950" in R.library().rs_version()
