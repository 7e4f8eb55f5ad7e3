"""The C-ABI library loads and exports every symbol the public header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mhlp.h")
LIB = os.path.join(ROOT, "paper_1908_07392_amd", "libmhlp.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mhlp_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("mhlp_eval_slp", "mhlp_eval_dlp", "mhlp_apply_bie_operator", "mhlp_gmres_solve",
              "mhlp_geometry_create", "mhlp_plan_create"):
        assert s in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmhlp.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmhlp.so not built (run __graft_entry__.build())")
def test_binding_signatures_cover_header():
    from paper_1908_07392_amd import mhlp
    assert set(declared_symbols()) <= set(mhlp._SIGS)
    lib = mhlp.load()
    assert lib.mhlp_last_error() is not None
