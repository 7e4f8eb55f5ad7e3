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


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmhlp.so not built (run __graft_entry__.build())")
def test_geometry_create_validates_before_any_device_work():
    """Argument checks of mhlp_geometry_create return before the library touches
    the device (the node pointer is a placeholder and is never read)."""
    lib = ctypes.CDLL(LIB)
    lib.mhlp_geometry_create.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_void_p)]
    lib.mhlp_last_error.restype = ctypes.c_char_p
    fake = ctypes.c_void_p(4096)
    out = ctypes.c_void_p()

    def call(nc, offs, npp, soa=fake):
        arr = (ctypes.c_int32 * len(offs))(*offs) if offs is not None else None
        return lib.mhlp_geometry_create(nc, arr, npp, soa, None, None, ctypes.byref(out))

    assert call(1, [0, 8], 8) == -3            # MHLP_UNSUPPORTED: 16 nodes per panel only
    assert b"16" in lib.mhlp_last_error()
    assert call(0, [0], 16) == -1              # no curve
    assert call(1, [1, 8], 16) == -1           # offsets must start at 0
    assert call(2, [0, 4, 4], 16) == -1        # an empty curve
    assert call(2, [0, 6, 5], 16) == -1        # decreasing
    assert call(1, None, 16) == -1             # no offsets
    assert call(1, [0, 8], 16, soa=None) == -1  # no node data
    assert out.value is None
