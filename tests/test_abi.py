"""The C-ABI library loads and exports every entry point include/swh.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "swh.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(swh_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ("swh_create", "swh_destroy", "swh_last_error", "swh_align", "swh_align_dev"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2211_10769_amd import _lib
    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2211_10769_amd import _lib
    assert set(_declared()) <= set(_lib.SIGNATURES)


def test_struct_layouts_match_header():
    from paper_2211_10769_amd import _lib
    assert ctypes.sizeof(_lib.swh_alignment) == 40
    assert ctypes.sizeof(_lib.swh_scoring) == 32
    assert _lib.swh_alignment.q_begin.offset == 8


def test_mode_constants_match_header():
    # every #define of the header that the binding mirrors has the same value
    from paper_2211_10769_amd import _lib
    text = open(HEADER).read()
    defs = {k: int(v, 0) for k, v in re.findall(r"#define\s+SWH_([A-Z_0-9]+)\s+(0x[0-9a-fA-F]+|\d+)\b", text)}
    for name in ("GLOBAL", "SEMIGLOBAL", "OVERLAP"):
        assert getattr(_lib, name) == defs[name], name
    forms = [defs["GLOBAL"], defs["SEMIGLOBAL"], defs["OVERLAP"]]
    # single bits, disjoint from each other and from the mode values
    assert all(f & (f - 1) == 0 for f in forms) and len(set(forms)) == 3
    assert all(f > 0xFF for f in forms)
