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
