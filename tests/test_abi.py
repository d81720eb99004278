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


def _lib():
    from paper_2211_10769_amd import _lib as L
    return L.load()


def test_null_context_is_rejected_everywhere():
    # every entry point that takes a context answers SWH_E_INVAL to NULL
    # before touching the device (runs without a GPU)
    from paper_2211_10769_amd import _lib as L
    lib = _lib()
    skip = {"swh_create", "swh_destroy", "swh_last_error", "swh_db_destroy", "swh_model_destroy",
            "swh_align_dev_noalloc"}
    for name, (res, args) in L.SIGNATURES.items():
        if name in skip:
            continue
        assert args[0] is ctypes.c_void_p, name
        fn = getattr(lib, name)
        call = [None] + [0 if a in (ctypes.c_int, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64) else
                         0.0 if a is ctypes.c_double else None for a in args[1:]]
        assert fn(*call) == -1, name
    assert lib.swh_last_error(None) == b"no context"
    assert lib.swh_create(0, None) == -1
    lib.swh_destroy(None)
    lib.swh_db_destroy(None)
    lib.swh_model_destroy(None)


def test_option_constants_match_header():
    from paper_2211_10769_amd import _lib as L
    text = open(HEADER).read()
    vals = dict(re.findall(r"SWH_OPT_([A-Z_0-9]+)\s*=\s*(\d+)", text))
    assert {k.lower(): int(v) for k, v in vals.items()} == {
        {"rows_per_lane": "rows_per_lane"}.get(k, k): v for k, v in L.OPTIONS.items()}


def _extern_c_functions():
    csrc = os.path.join(ROOT, "paper_2211_10769_amd", "csrc")
    src = open(os.path.join(csrc, "capi.cpp")).read()
    body = src[src.index('extern "C" {'):]
    # the entry point that allocates nothing lives beside its static array
    body += "\n" + open(os.path.join(csrc, "noalloc.hip")).read().split('extern "C"', 1)[1]
    funcs = {}
    for m in re.finditer(r"\n\s*(swh_status|void|const char \*)\s*(swh_[a-z_0-9]+)\(", body):
        start = m.end()
        depth, i = 0, body.index("{", start)
        j = i
        while True:
            if body[j] == "{":
                depth += 1
            elif body[j] == "}":
                depth -= 1
                if depth == 0:
                    break
            j += 1
        funcs[m.group(2)] = (m.group(1), body[i:j + 1])
    return funcs


def test_every_entry_point_sits_behind_the_exception_barrier():
    # no exception may cross the C ABI: every entry point either runs its body
    # in guarded() (std::bad_alloc -> SWH_E_NOMEM, anything else ->
    # SWH_E_DEVICE), or is a void destructor wrapped in try/catch(...), or
    # does nothing that can throw (flag stores, reads of plain fields)
    funcs = _extern_c_functions()
    assert set(funcs) == set(_declared()), set(funcs) ^ set(_declared())
    no_throw = {"swh_last_error", "swh_cancel", "swh_get_option", "swh_tune_get"}
    caught = {"swh_tune_save"}   # file output only, inside try/catch(...)
    for name, (ret, body) in funcs.items():
        if name in no_throw:
            assert "std::string" not in body and "new " not in body and "vector" not in body, name
        elif name in caught:
            assert "catch (...)" in body, name
        elif ret == "void" or name == "swh_align_dev_noalloc":
            assert "catch (...)" in body, name
        else:
            assert "guarded(" in body, name
