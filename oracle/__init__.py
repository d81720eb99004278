"""CPU oracle for the Smith-Waterman hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library neither imports nor
links anything from here, and nothing here imports the GPU library.

``liboracle.so`` is built from ``swh_oracle.c`` (plain C, 64-bit integer DP);
``brute.py`` enumerates alignments exhaustively on tiny inputs; ``mlp.py``
holds the float64 reference of the score-prediction network.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "swh_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, E_INVAL, E_ALPHABET, E_NOMEM, E_RANGE = 0, -1, -2, -3, -4


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain -O2, no vector tricks)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        i64p = ctypes.POINTER(ctypes.c_int64)
        cstr = ctypes.c_char_p
        L.orc_sw_align.argtypes = [cstr, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                   cstr, ctypes.c_int64, cstr, ctypes.c_int64, ctypes.c_int,
                                   ctypes.c_int64, i64p, i64p, ctypes.c_char_p, ctypes.c_int64, i64p]
        L.orc_sw_end.argtypes = [cstr, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                 cstr, ctypes.c_int64, cstr, ctypes.c_int64, i64p, i64p, i64p]
        L.orc_sw_coords_mt.argtypes = [cstr, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                       cstr, ctypes.c_int64, cstr, ctypes.c_int64, ctypes.c_int,
                                       ctypes.c_int64, ctypes.c_int64, i64p, i64p]
        L.orc_sw_end_mt.argtypes = [cstr, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                    cstr, ctypes.c_int64, cstr, ctypes.c_int64, ctypes.c_int,
                                    ctypes.c_int64, ctypes.c_int64, i64p, i64p, i64p]
        L.orc_global_cigar.argtypes = [cstr, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                       cstr, ctypes.c_int64, cstr, ctypes.c_int64, i64p,
                                       ctypes.c_char_p, ctypes.c_int64, i64p]
        L.orc_hw_align.argtypes = [cstr, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                   cstr, ctypes.c_int64, cstr, ctypes.c_int64, ctypes.c_int,
                                   i64p, i64p, ctypes.c_char_p, ctypes.c_int64, i64p]
        L.orc_ov_align.argtypes = L.orc_hw_align.argtypes
        L.orc_db_scores.argtypes = [cstr, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_int, ctypes.c_void_p]
        L.orc_topk.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                               ctypes.c_void_p, ctypes.c_void_p]
        for f in (L.orc_sw_align, L.orc_sw_end, L.orc_sw_coords_mt, L.orc_sw_end_mt, L.orc_global_cigar, L.orc_hw_align, L.orc_ov_align,
                  L.orc_db_scores, L.orc_topk):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def _as_bytes(s) -> bytes:
    if isinstance(s, str):
        return s.encode("ascii")
    if isinstance(s, np.ndarray):
        return s.tobytes()
    return bytes(s)


def _mat(matrix) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(matrix, dtype=np.int8))


def sw_align(a, b, scoring, want_cigar: bool = True, max_cells: int = 400_000_000):
    """Local alignment: returns dict(score, q_begin, q_end, t_begin, t_end, cigar).

    Coordinates are 0-based inclusive; all -1 and cigar '' when score == 0.
    """
    alphabet, matrix, o, e = scoring
    a, b = _as_bytes(a), _as_bytes(b)
    M = _mat(matrix)
    score = ctypes.c_int64()
    coords = (ctypes.c_int64 * 4)()
    clen = ctypes.c_int64()
    cap = len(a) + len(b) + 64 if want_cigar else 1
    cbuf = ctypes.create_string_buffer(2 * cap + 16)
    rc = lib().orc_sw_align(alphabet.encode(), len(alphabet), M.ctypes.data, o, e,
                            a, len(a), b, len(b), int(want_cigar), max_cells,
                            ctypes.byref(score), coords, cbuf, len(cbuf), ctypes.byref(clen))
    if rc != OK:
        raise OracleError(rc, "sw_align")
    return dict(score=score.value, q_begin=coords[0], q_end=coords[1], t_begin=coords[2],
                t_end=coords[3], cigar=cbuf.value.decode() if want_cigar else None)


def sw_end(a, b, scoring):
    """Score-only forward pass: (score, q_end, t_end), ends -1 when score == 0."""
    alphabet, matrix, o, e = scoring
    a, b = _as_bytes(a), _as_bytes(b)
    M = _mat(matrix)
    s, qe, te = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    rc = lib().orc_sw_end(alphabet.encode(), len(alphabet), M.ctypes.data, o, e, a, len(a), b, len(b),
                          ctypes.byref(s), ctypes.byref(qe), ctypes.byref(te))
    if rc != OK:
        raise OracleError(rc, "sw_end")
    return s.value, qe.value, te.value


def sw_coords_mt(a, b, scoring, threads: int | None = None, band: int = 256, chunk: int = 4096):
    """Score, end and start of one (long) pair with the banded threaded pass:
    dict(score, q_begin, q_end, t_begin, t_end), the same values as
    sw_align(..., want_cigar=False).  band / chunk / threads set only the
    running time (rows per band, columns per hand-over chunk, worker threads)."""
    alphabet, matrix, o, e = scoring
    a, b = _as_bytes(a), _as_bytes(b)
    M = _mat(matrix)
    s = ctypes.c_int64()
    co = (ctypes.c_int64 * 4)()
    rc = lib().orc_sw_coords_mt(alphabet.encode(), len(alphabet), M.ctypes.data, o, e, a, len(a), b, len(b),
                                int(threads or os.cpu_count() or 1), band, chunk, ctypes.byref(s), co)
    if rc != OK:
        raise OracleError(rc, "sw_coords_mt")
    return dict(score=s.value, q_begin=co[0], q_end=co[1], t_begin=co[2], t_end=co[3])


def sw_end_mt(a, b, scoring, threads: int | None = None, band: int = 256, chunk: int = 4096):
    """Score-only banded threaded pass: (score, q_end, t_end), as sw_end."""
    alphabet, matrix, o, e = scoring
    a, b = _as_bytes(a), _as_bytes(b)
    M = _mat(matrix)
    s, qe, te = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    rc = lib().orc_sw_end_mt(alphabet.encode(), len(alphabet), M.ctypes.data, o, e, a, len(a), b, len(b),
                             int(threads or os.cpu_count() or 1), band, chunk, ctypes.byref(s), ctypes.byref(qe),
                             ctypes.byref(te))
    if rc != OK:
        raise OracleError(rc, "sw_end_mt")
    return s.value, qe.value, te.value


def global_cigar(a, b, scoring):
    """Global optimum of a vs b and the canonical CIGAR of the greedy walk."""
    alphabet, matrix, o, e = scoring
    a, b = _as_bytes(a), _as_bytes(b)
    M = _mat(matrix)
    g = ctypes.c_int64()
    clen = ctypes.c_int64()
    cbuf = ctypes.create_string_buffer(2 * (len(a) + len(b)) + 16)
    rc = lib().orc_global_cigar(alphabet.encode(), len(alphabet), M.ctypes.data, o, e,
                                a, len(a), b, len(b), ctypes.byref(g), cbuf, len(cbuf),
                                ctypes.byref(clen))
    if rc != OK:
        raise OracleError(rc, "global_cigar")
    return g.value, cbuf.value.decode()


def hw_align(a, b, scoring, want_cigar: bool = True):
    """Semi-global alignment (whole query, free target ends): dict(score,
    q_begin, q_end, t_begin, t_end[, cigar]), the readings in swh_oracle.c."""
    alphabet, matrix, o, e = scoring
    a, b = _as_bytes(a), _as_bytes(b)
    M = _mat(matrix)
    S = ctypes.c_int64()
    co = (ctypes.c_int64 * 4)()
    clen = ctypes.c_int64()
    cbuf = ctypes.create_string_buffer(2 * (len(a) + len(b)) + 16)
    rc = lib().orc_hw_align(alphabet.encode(), len(alphabet), M.ctypes.data, o, e, a, len(a), b, len(b),
                            1 if want_cigar else 0, ctypes.byref(S), co, cbuf, len(cbuf), ctypes.byref(clen))
    if rc != OK:
        raise OracleError(rc, "hw_align")
    out = dict(score=S.value, q_begin=co[0], q_end=co[1], t_begin=co[2], t_end=co[3])
    if want_cigar:
        out["cigar"] = cbuf.value.decode()
    return out


def ov_align(a, b, scoring, want_cigar: bool = True):
    """Overlap alignment (end gaps of both sequences free): dict(score,
    q_begin, q_end, t_begin, t_end[, cigar]), the readings in swh_oracle.c."""
    alphabet, matrix, o, e = scoring
    a, b = _as_bytes(a), _as_bytes(b)
    M = _mat(matrix)
    S = ctypes.c_int64()
    co = (ctypes.c_int64 * 4)()
    clen = ctypes.c_int64()
    cbuf = ctypes.create_string_buffer(2 * (len(a) + len(b)) + 16)
    rc = lib().orc_ov_align(alphabet.encode(), len(alphabet), M.ctypes.data, o, e, a, len(a), b, len(b),
                            1 if want_cigar else 0, ctypes.byref(S), co, cbuf, len(cbuf), ctypes.byref(clen))
    if rc != OK:
        raise OracleError(rc, "ov_align")
    out = dict(score=S.value, q_begin=co[0], q_end=co[1], t_begin=co[2], t_end=co[3])
    if want_cigar:
        out["cigar"] = cbuf.value.decode()
    return out


def concat(seqs):
    """List of byte strings -> (concatenated bytes, int64 offsets)."""
    bs = [_as_bytes(s) for s in seqs]
    off = np.zeros(len(bs) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(x) for x in bs])
    return b"".join(bs), off


def db_scores(queries, db, scoring, threads: int | None = None) -> np.ndarray:
    """All local scores, shape (nq, ndb), int64."""
    alphabet, matrix, o, e = scoring
    if isinstance(queries, tuple):
        q_cat, q_off = queries
    else:
        q_cat, q_off = concat(queries)
    if isinstance(db, tuple):
        d_cat, d_off = db
    else:
        d_cat, d_off = concat(db)
    q_off = np.ascontiguousarray(q_off, dtype=np.int64)
    d_off = np.ascontiguousarray(d_off, dtype=np.int64)
    nq, ndb = len(q_off) - 1, len(d_off) - 1
    out = np.zeros((nq, ndb), dtype=np.int64)
    qb = np.frombuffer(_as_bytes(q_cat), dtype=np.uint8) if len(q_cat) else np.zeros(1, np.uint8)
    dbb = np.frombuffer(_as_bytes(d_cat), dtype=np.uint8) if len(d_cat) else np.zeros(1, np.uint8)
    M = _mat(matrix)
    rc = lib().orc_db_scores(alphabet.encode(), len(alphabet), M.ctypes.data, o, e,
                             nq, qb.ctypes.data, q_off.ctypes.data, ndb, dbb.ctypes.data,
                             d_off.ctypes.data, int(threads or os.cpu_count() or 1), out.ctypes.data)
    if rc != OK:
        raise OracleError(rc, "db_scores")
    return out


def topk(scores: np.ndarray, k: int):
    """Per row: indices and scores of the k best (score desc, index asc); -1 padding."""
    s = np.ascontiguousarray(scores, dtype=np.int64)
    nr, nc = s.shape
    idx = np.zeros((nr, k), dtype=np.int64)
    sc = np.zeros((nr, k), dtype=np.int64)
    rc = lib().orc_topk(nr, nc, s.ctypes.data, k, idx.ctypes.data, sc.ctypes.data)
    if rc != OK:
        raise OracleError(rc, "topk")
    return idx, sc
