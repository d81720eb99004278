"""MI355X-native Smith-Waterman engine: Python binding of libswh.so.

    import paper_2211_10769_amd as swh
    eng = swh.Engine()                       # one HIP context on device 0
    r = eng.align(query, target, swh.dna_scoring(), mode="cigar")

Sequences are ASCII ``bytes``/``str``/uint8 numpy arrays (host) or uint8
torch tensors on the GPU (``align_dev``).  All arithmetic runs in the HIP
library; this module only marshals arguments.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import MODE_CIGAR, MODE_COORDS, MODE_SCORE, STATUS_NAMES

_MODES = {"score": MODE_SCORE, "coords": MODE_COORDS, "cigar": MODE_CIGAR}


class SwhError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _bytes(x) -> bytes:
    if isinstance(x, str):
        return x.encode("ascii")
    if isinstance(x, np.ndarray):
        return np.ascontiguousarray(x, dtype=np.uint8).tobytes()
    return bytes(x)


class Scoring:
    """Alphabet, int8 substitution matrix (query symbol x target symbol), gap open/extend."""

    def __init__(self, alphabet: str, matrix, gap_open: int, gap_extend: int):
        self.alphabet = alphabet
        self.matrix = np.ascontiguousarray(np.asarray(matrix, dtype=np.int8))
        self.gap_open = int(gap_open)
        self.gap_extend = int(gap_extend)
        self._ab = alphabet.encode("ascii")
        self.c = _lib.swh_scoring(self._ab, len(alphabet), self.matrix.ctypes.data,
                                  self.gap_open, self.gap_extend)

    @classmethod
    def of(cls, sc) -> "Scoring":
        return sc if isinstance(sc, Scoring) else cls(*sc)


class Engine:
    """One library context (device, stream, grow-only device buffers)."""

    def __init__(self, device: int = 0):
        self.L = _lib.load()
        h = ctypes.c_void_p()
        st = self.L.swh_create(device, ctypes.byref(h))
        if st != 0:
            raise SwhError(st, f"swh_create(device={device}) failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.swh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != 0:
            raise SwhError(st, self.L.swh_last_error(self.h).decode(errors="replace"))

    @staticmethod
    def _result(a: _lib.swh_alignment, cigar, stats):
        r = dict(score=a.score, q_begin=a.q_begin, q_end=a.q_end, t_begin=a.t_begin, t_end=a.t_end,
                 flags=a.flags)
        if cigar is not None:
            r["cigar"] = cigar
        if stats is not None:
            r["stats"] = {k: getattr(stats, k) for k, _ in stats._fields_[2:]}
        return r

    def align(self, query, target, scoring, mode: str = "cigar", stats: bool = False):
        """Local alignment of host sequences; returns dict(score, q_begin, q_end, t_begin, t_end[, cigar])."""
        sc = Scoring.of(scoring)
        q, t = _bytes(query), _bytes(target)
        m = _MODES[mode]
        out = _lib.swh_alignment()
        st_obj = _lib.swh_stats(ctypes.sizeof(_lib.swh_stats)) if stats else None
        cap = 2 * (len(q) + len(t)) + 16 if m == MODE_CIGAR else 0
        buf = ctypes.create_string_buffer(cap) if cap else None
        clen = ctypes.c_int64()
        st = self.L.swh_align(self.h, q, len(q), t, len(t), ctypes.byref(sc.c), m, ctypes.byref(out),
                              buf, cap, ctypes.byref(clen),
                              ctypes.byref(st_obj) if st_obj is not None else None)
        self._check(st)
        return self._result(out, buf.value.decode() if buf is not None else None, st_obj)

    def align_dev(self, q_tensor, t_tensor, scoring, mode: str = "score", stream=None, stats: bool = False):
        """Local alignment of uint8 ASCII torch tensors already on the GPU."""
        sc = Scoring.of(scoring)
        m = _MODES[mode]
        out = _lib.swh_alignment()
        st_obj = _lib.swh_stats(ctypes.sizeof(_lib.swh_stats)) if stats else None
        cap = 2 * (q_tensor.numel() + t_tensor.numel()) + 16 if m == MODE_CIGAR else 0
        buf = ctypes.create_string_buffer(cap) if cap else None
        clen = ctypes.c_int64()
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        st = self.L.swh_align_dev(self.h, q_tensor.data_ptr(), q_tensor.numel(), t_tensor.data_ptr(),
                                  t_tensor.numel(), ctypes.byref(sc.c), m, stream, ctypes.byref(out), buf,
                                  cap, ctypes.byref(clen),
                                  ctypes.byref(st_obj) if st_obj is not None else None)
        self._check(st)
        return self._result(out, buf.value.decode() if buf is not None else None, st_obj)


def _concat(seqs):
    """list of sequences (or (concatenated bytes, offsets)) -> (uint8 array, int64 offsets)."""
    if isinstance(seqs, tuple):
        cat, off = seqs
        cat = np.frombuffer(_bytes(cat), dtype=np.uint8) if not isinstance(cat, np.ndarray) else cat
        return np.ascontiguousarray(cat, dtype=np.uint8), np.ascontiguousarray(off, dtype=np.int64)
    bs = [_bytes(x) for x in seqs]
    off = np.zeros(len(bs) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(b) for b in bs])
    cat = np.frombuffer(b"".join(bs), dtype=np.uint8) if bs else np.zeros(0, np.uint8)
    return np.ascontiguousarray(cat), off


class Database:
    """An encoded database on the device (swh_db); scoring fixed at creation."""

    def __init__(self, engine: Engine, seqs, scoring):
        self.eng = engine
        self.sc = Scoring.of(scoring)
        cat, off = _concat(seqs)
        self.ndb = len(off) - 1
        h = ctypes.c_void_p()
        catp = cat.ctypes.data if len(cat) else None
        st = engine.L.swh_db_create(engine.h, self.ndb, catp, off.ctypes.data, ctypes.byref(self.sc.c),
                                    ctypes.byref(h))
        engine._check(st)
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.eng.L.swh_db_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _stats(st):
        return {k: getattr(st, k) for k, _ in st._fields_[2:]}

    def search(self, queries, k: int = 10):
        """Top-k hits per query: (indices int64 [nq, k], scores int32 [nq, k], stats dict)."""
        cat, off = _concat(queries)
        nq = len(off) - 1
        hits = (_lib.swh_hit * max(1, nq * k))()
        st = _lib.swh_search_stats(ctypes.sizeof(_lib.swh_search_stats))
        rc = self.eng.L.swh_db_search(self.eng.h, self.h, nq, cat.ctypes.data if len(cat) else None,
                                      off.ctypes.data, k, hits, ctypes.byref(st))
        self.eng._check(rc)
        idx = np.array([hits[i].db_index for i in range(nq * k)], dtype=np.int64).reshape(nq, k)
        sco = np.array([hits[i].score for i in range(nq * k)], dtype=np.int32).reshape(nq, k)
        return idx, sco, self._stats(st)

    def scores(self, queries):
        """All scores: int32 array [nq, ndb] and stats dict."""
        cat, off = _concat(queries)
        nq = len(off) - 1
        out = np.zeros((nq, self.ndb), dtype=np.int32)
        st = _lib.swh_search_stats(ctypes.sizeof(_lib.swh_search_stats))
        rc = self.eng.L.swh_db_scores(self.eng.h, self.h, nq, cat.ctypes.data if len(cat) else None,
                                      off.ctypes.data, out.ctypes.data, ctypes.byref(st))
        self.eng._check(rc)
        return out, self._stats(st)


def dna_scoring(match: int = 1, mismatch: int = -3, gap_open: int = 5, gap_extend: int = 2) -> Scoring:
    mat = np.full((4, 4), mismatch, dtype=np.int8)
    np.fill_diagonal(mat, match)
    return Scoring("ACGT", mat, gap_open, gap_extend)
