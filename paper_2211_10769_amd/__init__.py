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
_ALIGNMENTS = {"local": 0, "global": _lib.GLOBAL, "semiglobal": _lib.SEMIGLOBAL,
               "overlap": _lib.OVERLAP}


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


# numpy view of swh_alignment (include/swh.h): score, flags, four int64 coordinates
_ALIGNMENT_DTYPE = np.dtype([("score", "<i4"), ("flags", "<u4"), ("q_begin", "<i8"), ("q_end", "<i8"),
                             ("t_begin", "<i8"), ("t_end", "<i8")])


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

    def set_option(self, name: str, value: int):
        """Set a context option (speed, memory or diagnostics only): rows_per_lane,
        grid, band_rows, tb_leaf, graph, prune, mem_cap, int16, inter_max, fault_nomem."""
        self._check(self.L.swh_set_option(self.h, _lib.OPTIONS[name], int(value)))

    def get_option(self, name: str) -> int:
        v = ctypes.c_int64()
        self._check(self.L.swh_get_option(self.h, _lib.OPTIONS[name], ctypes.byref(v)))
        return v.value

    def cancel(self) -> int:
        """Ask the call running on this context (in another thread) to stop; it then
        raises SwhError with status SWH_E_CANCELLED."""
        return self.L.swh_cancel(self.h)

    @staticmethod
    def _result(a: _lib.swh_alignment, cigar, stats):
        r = dict(score=a.score, q_begin=a.q_begin, q_end=a.q_end, t_begin=a.t_begin, t_end=a.t_end,
                 flags=a.flags)
        if cigar is not None:
            r["cigar"] = cigar
        if stats is not None:
            r["stats"] = {k: getattr(stats, k) for k, _ in stats._fields_[2:]}
        return r

    def align(self, query, target, scoring, mode: str = "cigar", stats: bool = False, alignment: str = "local"):
        """Local (or, alignment="global", Needleman-Wunsch; alignment="semiglobal",
        the whole query against part of the target; alignment="overlap", end gaps free) alignment of host sequences;
        returns dict(score, q_begin, q_end, t_begin, t_end[, cigar])."""
        sc = Scoring.of(scoring)
        q, t = _bytes(query), _bytes(target)
        m = _MODES[mode]
        g = _ALIGNMENTS[alignment]
        out = _lib.swh_alignment()
        st_obj = _lib.swh_stats(ctypes.sizeof(_lib.swh_stats)) if stats else None
        cap = 2 * (len(q) + len(t)) + 16 if m == MODE_CIGAR else 0
        buf = np.empty(cap, dtype=np.uint8) if cap else None    # written up to the CIGAR's length only
        clen = ctypes.c_int64()
        st = self.L.swh_align(self.h, q, len(q), t, len(t), ctypes.byref(sc.c), m | g, ctypes.byref(out),
                              buf.ctypes.data if buf is not None else None, cap, ctypes.byref(clen),
                              ctypes.byref(st_obj) if st_obj is not None else None)
        self._check(st)
        return self._result(out, buf[:clen.value].tobytes().decode() if buf is not None else None, st_obj)

    def align_dev(self, q_tensor, t_tensor, scoring, mode: str = "score", stream=None, stats: bool = False,
                  alignment: str = "local"):
        """Local (or global) alignment of uint8 ASCII torch tensors already on the GPU."""
        sc = Scoring.of(scoring)
        m = _MODES[mode]
        g = _ALIGNMENTS[alignment]
        out = _lib.swh_alignment()
        st_obj = _lib.swh_stats(ctypes.sizeof(_lib.swh_stats)) if stats else None
        cap = 2 * (q_tensor.numel() + t_tensor.numel()) + 16 if m == MODE_CIGAR else 0
        buf = np.empty(cap, dtype=np.uint8) if cap else None    # written up to the CIGAR's length only
        clen = ctypes.c_int64()
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        st = self.L.swh_align_dev(self.h, q_tensor.data_ptr(), q_tensor.numel(), t_tensor.data_ptr(),
                                  t_tensor.numel(), ctypes.byref(sc.c), m | g, stream, ctypes.byref(out),
                                  buf.ctypes.data if buf is not None else None, cap, ctypes.byref(clen),
                                  ctypes.byref(st_obj) if st_obj is not None else None)
        self._check(st)
        return self._result(out, buf[:clen.value].tobytes().decode() if buf is not None else None, st_obj)

    def align_batch(self, queries, targets, scoring, mode: str = "cigar", stats: bool = False,
                    alignment: str = "local"):
        """Many pairs (query i vs target i) in one call; returns a list of result dicts
        (and the summed stats dict when stats=True).  alignment="global": Needleman-Wunsch."""
        sc = Scoring.of(scoring)
        qcat, qoff = _concat(queries)
        tcat, toff = _concat(targets)
        return self._batch(len(qoff) - 1, qcat.ctypes.data if len(qcat) else None, qoff,
                           tcat.ctypes.data if len(tcat) else None, toff, sc, mode, stats, alignment, None)

    def align_batch_dev(self, q_tensor, q_off, t_tensor, t_off, scoring, mode: str = "cigar", stream=None,
                        stats: bool = False, alignment: str = "local"):
        """Many pairs from concatenated uint8 ASCII torch tensors on the GPU; q_off and
        t_off are host int64 offsets (pair i = q[q_off[i]:q_off[i+1]] vs t[t_off[i]:t_off[i+1]])."""
        sc = Scoring.of(scoring)
        qoff = np.ascontiguousarray(q_off, dtype=np.int64)
        toff = np.ascontiguousarray(t_off, dtype=np.int64)
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        return self._batch(len(qoff) - 1, q_tensor.data_ptr() if q_tensor.numel() else None, qoff,
                           t_tensor.data_ptr() if t_tensor.numel() else None, toff, sc, mode, stats, alignment,
                           stream)

    def _batch(self, n, qptr, qoff, tptr, toff, sc, mode, stats, alignment, stream):
        if len(toff) - 1 != n:
            raise ValueError("queries and targets differ in count")
        m = _MODES[mode]
        g = _ALIGNMENTS[alignment]
        out = np.zeros(max(1, n), dtype=_ALIGNMENT_DTYPE)
        st_obj = _lib.swh_stats(ctypes.sizeof(_lib.swh_stats)) if stats else None
        coff = np.zeros(n + 1, dtype=np.int64)
        # the CIGAR bound (two characters per residue) can run to gigabytes:
        # np.empty reserves it without touching it, and only the bytes the
        # library writes are read back
        cap = int(2 * (qoff[-1] - qoff[0] + toff[-1] - toff[0]) + 16) if m == MODE_CIGAR else 0
        buf = np.empty(cap, dtype=np.uint8) if cap else None
        tail = [out.ctypes.data, buf.ctypes.data if buf is not None else None, cap,
                coff.ctypes.data if m == MODE_CIGAR else None, ctypes.byref(st_obj) if st_obj is not None else None]
        head = [self.h, n, qptr, qoff.ctypes.data, tptr, toff.ctypes.data, ctypes.byref(sc.c), m | g]
        if stream is None:
            self._check(self.L.swh_align_batch(*head, *tail))
        else:
            self._check(self.L.swh_align_batch_dev(*head, stream, *tail))
        cols = [out[k][:n].tolist() for k in ("score", "q_begin", "q_end", "t_begin", "t_end", "flags")]
        if m == MODE_CIGAR:
            text = buf[:int(coff[n])].tobytes().decode()
            offs = coff.tolist()
            cigars = [text[offs[i]:offs[i + 1]] for i in range(n)]
            res = [dict(score=a, q_begin=b, q_end=c, t_begin=d, t_end=e, flags=f, cigar=cg)
                   for a, b, c, d, e, f, cg in zip(*cols, cigars)]
        else:
            res = [dict(score=a, q_begin=b, q_end=c, t_begin=d, t_end=e, flags=f) for a, b, c, d, e, f in zip(*cols)]
        if stats:
            return res, {k: getattr(st_obj, k) for k, _ in st_obj._fields_[2:]}
        return res

    def autotune(self, scoring, max_rows: int = 1 << 20, cells_per_trial: float = 2e10):
        """Measure and install the strip shapes; returns the table as a list of dicts."""
        sc = Scoring.of(scoring)
        self._check(self.L.swh_autotune(self.h, ctypes.byref(sc.c), int(max_rows), float(cells_per_trial)))
        return self.tune_table()

    def autotune_db(self, scoring) -> int:
        """Measure and install the database length switch; returns it."""
        sc = Scoring.of(scoring)
        v = ctypes.c_int32()
        self._check(self.L.swh_autotune_db(self.h, ctypes.byref(sc.c), ctypes.byref(v)))
        return v.value

    def tune_save(self, path: str):
        st = self.L.swh_tune_save(self.h, path.encode())
        if st != 0:
            raise SwhError(st, f"cannot write {path}")

    def tune_load(self, path: str):
        self._check(self.L.swh_tune_load(self.h, path.encode()))

    def tune_table(self):
        arr = (_lib.swh_tune_entry * 64)()
        cnt = ctypes.c_int32()
        self._check(self.L.swh_tune_get(self.h, arr, 64, ctypes.byref(cnt)))
        return [dict(max_rows=arr[i].max_rows, rows_per_lane=arr[i].rows_per_lane,
                     waves_per_simd=arr[i].waves_per_simd) for i in range(cnt.value)]

    def set_tune_table(self, table):
        arr = (_lib.swh_tune_entry * max(1, len(table)))()
        for i, t in enumerate(table):
            arr[i] = _lib.swh_tune_entry(int(t["max_rows"]), int(t["rows_per_lane"]), int(t["waves_per_simd"]))
        self._check(self.L.swh_tune_set(self.h, arr, len(table)))


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

    def search_dev(self, q_tensor, q_off, k: int = 10, stream=None):
        """search() with the concatenated queries in a uint8 ASCII torch tensor on the GPU
        (q_off: host int64 offsets)."""
        off = np.ascontiguousarray(q_off, dtype=np.int64)
        nq = len(off) - 1
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        hits = (_lib.swh_hit * max(1, nq * k))()
        st = _lib.swh_search_stats(ctypes.sizeof(_lib.swh_search_stats))
        rc = self.eng.L.swh_db_search_dev(self.eng.h, self.h, nq, q_tensor.data_ptr() if q_tensor.numel() else None,
                                          off.ctypes.data, k, stream, hits, ctypes.byref(st))
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


def _f32(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


class Model:
    """The prefilter network (swh_model): weights on the device, feature normalisation, Adam state."""

    def __init__(self, engine: Engine, scoring, theta=None, mu=None, sd=None, seed: int = 0, _handle=None):
        self.eng = engine
        self.sc = Scoring.of(scoring) if scoring is not None else None
        if _handle is not None:
            self.h = _handle
            return
        th = _f32(theta, _lib.MODEL_PARAMS) if theta is not None else None
        m = _f32(mu, _lib.MODEL_INPUTS) if mu is not None else None
        s = _f32(sd, _lib.MODEL_INPUTS) if sd is not None else None
        h = ctypes.c_void_p()
        rc = engine.L.swh_model_create(engine.h, ctypes.byref(self.sc.c),
                                       th.ctypes.data if th is not None else None,
                                       m.ctypes.data if m is not None else None,
                                       s.ctypes.data if s is not None else None, int(seed), ctypes.byref(h))
        engine._check(rc)
        self.h = h

    @classmethod
    def load(cls, engine: Engine, path: str) -> "Model":
        h = ctypes.c_void_p()
        engine._check(engine.L.swh_model_load(engine.h, path.encode(), ctypes.byref(h)))
        return cls(engine, None, _handle=h)

    def save(self, path: str):
        self.eng._check(self.eng.L.swh_model_save(self.eng.h, self.h, path.encode()))

    def close(self):
        if getattr(self, "h", None):
            self.eng.L.swh_model_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get(self):
        th = np.zeros(_lib.MODEL_PARAMS, np.float32)
        mu = np.zeros(_lib.MODEL_INPUTS, np.float32)
        sd = np.zeros(_lib.MODEL_INPUTS, np.float32)
        self.eng._check(self.eng.L.swh_model_get(self.eng.h, self.h, th.ctypes.data, mu.ctypes.data, sd.ctypes.data))
        return th, mu, sd

    def set(self, theta=None, mu=None, sd=None):
        th = _f32(theta, _lib.MODEL_PARAMS) if theta is not None else None
        m = _f32(mu, _lib.MODEL_INPUTS) if mu is not None else None
        s = _f32(sd, _lib.MODEL_INPUTS) if sd is not None else None
        self.eng._check(self.eng.L.swh_model_set(self.eng.h, self.h, th.ctypes.data if th is not None else None,
                                                 m.ctypes.data if m is not None else None,
                                                 s.ctypes.data if s is not None else None))

    def train(self, pool, rows, cols, scoring, scores=None, epochs: int = 4, batch: int = 4096, lr: float = 1e-3,
              seed: int = 0, return_labels: bool = False):
        """Train on labelled pairs (pool sequences, row/column indices); labels from the engine when scores is None."""
        sc = Scoring.of(scoring)
        cat, off = _concat(pool)
        r = np.ascontiguousarray(rows, dtype=np.int32)
        c = np.ascontiguousarray(cols, dtype=np.int32)
        n = len(r)
        sco = np.ascontiguousarray(scores, dtype=np.int32) if scores is not None else None
        lab = np.zeros(n, np.int32) if return_labels else None
        cfg = _lib.swh_train_cfg(ctypes.sizeof(_lib.swh_train_cfg), 0, int(epochs), int(batch), float(lr), int(seed))
        st = _lib.swh_train_stats(ctypes.sizeof(_lib.swh_train_stats))
        rc = self.eng.L.swh_prefilter_train(self.eng.h, self.h, ctypes.byref(sc.c), len(off) - 1,
                                            cat.ctypes.data if len(cat) else None, off.ctypes.data, n,
                                            r.ctypes.data, c.ctypes.data,
                                            sco.ctypes.data if sco is not None else None, ctypes.byref(cfg),
                                            lab.ctypes.data if lab is not None else None, ctypes.byref(st))
        self.eng._check(rc)
        stats = {k: getattr(st, k) for k, _ in st._fields_[2:]}
        return (stats, lab) if return_labels else stats

    def grad(self, z, y):
        z = _f32(z)
        y = _f32(y)
        B = len(y)
        g = np.zeros(_lib.MODEL_PARAMS, np.float32)
        loss = ctypes.c_double()
        self.eng._check(self.eng.L.swh_mlp_grad(self.eng.h, self.h, B, z.ctypes.data, y.ctypes.data,
                                                ctypes.byref(loss), g.ctypes.data))
        return loss.value, g

    def train_steps(self, z, y, steps: int, lr: float = 1e-3):
        z = _f32(z)
        y = _f32(y)
        self.eng._check(self.eng.L.swh_mlp_train_steps(self.eng.h, self.h, len(y), z.ctypes.data, y.ctypes.data,
                                                       int(steps), float(lr)))

    def predict(self, db: "Database", queries):
        cat, off = _concat(queries)
        nq = len(off) - 1
        out = np.zeros((nq, db.ndb), np.float32)
        self.eng._check(self.eng.L.swh_prefilter_predict(self.eng.h, self.h, db.h, nq,
                                                         cat.ctypes.data if len(cat) else None, off.ctypes.data,
                                                         out.ctypes.data))
        return out

    def search(self, db: "Database", queries, k: int = 10, rescore_frac: float = 0.05, audit_frac: float = 0.002,
               audit_seed: int = 0x5EED):
        """Top-k through the prefilter: (indices [nq, k], exact scores [nq, k], stats dict)."""
        cat, off = _concat(queries)
        nq = len(off) - 1
        hits = (_lib.swh_hit * max(1, nq * k))()
        st = _lib.swh_prefilter_stats(ctypes.sizeof(_lib.swh_prefilter_stats))
        rc = self.eng.L.swh_prefilter_search(self.eng.h, self.h, db.h, nq, cat.ctypes.data if len(cat) else None,
                                             off.ctypes.data, k, float(rescore_frac), float(audit_frac),
                                             int(audit_seed), hits, ctypes.byref(st))
        self.eng._check(rc)
        idx = np.array([hits[i].db_index for i in range(nq * k)], dtype=np.int64).reshape(nq, k)
        sco = np.array([hits[i].score for i in range(nq * k)], dtype=np.int32).reshape(nq, k)
        return idx, sco, {k2: getattr(st, k2) for k2, _ in st._fields_[2:]}


def dipeptide_counts(engine: Engine, seqs, scoring) -> np.ndarray:
    sc = Scoring.of(scoring)
    cat, off = _concat(seqs)
    n = len(off) - 1
    out = np.zeros((n, 400), np.int32)
    engine._check(engine.L.swh_dipeptide_counts(engine.h, ctypes.byref(sc.c), n, cat.ctypes.data if len(cat) else None,
                                                off.ctypes.data, out.ctypes.data))
    return out


def dna_scoring(match: int = 1, mismatch: int = -3, gap_open: int = 5, gap_extend: int = 2) -> Scoring:
    mat = np.full((4, 4), mismatch, dtype=np.int8)
    np.fill_diagonal(mat, match)
    return Scoring("ACGT", mat, gap_open, gap_extend)
