"""The C-ABI contract on the GPU: argument checks (NULL pointers, gap
penalties, k, mode, lifecycle), the exception barrier (an injected host
allocation failure becomes SWH_E_NOMEM and the context stays usable), the
context memory cap, cancellation from a second host thread, the device-input
variants of the batch and database calls, and empty queries in the database
search and the prefilter (score 0 against everything, as the oracle says)."""
import ctypes
import threading
import time

import numpy as np
import pytest

import oracle
import seqgen

pytestmark = pytest.mark.gpu

E_INVAL, E_NOMEM, E_RANGE, E_CANCELLED = -1, -3, -4, -7


@pytest.fixture(scope="module")
def swh():
    import paper_2211_10769_amd as m
    return m


@pytest.fixture(scope="module")
def eng(swh):
    return swh.Engine(0)


def _raw_align(swh, eng, q, t, sc, mode=2, cap=None):
    L = eng.L
    out = swh._lib.swh_alignment()
    cap = 2 * (len(q) + len(t)) + 16 if cap is None else cap
    buf = ctypes.create_string_buffer(max(cap, 1))
    clen = ctypes.c_int64()
    rc = L.swh_align(eng.h, q, len(q), t, len(t), ctypes.byref(sc.c), mode, ctypes.byref(out), buf, cap,
                     ctypes.byref(clen), None)
    return rc, out, buf.value.decode(), clen.value


def test_argument_checks(swh, eng):
    L = eng.L
    sc = swh.Scoring(*seqgen.dna_scoring())
    out = swh._lib.swh_alignment()
    # NULL sequences with a positive length, NULL out, bad mode
    assert L.swh_align(eng.h, None, 5, b"ACGTA", 5, ctypes.byref(sc.c), 0, ctypes.byref(out), None, 0, None,
                       None) == E_INVAL
    assert L.swh_align(eng.h, b"ACGTA", 5, b"ACGTA", 5, ctypes.byref(sc.c), 0, None, None, 0, None, None) == E_INVAL
    assert L.swh_align(eng.h, b"ACGTA", 5, b"ACGTA", 5, ctypes.byref(sc.c), 7, ctypes.byref(out), None, 0, None,
                       None) == E_INVAL
    assert L.swh_align(eng.h, b"ACGTA", 5, b"ACGTA", 5, None, 0, ctypes.byref(out), None, 0, None, None) == E_INVAL
    # gap penalties: e > o, e = 0, o = 0
    for o, e in ((2, 5), (5, 0), (0, 0)):
        bad = swh.Scoring("ACGT", np.eye(4, dtype=np.int8), o, e)
        assert L.swh_align(eng.h, b"ACGT", 4, b"ACGT", 4, ctypes.byref(bad.c), 0, ctypes.byref(out), None, 0, None,
                           None) == E_INVAL
        assert b"gap" in L.swh_last_error(eng.h)
    # alphabet too large, repeated symbol
    big = swh.Scoring("A" * 33, np.zeros((33, 33), np.int8), 5, 2)
    assert L.swh_align(eng.h, b"A", 1, b"A", 1, ctypes.byref(big.c), 0, ctypes.byref(out), None, 0, None,
                       None) == E_INVAL
    rep = swh.Scoring("AA", np.zeros((2, 2), np.int8), 5, 2)
    assert L.swh_align(eng.h, b"A", 1, b"A", 1, ctypes.byref(rep.c), 0, ctypes.byref(out), None, 0, None,
                       None) == E_INVAL
    # CIGAR buffer too small: SWH_E_RANGE with the required length
    rc, _, _, need = _raw_align(swh, eng, b"ACGTACGTAC", b"ACGTACGTAC", sc, cap=2)
    assert rc == E_RANGE and need == 3   # "10M"
    # the context is still fine
    rc, o2, cg, _ = _raw_align(swh, eng, b"ACGTACGTAC", b"ACGTACGTAC", sc)
    assert rc == 0 and o2.score == 10 and cg == "10M"


def test_database_argument_checks(swh, eng):
    L = eng.L
    sc = swh.Scoring(*seqgen.protein_scoring())
    db = swh.Database(eng, [b"ACDEFGHIK", b"LMNPQ"], sc)
    hits = (swh._lib.swh_hit * 64)()
    q = b"ACDEF"
    off = np.array([0, 5], np.int64)
    for k in (0, 33, -1):
        assert L.swh_db_search(eng.h, db.h, 1, q, off.ctypes.data, k, hits, None) == E_INVAL
    assert L.swh_db_search(eng.h, None, 1, q, off.ctypes.data, 10, hits, None) == E_INVAL
    assert L.swh_db_search(eng.h, db.h, 1, q, off.ctypes.data, 10, None, None) == E_INVAL
    assert L.swh_db_search(eng.h, db.h, -1, q, off.ctypes.data, 10, hits, None) == E_INVAL
    bad = np.array([5, 0], np.int64)   # decreasing offsets
    assert L.swh_db_search(eng.h, db.h, 1, q, bad.ctypes.data, 10, hits, None) == E_INVAL
    # k larger than the database: missing slots (-1, -1)
    idx, sco, _ = db.search([q], k=4)
    assert idx[0, 2:].tolist() == [-1, -1] and sco[0, 2:].tolist() == [-1, -1]
    db.close()
    # lifecycle: a second context on the same device is independent
    e2 = swh.Engine(0)
    r = e2.align(b"ACGT", b"ACGT", swh.dna_scoring(), mode="cigar")
    assert r["score"] == 4
    e2.close()
    e2.close()   # idempotent in the binding


def test_options_round_trip_and_range(swh, eng):
    for name, good, bad in (("rows_per_lane", 16, 12), ("grid", 512, -1), ("band_rows", -1, -2),
                            ("tb_leaf", 64, 600000), ("graph", 2, 3), ("prune", 0, 5), ("mem_cap", 1 << 30, -1),
                            ("int16", 2, 3), ("inter_max", 1024, 16), ("pf_rank", 0, 3), ("db_waves", 16, 3),
                            ("db_route", 50, -2)):
        old = eng.get_option(name)
        eng.set_option(name, good)
        assert eng.get_option(name) == good
        with pytest.raises(swh.SwhError) as ei:
            eng.set_option(name, bad)
        assert ei.value.status == E_INVAL
        assert eng.get_option(name) == good
        eng.set_option(name, old)
    assert eng.L.swh_set_option(eng.h, 999, 0) == E_INVAL


def test_exception_barrier_maps_bad_alloc(swh, eng):
    sc = swh.dna_scoring()
    eng.set_option("fault_nomem", 1)
    with pytest.raises(swh.SwhError) as ei:
        eng.align(b"ACGTACGT", b"ACGTACGT", sc, mode="cigar")
    assert ei.value.status == E_NOMEM and "bad_alloc" in str(ei.value)
    assert eng.get_option("fault_nomem") == 0
    # the same for the batch and the database calls, then everything works again
    eng.set_option("fault_nomem", 1)
    with pytest.raises(swh.SwhError) as ei:
        eng.align_batch([b"ACGT"], [b"ACGT"], sc, mode="cigar")
    assert ei.value.status == E_NOMEM
    r = eng.align(b"ACGTACGT", b"TTACGTACGTTT", sc, mode="cigar")
    assert (r["score"], r["t_begin"], r["cigar"]) == (8, 2, "8M")


def test_memory_cap(swh):
    eng = swh.Engine(0)
    sc = swh.dna_scoring()
    rng = np.random.default_rng(5)
    a = seqgen.random_dna(rng, 200_000)
    b = seqgen.mutate(rng, a, 0.02, 0.005)
    free = eng.align(bytes(a), bytes(b), sc, mode="cigar", stats=True)
    free_bands = free.pop("stats")["traceback_bands"]
    eng.close()
    eng = swh.Engine(0)
    eng.set_option("mem_cap", 1 << 20)
    with pytest.raises(swh.SwhError) as ei:
        eng.align(bytes(a), bytes(b), sc, mode="cigar")
    assert ei.value.status == E_NOMEM and "memory cap" in str(ei.value)
    # a cap the passes fit in, but not the rows the band traceback would keep:
    # the kept rows shrink, the result does not change
    eng.set_option("mem_cap", 320 << 20)
    capped = eng.align(bytes(a), bytes(b), sc, mode="cigar", stats=True)
    assert {k: capped[k] for k in free} == free
    assert 0 < capped["stats"]["traceback_bands"] < free_bands, (capped["stats"], free_bands)
    eng.set_option("mem_cap", 0)
    assert eng.align(bytes(a), bytes(b), sc, mode="cigar") == free
    eng.close()


def _run_in_thread(fn):
    res = {}

    def target():
        t0 = time.perf_counter()
        try:
            res["value"] = fn()
        except Exception as x:   # noqa: BLE001 -- reported to the test below
            res["error"] = x
        res["seconds"] = time.perf_counter() - t0

    th = threading.Thread(target=target)
    th.start()
    return th, res


def test_cancel_long_pass_from_another_thread(swh):
    eng = swh.Engine(0)
    sc = swh.dna_scoring()
    rng = np.random.default_rng(9)
    a = bytes(seqgen.random_dna(rng, 4_000_000))
    b = bytes(seqgen.random_dna(rng, 4_000_000))
    eng.align(a[:100_000], b[:100_000], sc, mode="score")   # warm
    t0 = time.perf_counter()
    eng.align(a[:2_000_000], b[:2_000_000], sc, mode="score")
    quarter = time.perf_counter() - t0                          # a quarter of the full pass's cells
    th, res = _run_in_thread(lambda: eng.align(a, b, sc, mode="score"))
    time.sleep(0.3)
    assert th.is_alive()
    assert eng.cancel() == 0
    th.join(timeout=120)
    assert not th.is_alive()
    assert isinstance(res.get("error"), swh.SwhError) and res["error"].status == E_CANCELLED, res
    assert res["seconds"] < 3 * quarter, (res["seconds"], quarter)
    # the context is usable afterwards and the result is exact
    x = seqgen.random_dna(rng, 3000)
    y = np.concatenate([seqgen.random_dna(rng, 200), seqgen.mutate(rng, x, 0.03, 0.01)])
    got = eng.align(bytes(x), bytes(y), sc, mode="cigar")
    want = oracle.sw_align(bytes(x), bytes(y), seqgen.dna_scoring())
    assert {k: got[k] for k in want} == want
    eng.close()


def test_cancel_batch_from_another_thread(swh):
    eng = swh.Engine(0)
    sc = swh.dna_scoring()
    rng = np.random.default_rng(10)
    qs = [bytes(seqgen.random_dna(rng, 400_000)) for _ in range(8)]
    ts = [bytes(seqgen.random_dna(rng, 400_000)) for _ in range(8)]
    th, res = _run_in_thread(lambda: eng.align_batch(qs, ts, sc, mode="score"))
    time.sleep(0.15)
    eng.cancel()
    th.join(timeout=120)
    assert not th.is_alive()
    if "error" in res:
        assert res["error"].status == E_CANCELLED, res
    # the context is usable afterwards and the results are exact
    small_q = [q[:3000] for q in qs[:3]]
    small_t = [t[:2500] for t in ts[:3]]
    got = eng.align_batch(small_q, small_t, sc, mode="cigar")
    for i in range(3):
        want = oracle.sw_align(small_q[i], small_t[i], seqgen.dna_scoring())
        assert {k: got[i][k] for k in want} == want


def test_batch_dev_equals_host(swh, eng):
    import torch
    sc = swh.dna_scoring()
    rng = np.random.default_rng(11)
    pairs = [seqgen.read_pair(rng, int(L)) for L in rng.integers(150, 3000, size=60)]
    qs = [bytes(p[0]) for p in pairs]
    ts = [bytes(p[1]) for p in pairs]
    qs[5] = b""
    host = eng.align_batch(qs, ts, sc, mode="cigar")
    qcat, qoff = swh._concat(qs)
    tcat, toff = swh._concat(ts)
    qd = torch.from_numpy(qcat.copy()).cuda()
    td = torch.from_numpy(tcat.copy()).cuda()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        dev = eng.align_batch_dev(qd, qoff, td, toff, sc, mode="cigar", stream=s.cuda_stream)
    assert dev == host
    for i in (0, 7, 33):
        want = oracle.sw_align(qs[i], ts[i], seqgen.dna_scoring())
        assert {k: host[i][k] for k in want} == want


def test_db_search_dev_equals_host(swh, eng):
    import torch
    rng = np.random.default_rng(12)
    sc = swh.Scoring(*seqgen.protein_scoring())
    db = [bytes(seqgen.random_protein(rng, int(L))) for L in seqgen.db_lengths(rng, 800)]
    D = swh.Database(eng, db, sc)
    qs = [bytes(seqgen.random_protein(rng, L)) for L in (50, 300, 900)]
    hi, hs, _ = D.search(qs, k=10)
    qcat, qoff = swh._concat(qs)
    qd = torch.from_numpy(qcat.copy()).cuda()
    di, ds, _ = D.search_dev(qd, qoff, k=10)
    assert np.array_equal(hi, di) and np.array_equal(hs, ds)
    want = oracle.db_scores(qs, db, seqgen.protein_scoring())
    oi, osc = oracle.topk(want, 10)
    assert np.array_equal(hi, oi) and np.array_equal(hs, osc)
    D.close()


def test_empty_query_scores_zero(swh, eng):
    # a search with ordinary queries first (buffers hold their scores), then a
    # batch with an empty query: the empty query scores 0 against everything,
    # and its top-k is the first k database indices with score 0
    rng = np.random.default_rng(13)
    sc = swh.Scoring(*seqgen.protein_scoring())
    db = [bytes(seqgen.random_protein(rng, int(L))) for L in seqgen.db_lengths(rng, 300)]
    D = swh.Database(eng, db, sc)
    q1 = [bytes(seqgen.random_protein(rng, 200)), bytes(seqgen.random_protein(rng, 90))]
    D.search(q1, k=10)
    D.scores(q1)
    qs = [q1[0], b"", q1[1]]
    got, _ = D.scores(qs)
    want = oracle.db_scores(qs, db, seqgen.protein_scoring())
    assert np.array_equal(got, want)
    assert not want[1].any()
    hi, hs, _ = D.search(qs, k=10)
    oi, osc = oracle.topk(want, 10)
    assert np.array_equal(hi, oi) and np.array_equal(hs, osc)
    # the prefilter path gives the same answer for the empty query
    model = swh.Model(eng, sc, seed=3)
    pi, ps, _ = model.search(D, qs, k=10, rescore_frac=0.2, audit_frac=0.0)
    assert pi[1].tolist() == list(range(10)) and ps[1].tolist() == [0] * 10
    D.close()
