"""GPU parity of batched pairwise alignment (many pairs per call) and of the
strip-shape autotuner: every pair's score, coordinates and CIGAR equal the
oracle's, whatever the batch composition or the strip shapes."""
import ctypes
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import seqgen

pytestmark = pytest.mark.gpu

KEYS = ["score", "q_begin", "q_end", "t_begin", "t_end", "cigar"]


@pytest.fixture(scope="module")
def eng():
    import paper_2211_10769_amd as swh
    return swh.Engine(0)


def _oracle_all(qs, ts, sc, cigar=True):
    with ThreadPoolExecutor(8) as ex:
        return list(ex.map(lambda p: oracle.sw_align(bytes(p[0]), bytes(p[1]), sc, want_cigar=cigar), zip(qs, ts)))


def _check(got, want, mode="cigar"):
    keys = {"score": KEYS[:1], "coords": KEYS[:5], "cigar": KEYS}[mode]
    bad = []
    for i, (g, w) in enumerate(zip(got, want)):
        if any(g[k] != w[k] for k in keys):
            bad.append((i, {k: (g[k], w[k]) for k in keys if g[k] != w[k]}))
    assert not bad, bad[:3]


def _read_pairs(n, hi, seed_stream=7):
    # the batched-reads generator (log-uniform lengths, 1-15% divergence, 1.2x windows) at a reduced size
    rng = seqgen.rng_for(4, seed_stream)
    lens = np.rint(np.exp(rng.uniform(np.log(150), np.log(hi), size=n))).astype(np.int64)
    pairs = [seqgen.read_pair(rng, int(L)) for L in lens]
    return [p[0] for p in pairs], [p[1] for p in pairs]


def test_read_pairs_cigar(eng):
    qs, ts = _read_pairs(160, 3000)
    sc = seqgen.dna_scoring()
    got, st = eng.align_batch(qs, ts, sc, mode="cigar", stats=True)
    _check(got, _oracle_all(qs, ts, sc))
    assert st["cells_forward"] == pytest.approx(sum(len(q) * len(t) for q, t in zip(qs, ts)))


def test_modes_agree(eng):
    qs, ts = _read_pairs(40, 1500, seed_stream=8)
    sc = seqgen.dna_scoring()
    want = _oracle_all(qs, ts, sc)
    _check(eng.align_batch(qs, ts, sc, mode="score"), want, "score")
    _check(eng.align_batch(qs, ts, sc, mode="coords"), want, "coords")


def test_mixed_edge_cases(eng):
    sc = seqgen.dna_scoring()
    rng = np.random.default_rng(5)
    a = seqgen.random_dna(rng, 900)
    qs = [b"", b"ACGT", b"A", b"AAAA", bytes(a), b"ACGT" * 40, bytes(seqgen.random_dna(rng, 64 * 4 + 1)), b"G"]
    ts = [b"ACGT", b"", b"A", b"CCCC", bytes(seqgen.mutate(rng, a, 0.05, 0.01)), b"TTTT" + b"ACGT" * 40,
          bytes(seqgen.random_dna(rng, 300)), b"C"]
    got = eng.align_batch(qs, ts, sc, mode="cigar")
    _check(got, _oracle_all(qs, ts, sc))
    assert got[0]["score"] == 0 and got[0]["q_begin"] == -1 and got[0]["cigar"] == ""
    assert got[3]["score"] == 0


def test_protein_pairs(eng):
    sc = seqgen.protein_scoring()
    rng = seqgen.rng_for(3, 40)
    qs, ts = [], []
    for L in (30, 120, 400, 700, 1500):
        q = seqgen.random_protein(rng, L)
        qs.append(q)
        ts.append(seqgen.homolog(rng, q))
        qs.append(seqgen.random_protein(rng, L // 2 + 5))
        ts.append(seqgen.random_protein(rng, L))
    _check(eng.align_batch(qs, ts, sc, mode="cigar"), _oracle_all(qs, ts, sc))


def test_tie_heavy_batch(eng, opt):
    # deep recursion inside every pair of the batch (tiny leaves), binary alphabet, o = e = 1
    opt("tb_leaf", 16)
    tie = ("AC", np.array([[1, -1], [-1, 1]], dtype=np.int8), 1, 1)
    rng = np.random.default_rng(11)
    qs = [bytes(rng.choice(np.frombuffer(b"AC", np.uint8), n)) for n in (20, 70, 150, 333)]
    ts = [bytes(rng.choice(np.frombuffer(b"AC", np.uint8), n + 17)) for n in (20, 70, 150, 333)]
    _check(eng.align_batch(qs, ts, tie, mode="cigar"), _oracle_all(qs, ts, tie))


def test_small_cigar_buffer_reports_size(eng):
    import paper_2211_10769_amd as swh
    from paper_2211_10769_amd import _lib
    qs, ts = _read_pairs(6, 800, seed_stream=9)
    sc = swh.Scoring(*seqgen.dna_scoring())
    qcat, qoff = swh._concat(qs)
    tcat, toff = swh._concat(ts)
    out = (_lib.swh_alignment * 6)()
    coff = np.zeros(7, dtype=np.int64)
    buf = ctypes.create_string_buffer(4)
    rc = eng.L.swh_align_batch(eng.h, 6, qcat.ctypes.data, qoff.ctypes.data, tcat.ctypes.data, toff.ctypes.data,
                               ctypes.byref(sc.c), _lib.MODE_CIGAR, out, buf, 4, coff.ctypes.data, None)
    assert rc == -4
    want = _oracle_all(qs, ts, seqgen.dna_scoring())
    assert coff[-1] == sum(len(w["cigar"]) for w in want)
    assert [out[i].score for i in range(6)] == [w["score"] for w in want]


def test_bad_symbol_names_pair(eng):
    import paper_2211_10769_amd as swh
    with pytest.raises(swh.SwhError) as ex:
        eng.align_batch([b"ACGT", b"ACGT", b"ACNT"], [b"ACGT", b"ACGT", b"ACGT"], seqgen.dna_scoring())
    assert ex.value.status == -2 and "pair 2" in str(ex.value) and "position 2" in str(ex.value)


def test_tuned_shapes_keep_results(eng):
    import paper_2211_10769_amd as swh
    sc = seqgen.dna_scoring()
    qs, ts = _read_pairs(30, 5000, seed_stream=10)
    base = eng.align_batch(qs, ts, sc, mode="cigar")
    try:
        table = eng.autotune(sc, max_rows=8192, cells_per_trial=2e9)
        assert table and table[-1]["max_rows"] == 2 ** 63 - 1
        assert all(t["rows_per_lane"] in (4, 8, 16, 20, 24, 32) and 1 <= t["waves_per_simd"] <= 8 for t in table)
        _check(eng.align_batch(qs, ts, sc, mode="cigar"), base)
        for R, w in ((8, 1), (16, 2), (20, 2), (24, 3), (32, 4)):
            eng.set_tune_table([{"max_rows": 2 ** 40, "rows_per_lane": R, "waves_per_simd": w}])
            _check(eng.align_batch(qs, ts, sc, mode="cigar"), base)
        with pytest.raises(swh.SwhError):
            eng.set_tune_table([{"max_rows": 10, "rows_per_lane": 5, "waves_per_simd": 1}])
        with pytest.raises(swh.SwhError):
            eng.set_tune_table([{"max_rows": 10, "rows_per_lane": 4, "waves_per_simd": 1},
                                {"max_rows": 10, "rows_per_lane": 8, "waves_per_simd": 1}])
    finally:
        eng.set_tune_table([])
    assert eng.tune_table() == []


@pytest.mark.parametrize("rows", [256, 1024])
def test_band_traceback_in_batches(eng, opt, rows):
    # kept rows every few strips in both passes of every pair; CIGARs unchanged
    opt("band_rows", rows)
    qs, ts = _read_pairs(120, 6000, seed_stream=12)
    sc = seqgen.dna_scoring()
    got, st = eng.align_batch(qs, ts, sc, mode="cigar", stats=True)
    _check(got, _oracle_all(qs, ts, sc))
    assert st["traceback_retries"] == 0
    assert st["traceback_bands"] > len(qs)
    opt("band_rows", -1)
    got2, st2 = eng.align_batch(qs, ts, sc, mode="cigar", stats=True)
    assert st2["traceback_bands"] == 0 and st2["cells_traceback"] > 2 * st["cells_traceback"]
    _check(got2, got)


def test_band_traceback_tie_heavy_batch(eng, opt):
    opt("band_rows", 256)
    opt("rows_per_lane", 4)
    tie = ("AC", np.array([[1, -1], [-1, 1]], dtype=np.int8), 1, 1)
    rng = np.random.default_rng(13)
    qs, ts = [], []
    for n in (300, 900, 1500, 2500):
        a = rng.choice(np.frombuffer(b"AC", np.uint8), n)
        flip = rng.random(n) < 0.1
        qs.append(bytes(a))
        ts.append(bytes(np.where(flip, np.where(a == ord("A"), ord("C"), ord("A")), a).astype(np.uint8)))
    got, st = eng.align_batch(qs, ts, tie, mode="cigar", stats=True)
    _check(got, _oracle_all(qs, ts, tie))
    assert st["traceback_retries"] == 0


@pytest.mark.parametrize("int16", [1, 0])
def test_many_multi_strip_pairs_spread_ticket_order(eng, opt, int16):
    # 1,200 pairs: at least as many problems as SIMDs, so each pair's strips are
    # spread over the ticket order (reads up to 2,500 bp: up to five 512-row
    # strips in 32 bits, three 1,024-row strips in 16); every pair equals the oracle
    opt("int16", int16)
    qs, ts = _read_pairs(1200, 2500, seed_stream=11)
    sc = seqgen.dna_scoring()
    assert sum(len(q) > 1024 for q in qs) > 300
    want = _oracle_all(qs, ts, sc, cigar=True)
    got, st = eng.align_batch(qs, ts, sc, mode="cigar", stats=True)
    _check(got, want)
    _check(eng.align_batch(qs, ts, sc, mode="coords"), want, "coords")
    assert (st["passes_int16"] > 0) == bool(int16)
