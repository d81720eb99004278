"""GPU parity of the packed 16-bit local passes: with the option on (the
default) and off, every score, end, start and CIGAR equals the oracle's, at
every 16-bit strip height, for single pairs and batches, with and without
block pruning and kept rows; pairs that reach the 16-bit limit are
recomputed in 32 bits and still equal the oracle."""
import numpy as np
import pytest

import oracle
import seqgen

pytestmark = pytest.mark.gpu

KEYS = ("score", "q_begin", "q_end", "t_begin", "t_end", "cigar")


@pytest.fixture(scope="module")
def swh():
    import paper_2211_10769_amd as m
    return m


@pytest.fixture(scope="module")
def eng(swh):
    return swh.Engine(0)


def _pairs(rng, lens, div=(0.01, 0.15)):
    out = []
    for L in lens:
        a = seqgen.random_dna(rng, int(L))
        d = rng.uniform(*div)
        b = np.concatenate([seqgen.random_dna(rng, int(rng.integers(0, L // 5 + 2))),
                            seqgen.mutate(rng, a, 0.8 * d, 0.2 * d),
                            seqgen.random_dna(rng, int(rng.integers(0, L // 5 + 2)))])
        out.append((bytes(a), bytes(b)))
    return out


def _check_batch(eng, pairs, sc_tuple, mode="cigar"):
    import paper_2211_10769_amd as swh
    sc = swh.Scoring(*sc_tuple)
    got, st = eng.align_batch([p[0] for p in pairs], [p[1] for p in pairs], sc, mode=mode, stats=True)
    for (a, b), g in zip(pairs, got):
        want = oracle.sw_align(a, b, sc_tuple, want_cigar=(mode == "cigar"))
        keys = KEYS if mode == "cigar" else KEYS[:-1]
        assert {k: g[k] for k in keys} == {k: want[k] for k in keys}, (len(a), len(b), g, want)
    return st


@pytest.mark.parametrize("rows", [0, 4, 8, 16, 20])
def test_batch_every_height(eng, opt, rows):
    # nominal heights 4, 8 and 16 rows per lane run the 16-bit kernel (strips of
    # two sub-strips of that height); 20 has no 16-bit form and runs in 32 bits
    rng = np.random.default_rng(300 + rows)
    opt("rows_per_lane", rows)
    lens = [1, 7, 63, 64, 65, 200, 255, 256, 257, 511, 512, 513, 1023, 1024, 1025, 2047, 3000, 5100]
    st = _check_batch(eng, _pairs(rng, lens), seqgen.dna_scoring())
    assert (st["passes_int16"] > 0) == (rows != 20) and st["saturated_int16"] == 0, st


@pytest.mark.parametrize("band_rows", [256, 512, 1024])
def test_batch_kept_rows_at_sub_strips(eng, opt, band_rows):
    # kept rows every 256 rows with 16-bit strips of 512 or 1,024 rows: rows at
    # the end of an upper sub-strip come from the packed kernel's low halves
    rng = np.random.default_rng(305 + band_rows)
    opt("band_rows", band_rows)
    opt("tb_leaf", 4096)
    st = _check_batch(eng, _pairs(rng, [900, 2600, 4100, 7000], div=(0.01, 0.05)), seqgen.dna_scoring())
    assert st["traceback_bands"] > 4 and st["traceback_retries"] == 0, st


def test_batch_int16_equals_int32(eng, opt):
    rng = np.random.default_rng(310)
    pairs = _pairs(rng, rng.integers(150, 6000, size=150))
    import paper_2211_10769_amd as swh
    sc = swh.dna_scoring()
    q, t = [p[0] for p in pairs], [p[1] for p in pairs]
    a, sa = eng.align_batch(q, t, sc, mode="cigar", stats=True)
    opt("int16", 0)
    b, sb = eng.align_batch(q, t, sc, mode="cigar", stats=True)
    assert a == b
    assert sa["passes_int16"] >= 150 and sb["passes_int16"] == 0
    for i in (0, 17, 99):
        want = oracle.sw_align(q[i], t[i], seqgen.dna_scoring())
        assert {k: a[i][k] for k in KEYS} == {k: want[k] for k in KEYS}


def test_batch_protein(eng):
    rng = np.random.default_rng(320)
    pairs = []
    for L in (30, 300, 700, 1500):
        q = seqgen.random_protein(rng, L)
        t = np.concatenate([seqgen.random_protein(rng, 40), seqgen.homolog(rng, q), seqgen.random_protein(rng, 25)])
        pairs.append((bytes(q), bytes(t)))
    st = _check_batch(eng, pairs, seqgen.protein_scoring())
    assert st["passes_int16"] > 0


def test_tie_heavy_batch(eng, opt):
    # binary alphabet, many co-optimal ends and starts
    rng = np.random.default_rng(330)
    sc = ("AC", np.array([[1, -1], [-1, 1]], dtype=np.int8), 1, 1)
    alph = np.frombuffer(b"AC", np.uint8)
    pairs = [(bytes(alph[rng.integers(0, 2, size=int(n))]), bytes(alph[rng.integers(0, 2, size=int(m))]))
             for n, m in rng.integers(5, 900, size=(25, 2))]
    opt("tb_leaf", 64)
    _check_batch(eng, pairs, sc)


def test_saturation_is_redone_in_32_bits(eng):
    # identical pairs score their length: 32,765 stays below the 16-bit limit
    # (32,767 - 1), 32,766 and longer reach it and are recomputed; the 40 kbp
    # pair far exceeds it; every result equals the oracle's
    rng = np.random.default_rng(340)
    base = seqgen.random_dna(rng, 40_000)
    pairs = [(bytes(base[:L]), bytes(base[:L])) for L in (32_765, 32_766, 32_767, 40_000)]
    pairs += _pairs(rng, [300, 2000])
    import paper_2211_10769_amd as swh
    got, st = eng.align_batch([p[0] for p in pairs], [p[1] for p in pairs], swh.dna_scoring(), mode="coords",
                              stats=True)
    for (a, b), g in zip(pairs, got):
        want = oracle.sw_coords_mt(a, b, seqgen.dna_scoring(), band=512, chunk=4096)
        assert {k: g[k] for k in want} == want, (len(a), g, want)
    assert st["saturated_int16"] >= 3, st
    assert [g["score"] for g in got[:4]] == [32_765, 32_766, 32_767, 40_000]


def test_saturation_with_cigar_and_kept_rows(eng, opt):
    # a saturating pair inside a CIGAR batch with forced kept rows: the 32-bit
    # redo rewrites the rows the band traceback reads
    rng = np.random.default_rng(350)
    a = seqgen.random_dna(rng, 36_000)
    b = seqgen.mutate(rng, a, 0.002, 0.0005)
    pairs = [(bytes(a), bytes(b))] + _pairs(rng, [4000, 9000])
    opt("band_rows", 1024)
    import paper_2211_10769_amd as swh
    got, st = eng.align_batch([p[0] for p in pairs], [p[1] for p in pairs], swh.dna_scoring(), mode="cigar",
                              stats=True)
    assert st["saturated_int16"] >= 1 and st["traceback_retries"] == 0, st
    for (x, y), g in zip(pairs, got):
        want = oracle.sw_align(x, y, seqgen.dna_scoring(), max_cells=1_400_000_000)
        assert {k: g[k] for k in KEYS} == {k: want[k] for k in KEYS}


@pytest.mark.parametrize("rows", [0, 4, 8, 16])
def test_single_pair_int16(eng, opt, rows):
    # a 30 kbp related pair can never reach the limit: with the option at 2
    # both passes run in 16 bits (at 1 only passes that fill the GPU do)
    rng = np.random.default_rng(360 + rows)
    a = seqgen.random_dna(rng, 30_000)
    b = np.concatenate([seqgen.random_dna(rng, 700), seqgen.mutate(rng, a, 0.03, 0.005), seqgen.random_dna(rng, 500)])
    opt("rows_per_lane", rows)
    opt("int16", 2)
    import paper_2211_10769_amd as swh
    got = eng.align(bytes(a), bytes(b), swh.dna_scoring(), mode="cigar", stats=True)
    assert got["stats"]["passes_int16"] == 2, got["stats"]
    want = oracle.sw_align(bytes(a), bytes(b), seqgen.dna_scoring(), max_cells=1_000_000_000)
    assert {k: got[k] for k in KEYS} == {k: want[k] for k in KEYS}


def test_single_pair_pruned_and_unpruned(eng, opt):
    rng = np.random.default_rng(370)
    a = seqgen.random_dna(rng, 20_000)
    b = np.concatenate([seqgen.random_dna(rng, 3000), seqgen.mutate(rng, a, 0.05, 0.01), seqgen.random_dna(rng, 100)])
    import paper_2211_10769_amd as swh
    sc = swh.dna_scoring()
    opt("int16", 2)
    pruned = eng.align(bytes(a), bytes(b), sc, mode="coords")
    opt("prune", 0)
    plain = eng.align(bytes(a), bytes(b), sc, mode="coords")
    opt("int16", 0)
    wide = eng.align(bytes(a), bytes(b), sc, mode="coords")
    want = oracle.sw_align(bytes(a), bytes(b), seqgen.dna_scoring(), want_cigar=False)
    for r in (pruned, plain, wide):
        assert {k: r[k] for k in KEYS[:-1]} == {k: want[k] for k in KEYS[:-1]}


def test_long_unrelated_pair_and_no_hit(eng, opt):
    # unrelated 200 kbp sequences: the forward pass could reach the 16-bit limit
    # (min(n, m) is above it) and runs in 32 bits; its score is tiny, so the
    # reverse pass runs in 16 bits
    opt("int16", 2)
    rng = np.random.default_rng(380)
    a = seqgen.random_dna(rng, 200_000)
    b = seqgen.random_dna(rng, 180_000)
    import paper_2211_10769_amd as swh
    got = eng.align(bytes(a), bytes(b), swh.dna_scoring(), mode="coords", stats=True)
    assert got["stats"]["passes_int16"] == 1
    want = oracle.sw_coords_mt(bytes(a), bytes(b), seqgen.dna_scoring())
    assert {k: got[k] for k in want} == want
    r = eng.align(b"AAAA", b"CCCC", swh.dna_scoring(), mode="cigar")
    assert r["score"] == 0 and r["cigar"] == ""
