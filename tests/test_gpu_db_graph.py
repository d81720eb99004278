"""The database search replayed as a captured HIP graph: every replay (new
query contents, same lengths) equals the eager search and the oracle's top-k,
with the program's own eager work, buffer reallocations and other searches
between replays; searches the graph cannot serve (an empty query, a 16-bit
saturation) fall back to the eager path with the same results."""
import numpy as np
import pytest

import oracle
import seqgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def swh():
    import paper_2211_10769_amd as m
    return m


@pytest.fixture(scope="module")
def eng(swh):
    e = swh.Engine(0)
    e.set_option("graph", 2)     # database searches replayed as graphs
    return e


@pytest.fixture(scope="module")
def dbase(swh, eng):
    rng = np.random.default_rng(900)
    lens = seqgen.db_lengths(rng, 3000)
    lens[:6] = [2100, 2500, 3300, 4000, 2049, 5000]     # single-pair kernel
    db = [bytes(seqgen.random_protein(rng, int(L))) for L in lens]
    return db, swh.Database(eng, db, seqgen.protein_scoring())


def _queries(rng, lens):
    return [bytes(seqgen.random_protein(rng, int(L))) for L in lens]


def _eager(eng, D, qs, k):
    eng.set_option("graph", 0)
    try:
        return D.search(qs, k=k)
    finally:
        eng.set_option("graph", 2)


def test_replays_equal_eager_and_oracle(swh, eng, dbase):
    db, D = dbase
    rng = np.random.default_rng(901)
    lens = [120, 700, 1500, 40]
    sc = seqgen.protein_scoring()
    for rep in range(4):
        qs = _queries(rng, lens)
        gi, gs, st = D.search(qs, k=10)
        assert st["graph"] == 1, st
        ei, es, est = _eager(eng, D, qs, 10)
        assert est["graph"] == 0
        assert np.array_equal(gi, ei) and np.array_equal(gs, es), rep
        if rep == 1:
            want = oracle.db_scores(qs, db, sc)
            oi, osc = oracle.topk(want, 10)
            assert np.array_equal(gi, oi) and np.array_equal(gs, osc)
        # eager work of other kinds between replays
        eng.align(b"ACGTACGT" * 50, b"ACGTACGA" * 60, swh.dna_scoring(), mode="cigar")
        D.scores(qs[:2])


def test_new_lengths_and_k_recapture(swh, eng, dbase):
    db, D = dbase
    rng = np.random.default_rng(902)
    for lens, k in (([300, 300], 5), ([2000, 10, 333], 32), ([300, 300], 5)):
        qs = _queries(rng, lens)
        gi, gs, st = D.search(qs, k=k)
        ei, es, _ = _eager(eng, D, qs, k)
        assert st["graph"] == 1 and np.array_equal(gi, ei) and np.array_equal(gs, es)


def test_buffer_reallocation_invalidates_the_plan(swh, eng, dbase):
    db, D = dbase
    rng = np.random.default_rng(903)
    qs = _queries(rng, [500, 900])
    a = D.search(qs, k=10)
    # a large alignment grows the context's buffers (new addresses)
    big = seqgen.random_dna(rng, 3_000_000)
    eng.align(bytes(big), bytes(big[:2_000_000]), swh.dna_scoring(), mode="score")
    qs2 = _queries(rng, [500, 900])
    gi, gs, st = D.search(qs2, k=10)
    ei, es, _ = _eager(eng, D, qs2, 10)
    assert st["graph"] == 1 and np.array_equal(gi, ei) and np.array_equal(gs, es)
    assert not np.array_equal(a[0], gi)


def test_empty_query_and_saturation_fall_back(swh, eng, opt):
    opt("db_route", -1)       # the saturating pair stays on the 16-bit inter-task kernel
    rng = np.random.default_rng(904)
    # +60 for identities: a 1,000-residue self-alignment scores 60,000, beyond 16 bits
    alph, _, o, e = seqgen.protein_scoring()
    mat = np.full((len(alph), len(alph)), -10, dtype=np.int8)
    np.fill_diagonal(mat, 60)
    sc = (alph, mat, o, e)
    long_q = seqgen.random_protein(rng, 3000)
    db = [bytes(seqgen.random_protein(rng, int(L))) for L in seqgen.db_lengths(rng, 800)]
    db[5] = bytes(long_q[:1000])
    D = swh.Database(eng, db, sc)
    qs = [bytes(long_q), bytes(seqgen.random_protein(rng, 200))]
    gi, gs, st = D.search(qs, k=10)
    want = oracle.db_scores(qs, db, sc)
    oi, osc = oracle.topk(want, 10)
    assert np.array_equal(gi, oi) and np.array_equal(gs, osc)
    assert st["saturated"] >= 1 and st["graph"] == 0, st
    qs = [bytes(seqgen.random_protein(rng, 150)), b"", bytes(seqgen.random_protein(rng, 90))]
    gi, gs, st = D.search(qs, k=10)
    want = oracle.db_scores(qs, db, sc)
    oi, osc = oracle.topk(want, 10)
    assert np.array_equal(gi, oi) and np.array_equal(gs, osc) and st["graph"] == 0
    D.close()
