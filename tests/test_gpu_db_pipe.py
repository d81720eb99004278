"""The database kernel's launch forms against the oracle: one wave per
(query, group) unit, and the pipelined forms in which 2 to 16 waves share a
unit (its 32-row query chunks on neighbouring waves, bottom rows handed on
through LDS rings and a global ring).  Scores bit-exact, top-k equal, for
queries of 1 to many chunks, chunk-boundary lengths, groups of empty
sequences, 16-bit saturation carried across chunks, and a small grid that
makes each work-group run many units (the unit table wraps).  Also the
routing of oversize units to the single-pair kernel."""
import numpy as np
import pytest

import oracle
import seqgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    import paper_2211_10769_amd as swh
    return swh.Engine(0)


def _mixed_db(rng, count, n_empty):
    lens = seqgen.db_lengths(rng, count)
    lens[:5] = [1, 2, 31, 32, 33]
    db = [bytes(seqgen.random_protein(rng, int(L))) for L in lens]
    return [b""] * n_empty + db


@pytest.mark.parametrize("waves", [1, 2, 4, 8, 12, 16])
def test_forms_match_oracle(eng, opt, waves):
    import paper_2211_10769_amd as swh
    opt("db_waves", waves)
    opt("db_route", -1)                     # every unit on the inter-task kernel
    rng = np.random.default_rng(500 + waves)
    sc = seqgen.protein_scoring()
    db = _mixed_db(rng, 900, 130)          # 130 empty sequences: one group has no columns
    qlens = (1, 31, 32, 33, 64, 97, 400, 1100)
    qs = [bytes(seqgen.random_protein(rng, L)) for L in qlens]
    for qi, q in enumerate(qs[4:]):
        db[200 + 9 * qi] = bytes(seqgen.homolog(rng, np.frombuffer(q, np.uint8)))
    D = swh.Database(eng, db, sc)
    got, st = D.scores(qs)
    want = oracle.db_scores(qs, db, sc)
    mism = np.argwhere(got != want)
    assert len(mism) == 0, (waves, mism[:5])
    idx, sco, _ = D.search(qs, k=10)
    widx, wsco = oracle.topk(want, 10)
    assert (idx == widx).all() and (sco == wsco).all()


@pytest.mark.parametrize("waves", [2, 4, 12, 16])
def test_saturation_carried_across_chunks(eng, opt, waves):
    import paper_2211_10769_amd as swh
    opt("db_waves", waves)
    opt("db_route", -1)                     # every unit on the inter-task kernel
    # +100 per match: the 1,000-residue identity (32 chunks) saturates in its
    # last chunks; the flag rides the running maximum down the pipeline
    mat = np.full((4, 4), -50, dtype=np.int8)
    np.fill_diagonal(mat, 100)
    sc = ("ACGT", mat, 120, 60)
    rng = np.random.default_rng(70 + waves)
    q = bytes(seqgen.random_dna(rng, 1000))
    db = [bytes(seqgen.random_dna(rng, 300)) for _ in range(300)]
    db[17] = q
    db[150] = q[:700] + bytes(seqgen.random_dna(rng, 50))
    db[299] = q[:330]                      # reaches the limit in chunk 10 (row 326)
    D = swh.Database(eng, db, sc)
    got, st = D.scores([q])
    want = oracle.db_scores([q], db, sc)
    assert (got == want).all()
    assert st["saturated"] >= 3
    assert got[0, 17] == 100_000


@pytest.mark.parametrize("waves", [2, 4, 12, 16])
def test_small_grid_runs_many_units_per_work_group(eng, opt, waves):
    import paper_2211_10769_amd as swh
    opt("db_waves", waves)
    opt("db_route", -1)                     # every unit on the inter-task kernel
    opt("grid", 3)                          # 3 work-groups for some 90 units
    rng = np.random.default_rng(900 + waves)
    sc = seqgen.protein_scoring()
    db = _mixed_db(rng, 1400, 0)
    qs = [bytes(seqgen.random_protein(rng, int(L))) for L in rng.integers(1, 300, 8)]
    D = swh.Database(eng, db, sc)
    got, _ = D.scores(qs)
    want = oracle.db_scores(qs, db, sc)
    assert (got == want).all()
    idx, sco, st = D.search(qs, k=5)
    widx, wsco = oracle.topk(want, 5)
    assert (idx == widx).all() and (sco == wsco).all()


@pytest.mark.parametrize("route", [0, 30, 400])
def test_oversize_units_routed_to_single_pair_kernel(eng, opt, route):
    import paper_2211_10769_amd as swh
    opt("db_route", route)
    rng = np.random.default_rng(31 + route)
    sc = seqgen.protein_scoring()
    db = _mixed_db(rng, 2000, 3)            # the first group holds empty sequences: never moved
    qs = [bytes(seqgen.random_protein(rng, L)) for L in (40, 700)]
    D = swh.Database(eng, db, sc)
    got, st = D.scores(qs)
    want = oracle.db_scores(qs, db, sc)
    assert (got == want).all()
    # the rule, recomputed from the layout: groups of 128 by ascending length
    lens = np.array(sorted(len(x) for x in db if len(x) <= 2048))
    groups = [lens[i:i + 128] for i in range(0, len(lens), 128)]
    colsum = sum(128 * int(g.max()) for g in groups)
    import torch
    num_cu = torch.cuda.get_device_properties(0).multi_processor_count
    share = sum(len(q) for q in qs) * colsum / num_cu
    limit = share * (100 if route == 0 else route) / 100
    moved = sum(len(g) for q in qs for g in groups if g[0] > 0 and len(q) * 128 * int(g.max()) > limit)
    n_long = sum(len(x) > 2048 for x in db)
    assert st["intra_pairs"] == moved + len(qs) * n_long
    assert moved > 0
    idx, sco, _ = D.search(qs, k=7)
    widx, wsco = oracle.topk(want, 7)
    assert (idx == widx).all() and (sco == wsco).all()


def test_high_scores_on_the_single_pair_kernel(eng):
    import paper_2211_10769_amd as swh
    # sequences beyond the length switch go to the single-pair kernel (32-bit):
    # with +100 per match the query's copy inside one of them scores 100,000
    mat = np.full((4, 4), -50, dtype=np.int8)
    np.fill_diagonal(mat, 100)
    sc = ("ACGT", mat, 120, 60)
    rng = np.random.default_rng(4242)
    q = bytes(seqgen.random_dna(rng, 1000))
    db = [bytes(seqgen.random_dna(rng, int(L))) for L in rng.integers(50, 400, 500)]
    db += [bytes(seqgen.random_dna(rng, int(L))) for L in (2100, 2600, 3000)]
    db[-2] = bytes(seqgen.random_dna(rng, 800)) + q + bytes(seqgen.random_dna(rng, 900))
    D = swh.Database(eng, db, sc)
    got, st = D.scores([q])
    want = oracle.db_scores([q], db, sc)
    assert (got == want).all()
    assert got[0, len(db) - 2] == 100_000
    assert st["intra_pairs"] >= 3
