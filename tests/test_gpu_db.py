"""GPU parity of the exhaustive database search against the CPU oracle:
every score bit-exact, top-k equal to the stable sort of oracle scores."""
import numpy as np
import pytest

import oracle
import seqgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    import paper_2211_10769_amd as swh
    return swh.Engine(0)


def _db(rng, count):
    lens = seqgen.db_lengths(rng, count)
    lens[: max(1, count // 200)] = rng.integers(2100, 3200, size=max(1, count // 200))   # beyond the inter-task limit
    lens[-3:] = [1, 2, 25]
    return [bytes(seqgen.random_protein(rng, int(L))) for L in lens]


def test_scores_and_topk_match_oracle(eng):
    import paper_2211_10769_amd as swh
    rng = np.random.default_rng(42)
    sc = seqgen.protein_scoring()
    db = _db(rng, 1500)
    qs = [bytes(seqgen.random_protein(rng, int(L))) for L in (30, 140, 333, 700)]
    # plant homologs so the top hits are well separated
    for qi, q in enumerate(qs):
        for k in range(3):
            db[100 * qi + 7 * k + 3] = bytes(seqgen.homolog(rng, np.frombuffer(q, np.uint8)))
    D = swh.Database(eng, db, sc)
    got, st = D.scores(qs)
    want = oracle.db_scores(qs, db, sc)
    mism = np.argwhere(got != want)
    assert len(mism) == 0, (mism[:5], got[tuple(mism[0])] if len(mism) else None)
    assert st["intra_pairs"] >= 4 * 7
    idx, sco, st2 = D.search(qs, k=10)
    widx, wsco = oracle.topk(want, 10)
    assert (idx == widx).all() and (sco == wsco).all()


def test_saturation_is_recomputed(eng, opt):
    import paper_2211_10769_amd as swh
    opt("db_route", -1)      # keep every group on the 16-bit inter-task kernel
    # match +100: a 1,000-residue identity scores 100,000 > 65,535 and must be redone in 32 bits
    mat = np.full((4, 4), -50, dtype=np.int8)
    np.fill_diagonal(mat, 100)
    sc = ("ACGT", mat, 120, 60)
    rng = np.random.default_rng(7)
    q = bytes(seqgen.random_dna(rng, 1000))
    db = [bytes(seqgen.random_dna(rng, 300)) for _ in range(200)]
    db[17] = q
    db[150] = q[:700] + bytes(seqgen.random_dna(rng, 50))
    D = swh.Database(eng, db, sc)
    got, st = D.scores([q])
    want = oracle.db_scores([q], db, sc)
    assert (got == want).all()
    assert st["saturated"] >= 2
    assert got[0, 17] == 100_000


def test_edge_cases(eng):
    import paper_2211_10769_amd as swh
    sc = seqgen.protein_scoring()
    rng = np.random.default_rng(9)
    db = [bytes(seqgen.random_protein(rng, 50)) for _ in range(5)]
    D = swh.Database(eng, db, sc)
    q = [bytes(seqgen.random_protein(rng, 60))]
    idx, sco, _ = D.search(q, k=8)          # k > ndb: missing slots are (-1, -1)
    want = oracle.db_scores(q, db, sc)
    widx, wsco = oracle.topk(want, 8)
    assert (idx == widx).all() and (sco[:, :5] == wsco[:, :5]).all() and (sco[:, 5:] == -1).all()
    with pytest.raises(swh.SwhError) as ei:
        swh.Database(eng, [b"ACDX1"], sc)
    assert ei.value.status == -2


def test_length_switch_autotune_and_tuning_file(tmp_path):
    # the measured switch moves sequences between the kernels; scores never change,
    # and a saved tuning file restores the switch in another context
    import paper_2211_10769_amd as swh
    sc = seqgen.protein_scoring()
    rng = np.random.default_rng(77)
    lens = np.concatenate([rng.integers(20, 500, 300), rng.integers(500, 9000, 40)])
    db = [bytes(seqgen.random_protein(rng, int(L))) for L in lens]
    qs = [bytes(seqgen.random_protein(rng, int(L))) for L in (60, 250)]
    want = oracle.db_scores(qs, db, sc)
    a = swh.Engine(0)
    b = swh.Engine(0)
    try:
        for x in (a, b):
            x.set_option("db_route", -1)   # count only the sequences beyond the switch
        v = a.autotune_db(sc)
        assert v in (512, 1024, 2048, 4096, 8192)
        got, st = swh.Database(a, db, sc).scores(qs)
        assert (got == want).all()
        assert st["intra_pairs"] == len(qs) * int((lens > v).sum())
        path = str(tmp_path / "tune.txt")
        a.tune_save(path)
        text = open(path).read()
        assert text.startswith("swh-tune 1\n") and f"inter_max {v}\n" in text
        b.tune_load(path)
        got_b, st_b = swh.Database(b, db, sc).scores(qs)
        assert (got_b == want).all() and st_b["intra_pairs"] == st["intra_pairs"]
        # files of another device, or not tuning files at all, are refused
        lines = text.splitlines()
        other = tmp_path / "other.txt"
        other.write_text("\n".join(["swh-tune 1", "device some other gpu"] + lines[2:]) + "\n")
        bad = tmp_path / "bad.txt"
        bad.write_text("hello\n")
        for p in (other, bad, tmp_path / "missing.txt"):
            with pytest.raises(swh.SwhError) as ex:
                b.tune_load(str(p))
            assert ex.value.status == -1
        # an explicit option still wins over the measured switch
        b.set_option("inter_max", 8192)
        got_c, st_c = swh.Database(b, db, sc).scores(qs)
        assert (got_c == want).all() and st_c["intra_pairs"] == len(qs) * int((lens > 8192).sum())
    finally:
        a.close()
        b.close()


@pytest.mark.parametrize("which", [50, 45])
def test_other_blosum_tables(eng, which):
    import paper_2211_10769_amd as swh
    sc = seqgen.blosum_scoring(which)
    rng = np.random.default_rng(100 + which)
    db = _db(rng, 600)
    qs = [bytes(seqgen.random_protein(rng, int(L))) for L in (45, 300)]
    db[11] = bytes(seqgen.homolog(rng, np.frombuffer(qs[1], np.uint8)))
    D = swh.Database(eng, db, sc)
    got, _ = D.scores(qs)
    want = oracle.db_scores(qs, db, sc)
    assert (got == want).all()
    idx, sco, _ = D.search(qs, k=5)
    widx, wsco = oracle.topk(want, 5)
    assert (idx == widx).all() and (sco == wsco).all()
