"""Parity at the benchmark's own sizes, in the launch configurations bench.py
times: the database search of 20 queries against 500,000 proteins and the
batch of 200,000 read/reference pairs.  The oracle cannot score everything at
these sizes, so it checks sampled outputs one by one (every top-10 hit and
random query/database pairs; random pairs of the batch, CIGARs included), and
pairs of the batch are checked by properties that hold at any size.  At 20
queries x 20,000 proteins every score is compared with the oracle's, stored by
tests/golden/make_db_20k.py."""
import os
import re

import numpy as np
import pytest

import oracle
import seqgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    import paper_2211_10769_amd as swh
    return swh.Engine(0)


def test_database_search_full_size_sampled(eng):
    import paper_2211_10769_amd as swh
    qs, (cat, off) = seqgen.workload2()
    sc = seqgen.protein_scoring()
    D = swh.Database(eng, (cat, off), sc)
    qb = [bytes(q) for q in qs]
    idx, sco, _ = D.search(qb, k=10)
    allsc, _ = D.scores(qb)
    D.close()
    ndb = len(off) - 1
    # the top-10 lists agree with the full score matrix (score desc, index asc)
    for q in range(len(qb)):
        order = np.lexsort((np.arange(ndb), -allsc[q].astype(np.int64)))[:10]
        assert (idx[q] == order).all() and (sco[q] == allsc[q][order]).all(), q
    # sampled pairs and every top hit, each recomputed by the oracle
    rng = np.random.default_rng(2024)
    for q in range(len(qb)):
        pick = np.unique(np.concatenate([idx[q], rng.integers(0, ndb, size=8)]))
        subs = [bytes(cat[off[i]:off[i + 1]]) for i in pick]
        want = oracle.db_scores([qb[q]], subs, sc)[0]
        assert (allsc[q][pick] == want).all(), (q, pick[allsc[q][pick] != want])


def _rescore(q, t, r, scoring):
    alphabet, mat, o, e = scoring
    lut = np.full(256, -1, dtype=np.int64)
    for k, ch in enumerate(alphabet):
        lut[ord(ch)] = k
    A = lut[np.frombuffer(q, np.uint8)][r["q_begin"]:r["q_end"] + 1]
    B = lut[np.frombuffer(t, np.uint8)][r["t_begin"]:r["t_end"] + 1]
    i = j = total = 0
    for n, op in re.findall(r"(\d+)([MID])", r["cigar"]):
        n = int(n)
        if op == "M":
            total += int(np.asarray(mat)[A[i:i + n], B[j:j + n]].astype(np.int64).sum())
            i += n
            j += n
        else:
            total -= o + (n - 1) * e
            i, j = (i + n, j) if op == "I" else (i, j + n)
    return total, (i, j) == (len(A), len(B))


def test_batch_of_read_pairs_bench_config(eng):
    # all 200,000 pairs of the bench's batched leg in one call (its chunking,
    # 16-bit passes and kept-row groups as timed)
    pairs = seqgen.workload4(n_pairs=200_000)
    qs = [bytes(p[0]) for p in pairs]
    ts = [bytes(p[1]) for p in pairs]
    del pairs
    sc = seqgen.dna_scoring()
    got = eng.align_batch(qs, ts, sc, mode="cigar")
    assert len(got) == len(qs) and all(r["score"] > 0 for r in got)
    # properties on 20,000 pairs drawn at random: the CIGAR spans the reported
    # rectangle, starts and ends with a match run, and rescores to the optimum
    rng = np.random.default_rng(11)
    for i in rng.choice(len(qs), size=20_000, replace=False):
        r = got[i]
        assert r["cigar"][-1] == "M" and re.match(r"^\d+M", r["cigar"]), i
        total, spans = _rescore(qs[i], ts[i], r, sc)
        assert spans and total == r["score"], i
    # the oracle on a sample small enough for its quadratic traceback
    rng = np.random.default_rng(7)
    small = [i for i in range(len(qs)) if len(qs[i]) * len(ts[i]) < 6e7]
    for i in rng.choice(small, size=40, replace=False):
        want = oracle.sw_align(qs[i], ts[i], sc)
        assert {k: got[i][k] for k in want} == want, i


@pytest.mark.parametrize("waves", [0, 1, 8, 12])
def test_database_20_queries_20k_proteins_equal_the_oracle(eng, opt, waves):
    # every score of the 20 database queries against 20,000 proteins equals the
    # oracle's (stored by tests/golden/make_db_20k.py, 2.3e11 cells), and the
    # top-10 lists are its stable sort; the launch rule's form and forced ones
    import paper_2211_10769_amd as swh
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "db_20k_scores.npz"))
    qs, (cat, off) = seqgen.workload2(n_db=20_000, n_queries=20)
    assert [len(q) for q in qs] == list(g["query_lengths"]) and int(off[-1] - off[0]) == int(g["db_residues"])
    opt("db_waves", waves)
    sc = seqgen.protein_scoring()
    D = swh.Database(eng, (cat, off), sc)
    qb = [bytes(q) for q in qs]
    got, _ = D.scores(qb)
    idx, sco, _ = D.search(qb, k=10)
    D.close()
    want = g["scores"].astype(np.int64)
    mism = np.argwhere(got != want)
    assert len(mism) == 0, (mism[:5], [(int(got[tuple(m)]), int(want[tuple(m)])) for m in mism[:5]])
    widx, wsco = oracle.topk(want, 10)
    assert (idx == widx).all() and (sco == wsco).all()
