"""Input generators: determinism and the statistics each workload promises."""
import hashlib

import numpy as np
import pytest

import seqgen


def test_scoring_data_sanity():
    M = seqgen.BLOSUM62
    assert M.shape == (24, 24)
    assert (M == M.T).all()
    assert (np.diag(M)[:20] > 0).all()      # X-X is -1 in the published table
    assert abs(seqgen.BACKGROUND.sum() - 1.0) < 1e-12
    assert len(seqgen.BACKGROUND) == 20
    # a few table entries (Henikoff & Henikoff 1992)
    A = seqgen.PROTEIN_ALPHABET
    assert M[A.index("W"), A.index("W")] == 11
    assert M[A.index("C"), A.index("C")] == 9
    assert M[A.index("I"), A.index("V")] == 3
    assert M[A.index("D"), A.index("E")] == 2


def _karlin_lambda_entropy(S):
    # lambda: the positive root of sum_ij p_i p_j exp(lambda s_ij) = 1;
    # H = sum_ij q_ij lambda s_ij with target frequencies q_ij = p_i p_j exp(lambda s_ij)
    from scipy.optimize import brentq
    pp = np.outer(seqgen.BACKGROUND, seqgen.BACKGROUND)
    S = S.astype(np.float64)
    lam = brentq(lambda x: (pp * np.exp(x * S)).sum() - 1.0, 1e-3, 2.0)
    return lam, (pp * np.exp(lam * S) * lam * S).sum()


@pytest.mark.parametrize("which, lam, ent", [(62, 0.3176, 0.4012), (50, 0.2318, 0.3362), (45, 0.2291, 0.2514)])
def test_blosum_tables_give_published_statistics(which, lam, ent):
    # the ungapped Karlin-Altschul lambda and relative entropy (nats) that BLAST
    # publishes for each matrix under the Robinson & Robinson background; a +-1
    # change of any one symmetric pair of entries moves one of them in the
    # fourth decimal, so the tables are pinned entry by entry
    alph, M, o, e = seqgen.blosum_scoring(which)
    assert M.shape == (20, 20) and alph == seqgen.PROTEIN_ALPHABET[:20] and (o, e) == (10, 2)
    assert (M == M.T).all() and (np.diag(M) > 0).all()
    assert (np.outer(seqgen.BACKGROUND, seqgen.BACKGROUND) * M).sum() < 0   # negative expected score
    got_lam, got_ent = _karlin_lambda_entropy(M)
    assert round(got_lam, 4) == lam and round(got_ent, 4) == ent


def test_statistics_pin_catches_single_entry_errors():
    M = seqgen.BLOSUM50.astype(np.int64)
    base = _karlin_lambda_entropy(M)
    for (i, j) in ((0, 0), (3, 6), (17, 17), (9, 19), (4, 13)):
        T = M.copy()
        T[i, j] += 1
        T[j, i] = T[i, j]
        got = _karlin_lambda_entropy(T)
        assert (round(got[0], 4), round(got[1], 4)) != (round(base[0], 4), round(base[1], 4))


def test_generators_are_deterministic():
    a1, b1 = seqgen.workload0(1000, 900)
    a2, b2 = seqgen.workload0(1000, 900)
    assert hashlib.sha256(a1.tobytes()).hexdigest() == hashlib.sha256(a2.tobytes()).hexdigest()
    assert (b1 == b2).all() and len(a1) == 1000 and len(b1) == 900
    assert set(np.unique(a1).tobytes()) <= set(b"ACGT")


def test_long_pair_mutation_rates():
    q, t = seqgen.workload1(200_000, flank=5_000)
    core_len = len(t) - 10_000
    # 0.5% indel events, half insertions/half deletions, mean length 3: net length change ~0
    assert abs(core_len - len(q)) < 0.003 * len(q)
    # the core starts with the query's first bases unless a mutation hit them
    assert (t[5000:5100] == q[:100]).mean() > 0.9


def test_protein_db_lengths():
    cat, off = seqgen.protein_db(20_000)
    L = np.diff(off)
    assert L.min() >= 25 and L.max() <= 35_000
    assert 280 <= np.median(L) <= 320
    assert 340 <= L.mean() <= 380          # calibrated to Swiss-Prot's mean length (~361)
    freq = np.bincount(np.searchsorted(np.frombuffer(b"ACDEFGHIKLMNPQRSTVWY", np.uint8), cat),
                       minlength=20)
    assert freq.sum() == len(cat)


def test_query_lengths_range():
    qs = seqgen.queries(20)
    L = [len(q) for q in qs]
    assert len(L) == 20 and min(L) >= 100 and max(L) <= 5000


def test_read_pairs_window():
    rng = seqgen.rng_for(4, 9)
    for L in (150, 1000, 5000):
        r, ref = seqgen.read_pair(rng, L)
        assert len(r) == L
        assert abs(len(ref) - round(1.2 * L)) <= 0.2 * L + 10


def test_mutate_identity():
    rng = np.random.default_rng(3)
    q = seqgen.random_protein(rng, 20_000)
    t = seqgen.mutate(rng, q, 0.3, 0.0, protein=True)
    assert len(t) == len(q)
    assert abs((t != q).mean() - 0.3) < 0.02


def test_prefilter_training_set_shape():
    cat, off, rows, cols = seqgen.prefilter_training_set(n_pairs=4000, n_queries=40, homologs=5,
                                                         n_background=300)
    n_pool = 40 + 40 * 5 + 300
    assert len(off) == n_pool + 1 and off[-1] == len(cat)
    assert len(rows) == len(cols) == 4000
    assert rows.min() >= 0 and cols.max() < n_pool
    fam = lambda i: np.where(i < 40, i, np.where(i < 240, (i - 40) // 5, -1))
    related = (fam(rows) == fam(cols)) & (fam(cols) >= 0)
    unrelated = (rows < 40) & (cols >= 240)
    assert related.sum() == 2000 and unrelated.sum() == 2000
    assert np.all(rows != cols)
    again = seqgen.prefilter_training_set(n_pairs=4000, n_queries=40, homologs=5, n_background=300)
    assert np.array_equal(again[0], cat) and np.array_equal(again[2], rows)
