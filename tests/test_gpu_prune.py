"""Block pruning of the reverse pass (its maximum, the forward score, is
known): results identical to the oracle and to the unpruned pass, on related
pairs where most blocks are pruned, with ties, long gaps and kept rows."""
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


def _both(eng, a, b, sc, opt, mode="cigar"):
    opt("prune", 0)
    plain = eng.align(a, b, sc, mode=mode, stats=True)
    opt("prune", 1)
    pruned = eng.align(a, b, sc, mode=mode, stats=True)
    keys = KEYS if mode == "cigar" else KEYS[:-1]
    assert {k: pruned[k] for k in keys} == {k: plain[k] for k in keys}
    return pruned, plain


@pytest.mark.parametrize("n,sub,indel", [(16_000, 0.02, 0.005), (12_345, 0.10, 0.02), (18_000, 0.01, 0.0)])
def test_related_pairs_match_oracle(eng, opt, n, sub, indel):
    rng = np.random.default_rng(n)
    sc = seqgen.dna_scoring()
    a = seqgen.random_dna(rng, n)
    b = np.concatenate([seqgen.random_dna(rng, 777), seqgen.mutate(rng, a, sub, indel), seqgen.random_dna(rng, 555)])
    got, _ = _both(eng, bytes(a), bytes(b), sc, opt)
    want = oracle.sw_align(bytes(a), bytes(b), sc)
    assert {k: got[k] for k in KEYS} == want


def test_long_gap_and_ties(eng, opt):
    rng = np.random.default_rng(77)
    sc = seqgen.dna_scoring()
    a = seqgen.random_dna(rng, 16_000)
    # a 1 kbp deletion in the middle of an otherwise identical copy
    b = np.concatenate([a[:7000], a[8000:]])
    got, _ = _both(eng, bytes(a), bytes(b), sc, opt)
    assert {k: got[k] for k in KEYS} == oracle.sw_align(bytes(a), bytes(b), sc)
    # two-letter alphabet: many co-optimal starts
    tie = ("AC", np.array([[1, -1], [-1, 1]], dtype=np.int8), 1, 1)
    x = rng.choice(np.frombuffer(b"AC", np.uint8), 9000)
    y = seqgen.mutate(rng, x, 0.0, 0.0)
    y = np.where(rng.random(len(y)) < 0.03, np.uint8(ord("A")) + np.uint8(ord("C")) - y, y).astype(np.uint8)
    got, _ = _both(eng, bytes(x), bytes(y), tie, opt)
    assert {k: got[k] for k in KEYS} == oracle.sw_align(bytes(x), bytes(y), tie)


def test_protein(eng, opt):
    rng = np.random.default_rng(5)
    sc = seqgen.protein_scoring()
    q = seqgen.random_protein(rng, 6000)
    t = np.concatenate([seqgen.random_protein(rng, 900), seqgen.homolog(rng, q), seqgen.random_protein(rng, 400)])
    got, _ = _both(eng, bytes(q), bytes(t), sc, opt)
    assert {k: got[k] for k in KEYS} == oracle.sw_align(bytes(q), bytes(t), sc)


def test_megabase_pair_with_kept_rows(eng, opt):
    # 1 Mbp: kept rows in both passes (band traceback), most reverse blocks pruned
    q, t = seqgen.workload1(1_000_000, flank=10_000)
    q, t = bytes(q), bytes(t)
    sc = seqgen.dna_scoring()
    opt("band_rows", 8192)
    pruned, plain = _both(eng, q, t, sc, opt)
    assert pruned["stats"]["traceback_bands"] > 50 and pruned["stats"]["traceback_retries"] == 0
    # one round of strips: the pass is bound by its diagonal dependency chain
    # either way (the gain comes with several rounds), but never slower
    assert pruned["stats"]["ms_reverse"] < 1.1 * plain["stats"]["ms_reverse"], (pruned["stats"], plain["stats"])


def test_batch_matches_unpruned(eng, opt):
    sc = seqgen.dna_scoring()
    rng = seqgen.rng_for(4, 77)
    qs, ts = [], []
    for L in np.rint(np.exp(rng.uniform(np.log(150), np.log(20_000), size=60))).astype(int):
        a = seqgen.random_dna(rng, int(L))
        div = rng.uniform(0.01, 0.15)
        core = seqgen.mutate(rng, a, div * 0.8, div * 0.2)
        pad = int(0.1 * len(core)) + 1
        qs.append(bytes(a))
        ts.append(bytes(np.concatenate([seqgen.random_dna(rng, pad), core, seqgen.random_dna(rng, pad)])))
    opt("prune", 0)
    plain = eng.align_batch(qs, ts, sc, mode="cigar")
    opt("prune", 1)
    pruned = eng.align_batch(qs, ts, sc, mode="cigar")
    assert [{k: r[k] for k in KEYS} for r in pruned] == [{k: r[k] for k in KEYS} for r in plain]
    for i in (0, 7, 23):
        if len(qs[i]) * len(ts[i]) < 1e8:
            assert {k: pruned[i][k] for k in KEYS} == oracle.sw_align(qs[i], ts[i], sc)
