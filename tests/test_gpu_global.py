"""GPU parity of the global (Needleman-Wunsch) variant against the oracle's
global DP and greedy walk (pinned by path enumeration in test_oracle_pins):
scores and CIGARs byte for byte, single pairs and batches."""
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


def _want(a, b, sc):
    g, cg = oracle.global_cigar(a, b, sc)
    return dict(score=g, q_begin=0 if a else -1, q_end=len(a) - 1, t_begin=0 if b else -1, t_end=len(b) - 1,
                cigar=cg)


KEYS = ["score", "q_begin", "q_end", "t_begin", "t_end", "cigar"]


def _cmp(eng, a, b, sc):
    got = eng.align(a, b, sc, mode="cigar", alignment="global")
    want = _want(a, b, sc)
    assert {k: got[k] for k in KEYS} == want, (len(a), len(b))
    return got


def test_small_and_empty(eng):
    sc = seqgen.dna_scoring()
    for a, b in [(b"", b""), (b"", b"ACGT"), (b"ACG", b""), (b"A", b"A"), (b"A", b"C"), (b"ACGT", b"ACGT"),
                 (b"AAAA", b"CCCC"), (b"ACGTTTACGT", b"ACGT"), (b"ACGT", b"TTTTACGTTTTT")]:
        _cmp(eng, a, b, sc)


@pytest.mark.parametrize("n,m", [(300, 300), (1000, 1400), (2500, 900), (64 * 16 + 1, 70)])
def test_random_and_related(eng, n, m):
    rng = np.random.default_rng(n * 7 + m)
    sc = seqgen.dna_scoring()
    _cmp(eng, bytes(seqgen.random_dna(rng, n)), bytes(seqgen.random_dna(rng, m)), sc)
    a = seqgen.random_dna(rng, n)
    b = np.concatenate([seqgen.random_dna(rng, 40), seqgen.mutate(rng, a, 0.05, 0.02), seqgen.random_dna(rng, 25)])
    _cmp(eng, bytes(a), bytes(b), sc)


def test_tie_heavy_and_protein(eng, opt):
    opt("tb_leaf", 16)
    tie = ("AC", np.array([[1, -1], [-1, 1]], dtype=np.int8), 1, 1)
    rng = np.random.default_rng(3)
    for n in (50, 333):
        a = bytes(rng.choice(np.frombuffer(b"AC", np.uint8), n))
        b = bytes(rng.choice(np.frombuffer(b"AC", np.uint8), n + 11))
        _cmp(eng, a, b, tie)
    opt("tb_leaf", 0)
    sc = seqgen.protein_scoring()
    q = seqgen.random_protein(rng, 800)
    _cmp(eng, bytes(q), bytes(seqgen.homolog(rng, q)), sc)


def test_batch_and_modes(eng):
    sc = seqgen.dna_scoring()
    rng = seqgen.rng_for(4, 31)
    qs, ts = [b"", b"ACGT", b""], [b"GG", b"", b""]
    for L in rng.integers(1, 2500, size=40):
        a = seqgen.random_dna(rng, int(L))
        qs.append(bytes(a))
        ts.append(bytes(seqgen.mutate(rng, a, 0.08, 0.03)))
    want = [_want(a, b, sc) for a, b in zip(qs, ts)]
    got = eng.align_batch(qs, ts, sc, mode="cigar", alignment="global")
    assert [{k: g[k] for k in KEYS} for g in got] == want
    for mode in ("score", "coords"):
        got = eng.align_batch(qs, ts, sc, mode=mode, alignment="global")
        assert [(g["score"], g["q_end"], g["t_end"]) for g in got] == [(w["score"], w["q_end"], w["t_end"])
                                                                       for w in want]


def test_large_pair_rescores(eng):
    # beyond the oracle's full matrix: the CIGAR consumes both sequences and
    # rescores to the reported optimum
    sc = seqgen.dna_scoring()
    alphabet, mat, o, e = sc
    rng = np.random.default_rng(9)
    a = seqgen.random_dna(rng, 200_000)
    b = seqgen.mutate(rng, a, 0.03, 0.01)
    got = eng.align(bytes(a), bytes(b), sc, mode="cigar", alignment="global")
    lut = {ord(c): k for k, c in enumerate(alphabet)}
    A = np.array([lut[x] for x in bytes(a)])
    B = np.array([lut[x] for x in bytes(b)])
    i = j = total = 0
    for n, op in re.findall(r"(\d+)([MID])", got["cigar"]):
        n = int(n)
        if op == "M":
            total += int(np.asarray(mat)[A[i:i + n], B[j:j + n]].astype(np.int64).sum())
            i += n
            j += n
        else:
            total -= o + (n - 1) * e
            i, j = (i + n, j) if op == "I" else (i, j + n)
    assert (i, j) == (len(a), len(b)) and total == got["score"]


def test_range_limit(eng):
    import paper_2211_10769_amd as swh
    sc = ("ACGT", seqgen.dna_scoring()[1], 60000, 60000)
    with pytest.raises(swh.SwhError) as ex:
        eng.align(b"A" * 2000, b"C" * 2000, sc, mode="score", alignment="global")
    assert ex.value.status == -4


@pytest.mark.parametrize("band_rows", [512, 1024, 2560])
def test_banded_traceback_matches_oracle(eng, opt, band_rows):
    # kept rows of a forward and a corner-anchored reverse global pass cut the
    # traceback into bands; the CIGAR must not change
    opt("band_rows", band_rows)
    rng = np.random.default_rng(band_rows)
    sc = seqgen.dna_scoring()
    a = seqgen.random_dna(rng, 6000)
    cases = [(a, seqgen.mutate(rng, a, 0.05, 0.02)),
             # long unaligned query ends: the path runs down column 0 and column m
             (np.concatenate([seqgen.random_dna(rng, 1500), a[:3000], seqgen.random_dna(rng, 1200)]),
              seqgen.mutate(rng, a[:3000], 0.03, 0.01)),
             # long unaligned target ends: rows 0 and n carry long D runs
             (a[:4000], np.concatenate([seqgen.random_dna(rng, 900), seqgen.mutate(rng, a[:4000], 0.03, 0.01),
                                        seqgen.random_dna(rng, 700)]))]
    for x, y in cases:
        got = eng.align(bytes(x), bytes(y), sc, mode="cigar", alignment="global", stats=True)
        assert {k: got[k] for k in KEYS} == _want(bytes(x), bytes(y), sc), (len(x), len(y))
        assert got["stats"]["traceback_retries"] == 0
    tie = ("AC", np.array([[1, -1], [-1, 1]], dtype=np.int8), 1, 1)
    x = bytes(rng.choice(np.frombuffer(b"AC", np.uint8), 3000))
    y = bytes(rng.choice(np.frombuffer(b"AC", np.uint8), 3100))
    _cmp(eng, x, y, tie)


def test_banded_equals_plain_at_300kbp(eng, opt):
    rng = np.random.default_rng(21)
    sc = seqgen.dna_scoring()
    a = seqgen.random_dna(rng, 300_000)
    b = seqgen.mutate(rng, a, 0.03, 0.01)
    opt("band_rows", -1)
    plain = eng.align(bytes(a), bytes(b), sc, mode="cigar", alignment="global", stats=True)
    opt("band_rows", 0)
    banded = eng.align(bytes(a), bytes(b), sc, mode="cigar", alignment="global", stats=True)
    assert banded["stats"]["traceback_bands"] > 10 and banded["stats"]["traceback_retries"] == 0
    assert {k: banded[k] for k in KEYS} == {k: plain[k] for k in KEYS}
