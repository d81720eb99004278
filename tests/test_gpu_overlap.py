"""GPU parity of the overlap variant (end gaps of both sequences free)
against the oracle's overlap DP (pinned by enumeration of every
boundary-to-boundary rectangle in test_oracle_pins): score, coordinates and
CIGAR byte for byte."""
import re

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


def _cmp(eng, a, b, sc):
    got = eng.align(a, b, sc, mode="cigar", alignment="overlap")
    want = oracle.ov_align(a, b, sc)
    assert {k: got[k] for k in KEYS} == want, (len(a), len(b))
    for mode in ("score", "coords"):
        g = eng.align(a, b, sc, mode=mode, alignment="overlap")
        assert (g["score"], g["q_end"], g["t_end"]) == (want["score"], want["q_end"], want["t_end"]), mode
        if mode == "coords":
            assert (g["q_begin"], g["t_begin"]) == (want["q_begin"], want["t_begin"])
    return got


def test_small_and_empty(eng):
    sc = seqgen.dna_scoring()
    for a, b in [(b"", b""), (b"", b"ACGT"), (b"ACG", b""), (b"A", b"A"), (b"A", b"C"), (b"ACGT", b"ACGT"),
                 (b"AAAA", b"CCCC"), (b"TTTACGT", b"ACGTGGG"), (b"ACGTGGG", b"TTTACGT"), (b"GGACGTACC", b"ACGTA"),
                 (b"ACGTA", b"GGACGTACC"), (b"C", b"ACGTC"), (b"ACGTC", b"C")]:
        _cmp(eng, a, b, sc)


def _dovetail(rng, n, m, k, sub=0.05, indel=0.02):
    """query = x + core, target = mutated core + y: a suffix-prefix overlap of about k."""
    core = seqgen.random_dna(rng, k)
    a = np.concatenate([seqgen.random_dna(rng, n - k), core])
    b = np.concatenate([seqgen.mutate(rng, core, sub, indel), seqgen.random_dna(rng, m - k)])
    return bytes(a), bytes(b)


@pytest.mark.parametrize("n,m,k", [(300, 300, 120), (1000, 3400, 700), (2500, 900, 600), (64 * 16 + 1, 2000, 1025),
                                   (3000, 3000, 3000)])
def test_random_and_dovetail(eng, n, m, k):
    rng = np.random.default_rng(n * 31 + m + k)
    sc = seqgen.dna_scoring()
    _cmp(eng, bytes(seqgen.random_dna(rng, n)), bytes(seqgen.random_dna(rng, m)), sc)
    a, b = _dovetail(rng, n, m, k)
    got = _cmp(eng, a, b, sc)
    assert got["score"] > 0
    _cmp(eng, b, a, sc)   # the overlap at the other ends (start on the left column)


def test_containment(eng):
    rng = np.random.default_rng(8)
    sc = seqgen.dna_scoring()
    a = seqgen.random_dna(rng, 1500)
    b = np.concatenate([seqgen.random_dna(rng, 400), seqgen.mutate(rng, a, 0.04, 0.01), seqgen.random_dna(rng, 300)])
    _cmp(eng, bytes(a), bytes(b), sc)
    _cmp(eng, bytes(b), bytes(a), sc)


def test_tie_heavy_asymmetric_and_protein(eng, opt):
    opt("tb_leaf", 16)
    tie = ("AC", np.array([[1, -1], [-1, 1]], dtype=np.int8), 1, 1)
    rng = np.random.default_rng(6)
    for n, m in ((50, 61), (333, 900), (200, 150), (700, 700)):
        a = bytes(rng.choice(np.frombuffer(b"AC", np.uint8), n))
        b = bytes(rng.choice(np.frombuffer(b"AC", np.uint8), m))
        _cmp(eng, a, b, tie)
    # an asymmetric matrix: the swapped passes must read it transposed
    asym = ("ACG", np.array([[3, -4, 1], [-1, 2, -5], [-3, 0, 4]], dtype=np.int8), 4, 1)
    for n, m in ((40, 55), (600, 800), (1300, 500)):
        a = bytes(rng.choice(np.frombuffer(b"ACG", np.uint8), n))
        b = bytes(rng.choice(np.frombuffer(b"ACG", np.uint8), m))
        _cmp(eng, a, b, asym)
        _cmp(eng, b, a, asym)
    opt("tb_leaf", 0)
    sc = seqgen.protein_scoring()
    q = seqgen.random_protein(rng, 600)
    h = seqgen.homolog(rng, q)
    _cmp(eng, bytes(np.concatenate([seqgen.random_protein(rng, 300), q[:400]])),
         bytes(np.concatenate([h[100:], seqgen.random_protein(rng, 200)])), sc)


def test_large_dovetail_rescores(eng):
    # beyond the oracle's quadratic passes: 300 kbp reads overlapping by
    # 100 kbp; the CIGAR rescores to the optimum and the oracle agrees on a
    # window around the overlap
    sc = seqgen.dna_scoring()
    alphabet, mat, o, e = sc
    rng = np.random.default_rng(23)
    a, b = _dovetail(rng, 300_000, 300_000, 100_000, 0.02, 0.005)
    got = eng.align(a, b, sc, mode="cigar", alignment="overlap")
    assert got["q_end"] == len(a) - 1 and abs(got["q_begin"] - 200_000) < 200 and got["t_begin"] == 0
    lut = {ord(c): k for k, c in enumerate(alphabet)}
    A = np.array([lut[x] for x in a[got["q_begin"]:got["q_end"] + 1]])
    B = np.array([lut[x] for x in b[got["t_begin"]:got["t_end"] + 1]])
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
    assert (i, j) == (len(A), len(B)) and total == got["score"]
    # the start of the overlap on shortened reads the oracle finishes quickly
    a2, b2 = a[197_000:203_000], b[:3000]
    want = oracle.ov_align(a2, b2, sc)
    part = eng.align(a2, b2, sc, mode="cigar", alignment="overlap")
    assert {k: part[k] for k in KEYS} == want


def test_batch_matches_oracle(eng):
    sc = seqgen.dna_scoring()
    rng = np.random.default_rng(99)
    qs, ts = [b"", b"ACGT", b"", b"AAAA", b"C"], [b"GG", b"", b"", b"CCCC", b"ACGTC"]
    for _ in range(30):
        n, m = (int(x) for x in rng.integers(100, 3000, size=2))
        k = int(rng.integers(50, min(n, m)))
        a, b = _dovetail(rng, n, m, k)
        if rng.random() < 0.5:
            a, b = b, a
        qs.append(a)
        ts.append(b)
    core = seqgen.random_dna(rng, 800)
    qs.append(bytes(core))
    ts.append(bytes(np.concatenate([seqgen.random_dna(rng, 300), seqgen.mutate(rng, core, 0.03, 0.01),
                                    seqgen.random_dna(rng, 200)])))
    want = [oracle.ov_align(a, b, sc) for a, b in zip(qs, ts)]
    got = eng.align_batch(qs, ts, sc, mode="cigar", alignment="overlap")
    assert [{k: g[k] for k in KEYS} for g in got] == want
    for mode, keys in (("score", ["score", "q_end", "t_end"]),
                       ("coords", ["score", "q_begin", "q_end", "t_begin", "t_end"])):
        got = eng.align_batch(qs, ts, sc, mode=mode, alignment="overlap")
        assert [{k: g[k] for k in keys} for g in got] == [{k: w[k] for k in keys} for w in want], mode
    # an asymmetric table through the swapped passes of a batch
    asym = ("ACG", np.array([[3, -4, 1], [-1, 2, -5], [-3, 0, 4]], dtype=np.int8), 4, 1)
    xs = [bytes(rng.choice(np.frombuffer(b"ACG", np.uint8), int(L))) for L in rng.integers(30, 900, size=12)]
    ys = [bytes(rng.choice(np.frombuffer(b"ACG", np.uint8), int(L))) for L in rng.integers(30, 900, size=12)]
    got = eng.align_batch(xs, ys, asym, mode="cigar", alignment="overlap")
    assert [{k: g[k] for k in KEYS} for g in got] == [oracle.ov_align(x, y, asym) for x, y in zip(xs, ys)]


def test_exclusive_flags(eng):
    import paper_2211_10769_amd as swh
    from paper_2211_10769_amd import _lib
    sc = seqgen.dna_scoring()
    saved = dict(swh._ALIGNMENTS)
    try:
        swh._ALIGNMENTS["both"] = _lib.OVERLAP | _lib.GLOBAL
        with pytest.raises(swh.SwhError) as ex:
            eng.align(b"ACGT", b"ACGT", sc, mode="score", alignment="both")
        assert ex.value.status == -1
        with pytest.raises(swh.SwhError) as ex:
            eng.align_batch([b"ACGT"], [b"ACGT"], sc, mode="score", alignment="both")
        assert ex.value.status == -1
    finally:
        swh._ALIGNMENTS.clear()
        swh._ALIGNMENTS.update(saved)
