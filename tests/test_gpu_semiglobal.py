"""GPU parity of the semi-global variant (whole query, free target ends)
against the oracle's semi-global DP (pinned by enumeration of every target
substring in test_oracle_pins): score, coordinates and CIGAR byte for byte."""
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
    got = eng.align(a, b, sc, mode="cigar", alignment="semiglobal")
    want = oracle.hw_align(a, b, sc)
    assert {k: got[k] for k in KEYS} == want, (len(a), len(b))
    for mode in ("score", "coords"):
        g = eng.align(a, b, sc, mode=mode, alignment="semiglobal")
        assert g["score"] == want["score"] and g["t_end"] == want["t_end"], mode
        if mode == "coords":
            assert g["t_begin"] == want["t_begin"]
    return got


def test_small_and_empty(eng):
    sc = seqgen.dna_scoring()
    for a, b in [(b"", b""), (b"", b"ACGT"), (b"ACG", b""), (b"A", b"A"), (b"A", b"C"), (b"ACGT", b"ACGT"),
                 (b"AAAA", b"CCCC"), (b"ACGT", b"TTTTACGTTTTT"), (b"ACGTTTACGT", b"ACGT"),
                 (b"GATTACA", b"CCGATTACACCGATTACA")]:
        _cmp(eng, a, b, sc)


@pytest.mark.parametrize("n,m", [(300, 300), (1000, 3400), (2500, 900), (64 * 16 + 1, 7000)])
def test_random_and_embedded(eng, n, m):
    rng = np.random.default_rng(n * 13 + m)
    sc = seqgen.dna_scoring()
    _cmp(eng, bytes(seqgen.random_dna(rng, n)), bytes(seqgen.random_dna(rng, m)), sc)
    # a mutated copy of the query inside a longer random target
    a = seqgen.random_dna(rng, n)
    flank = max(1, (m - n) // 2)
    b = np.concatenate([seqgen.random_dna(rng, flank), seqgen.mutate(rng, a, 0.05, 0.02),
                        seqgen.random_dna(rng, flank + 3)])
    got = _cmp(eng, bytes(a), bytes(b), sc)
    assert got["t_begin"] >= 0


def test_tie_heavy_and_protein(eng, opt):
    opt("tb_leaf", 16)
    tie = ("AC", np.array([[1, -1], [-1, 1]], dtype=np.int8), 1, 1)
    rng = np.random.default_rng(5)
    for n, m in ((50, 61), (333, 900), (200, 150)):
        a = bytes(rng.choice(np.frombuffer(b"AC", np.uint8), n))
        b = bytes(rng.choice(np.frombuffer(b"AC", np.uint8), m))
        _cmp(eng, a, b, tie)
    opt("tb_leaf", 0)
    sc = seqgen.protein_scoring()
    q = seqgen.random_protein(rng, 600)
    t = np.concatenate([seqgen.random_protein(rng, 300), seqgen.homolog(rng, q), seqgen.random_protein(rng, 200)])
    _cmp(eng, bytes(q), bytes(t), sc)


def test_no_target_residue_pays(eng):
    # a query that scores worse against any target residue than as one gap
    sc = ("AC", np.array([[1, -30], [-30, 1]], dtype=np.int8), 2, 1)
    got = _cmp(eng, b"AAAA", b"CCCCCC", sc)
    assert got["cigar"] == "4I" and got["t_begin"] == -1


def test_large_read_rescores(eng):
    # beyond the oracle's quadratic passes: a 20 kbp read inside a 2 Mbp
    # target; the CIGAR consumes the whole query and rescores to the optimum
    sc = seqgen.dna_scoring()
    alphabet, mat, o, e = sc
    rng = np.random.default_rng(17)
    ref = seqgen.random_dna(rng, 2_000_000)
    pos = 1_234_567
    a = seqgen.mutate(rng, ref[pos:pos + 20_000], 0.03, 0.01)
    got = eng.align(bytes(a), bytes(ref), sc, mode="cigar", alignment="semiglobal")
    assert abs(got["t_begin"] - pos) < 200
    lut = {ord(c): k for k, c in enumerate(alphabet)}
    A = np.array([lut[x] for x in bytes(a)])
    B = np.array([lut[x] for x in bytes(ref[got["t_begin"]:got["t_end"] + 1])])
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
    # the oracle over a window holding the read: the same alignment
    w0 = pos - 3000
    want = oracle.hw_align(bytes(a[:6000]), bytes(ref[w0:pos + 9000]), sc)
    part = eng.align(bytes(a[:6000]), bytes(ref), sc, mode="cigar", alignment="semiglobal")
    want.update(t_begin=want["t_begin"] + w0, t_end=want["t_end"] + w0)
    assert {k: part[k] for k in KEYS} == want


def test_batch_matches_oracle(eng):
    # reads against reference windows (workload-4 shape), plus empty sides and
    # reads that align to no target residue
    sc = seqgen.dna_scoring()
    rng = seqgen.rng_for(4, 55)
    qs, ts = [b"", b"ACGT", b"", b"AAAA"], [b"GG", b"", b"", b"CCCCCC"]
    for L in np.rint(np.exp(rng.uniform(np.log(150), np.log(4000), size=40))).astype(int):
        a = seqgen.random_dna(rng, int(L))
        div = rng.uniform(0.01, 0.15)
        pad = int(0.1 * L) + 1
        qs.append(bytes(a))
        ts.append(bytes(np.concatenate([seqgen.random_dna(rng, pad), seqgen.mutate(rng, a, 0.8 * div, 0.2 * div),
                                        seqgen.random_dna(rng, pad)])))
    qs.append(bytes(seqgen.random_dna(rng, 300)))
    ts.append(bytes(seqgen.random_dna(rng, 5000)))
    hard = ("AC", np.array([[1, -30], [-30, 1]], dtype=np.int8), 2, 1)
    want = [oracle.hw_align(a, b, sc) for a, b in zip(qs, ts)]
    got = eng.align_batch(qs, ts, sc, mode="cigar", alignment="semiglobal")
    assert [{k: g[k] for k in KEYS} for g in got] == want
    for mode, keys in (("score", ["score", "t_end"]), ("coords", ["score", "q_begin", "q_end", "t_begin", "t_end"])):
        got = eng.align_batch(qs, ts, sc, mode=mode, alignment="semiglobal")
        assert [{k: g[k] for k in keys} for g in got] == [{k: w[k] for k in keys} for w in want], mode
    got = eng.align_batch([b"AAAA", b"ACAC"], [b"CCCCCC", b"CACA"], hard, mode="cigar", alignment="semiglobal")
    assert [{k: g[k] for k in KEYS} for g in got] == [oracle.hw_align(b"AAAA", b"CCCCCC", hard),
                                                     oracle.hw_align(b"ACAC", b"CACA", hard)]
