"""Pins of the CPU oracle against things other than itself.

* exhaustive enumeration of every alignment on tiny inputs (score, end/start
  rules, canonical CIGAR through enumeration of every path of the H/E/F graph);
* special cases that reduce to textbook routines (maximum-subarray sums on
  diagonals, longest common substring, linear-gap Smith-Waterman);
* closed forms (self-alignment, one-residue query) and invariants;
* hand-derived worked examples in tests/golden/worked_examples.txt.
"""
import os
import random

import numpy as np
import pytest

import oracle
import seqgen
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.txt")


def _mat(alphabet_size, match, mismatch):
    return np.array([[match if i == j else mismatch for j in range(alphabet_size)]
                     for i in range(alphabet_size)], dtype=np.int8)


SCHEMES = [
    ("AC", _mat(2, 1, -1), 1, 1),          # tie-heavy, linear gaps
    ("ACG", _mat(3, 2, -1), 3, 1),
    ("ACGT", _mat(4, 1, -3), 5, 2),        # the paper's DNA scheme
    ("ACGT", _mat(4, 2, -2), 2, 2),        # open == extend
    ("AB", np.array([[3, -2], [0, 1]], dtype=np.int8), 2, 1),   # asymmetric, zero entry
    ("ACG", _mat(3, 1, -1), 100, 1),       # gaps never pay
]


def _rand(rng, alphabet, lo, hi):
    return "".join(rng.choice(alphabet) for _ in range(rng.randint(lo, hi)))


@pytest.mark.parametrize("scheme", range(len(SCHEMES)))
def test_local_matches_enumeration(scheme):
    alphabet, mat, o, e = SCHEMES[scheme]
    sc = (alphabet, mat, o, e)
    rng = random.Random(1000 + scheme)
    for _ in range(30):
        a = _rand(rng, alphabet, 1, 4)
        b = _rand(rng, alphabet, 1, 5)
        want = brute.local_with_cigar(a, b, sc)
        got = oracle.sw_align(a, b, sc)
        assert got == want, (a, b, got, want)


def test_local_matches_enumeration_len6():
    sc = ("AC", _mat(2, 1, -1), 1, 1)
    rng = random.Random(77)
    for _ in range(4):
        a, b = _rand(rng, "AC", 5, 6), _rand(rng, "AC", 5, 6)
        assert oracle.sw_align(a, b, sc) == brute.local_with_cigar(a, b, sc), (a, b)


@pytest.mark.parametrize("scheme", range(len(SCHEMES)))
def test_global_walk_matches_path_enumeration(scheme):
    alphabet, mat, o, e = SCHEMES[scheme]
    sc = (alphabet, mat, o, e)
    rng = random.Random(2000 + scheme)
    for _ in range(25):
        a = _rand(rng, alphabet, 0, 4)
        b = _rand(rng, alphabet, 0, 4)
        if not a and not b:
            continue
        assert oracle.global_cigar(a, b, sc) == brute.global_canonical(a, b, sc), (a, b)


@pytest.mark.parametrize("scheme", range(len(SCHEMES)))
def test_semiglobal_matches_enumeration(scheme):
    alphabet, mat, o, e = SCHEMES[scheme]
    sc = (alphabet, mat, o, e)
    rng = random.Random(3000 + scheme)
    for _ in range(20):
        a = _rand(rng, alphabet, 0, 3)
        b = _rand(rng, alphabet, 0, 5)
        assert oracle.hw_align(a, b, sc) == brute.hw_result(a, b, sc), (a, b)


def test_semiglobal_closed_forms():
    sc = seqgen.dna_scoring()
    # a query that occurs in the target: all matches, placed at its first occurrence's end
    r = oracle.hw_align(b"ACGTA", b"TTACGTAGGACGTA", sc)
    assert (r["score"], r["t_begin"], r["t_end"], r["cigar"]) == (5, 2, 6, "5M")
    # empty target: one gap run; empty query: nothing
    assert oracle.hw_align(b"ACG", b"", sc)["score"] == -(5 + 2 * 2)
    assert oracle.hw_align(b"", b"ACG", sc)["score"] == 0


@pytest.mark.parametrize("scheme", range(len(SCHEMES)))
def test_overlap_matches_enumeration(scheme):
    alphabet, mat, o, e = SCHEMES[scheme]
    sc = (alphabet, mat, o, e)
    rng = random.Random(4000 + scheme)
    for _ in range(20):
        a = _rand(rng, alphabet, 0, 4)
        b = _rand(rng, alphabet, 0, 4)
        assert oracle.ov_align(a, b, sc) == brute.ov_result(a, b, sc), (a, b)


def test_overlap_closed_forms():
    sc = seqgen.dna_scoring()
    # a suffix of the query is a prefix of the target: the overlap alone, all matches
    r = oracle.ov_align(b"TTTACGT", b"ACGTGGG", sc)
    assert (r["score"], r["q_begin"], r["q_end"], r["t_begin"], r["t_end"], r["cigar"]) == (4, 3, 6, 0, 3, "4M")
    # the target inside the query
    r = oracle.ov_align(b"GGACGTACC", b"ACGTA", sc)
    assert (r["score"], r["q_begin"], r["q_end"], r["t_begin"], r["t_end"], r["cigar"]) == (5, 2, 6, 0, 4, "5M")
    # nothing overlaps with a positive score: no alignment
    assert oracle.ov_align(b"AAAA", b"CCCC", sc) == dict(score=0, q_begin=-1, q_end=-1, t_begin=-1, t_end=-1,
                                                          cigar="")
    assert oracle.ov_align(b"", b"ACG", sc)["score"] == 0 and oracle.ov_align(b"ACG", b"", sc)["score"] == 0
    # swapping the sequences under a symmetric matrix keeps the score
    rng = random.Random(11)
    for _ in range(20):
        a, b = _rand(rng, "ACGT", 0, 30), _rand(rng, "ACGT", 0, 30)
        assert oracle.ov_align(a, b, sc)["score"] == oracle.ov_align(b, a, sc)["score"]
        # every overlap is a local alignment, and the overlap's score is bounded by the local optimum
        assert oracle.ov_align(a, b, sc)["score"] <= oracle.sw_align(a, b, sc)["score"]


def test_enumeration_counts_are_delannoy():
    # the op-string enumerator itself: Delannoy numbers D(p,q)
    assert len(brute.op_strings(2, 2)) == 13
    assert len(brute.op_strings(3, 3)) == 63
    assert len(brute.op_strings(4, 2)) == 41


def _load_golden():
    cases = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        f = [x.strip() for x in line.split("|")]
        cases.append(f)
    return cases


@pytest.mark.parametrize("case", _load_golden(), ids=lambda c: c[0])
def test_golden_worked_examples(case):
    name, scheme, q, t, score, coords, cigar = case
    sc = seqgen.dna_scoring() if scheme == "dna" else seqgen.protein_scoring()
    got = oracle.sw_align(q, t, sc)
    qb, qe, tb, te = (int(x) for x in coords.split())
    assert (got["score"], got["q_begin"], got["q_end"], got["t_begin"], got["t_end"]) == \
        (int(score), qb, qe, tb, te)
    assert got["cigar"] == cigar


def test_one_residue_gap_costs_open():
    # gap convention g(k) = o + (k-1) e: single gap costs exactly o
    alphabet, mat, o, e = seqgen.dna_scoring()
    x, y = "ACACACACAC", "TGTGTGTGTG"
    s1 = oracle.sw_align(x + "G" + y, x + y, (alphabet, mat, o, e))["score"]
    assert s1 == 20 - o
    # two inserted residues: a mismatch penalty of -10 keeps the gapped path optimal
    # (the (TG)^5 repeat realigns in phase after a shift of two)
    s2 = oracle.sw_align(x + "GG" + y, x + y, ("ACGT", _mat(4, 1, -10), o, e))["score"]
    assert s2 == 20 - o - e


# ------------------------------------------------------------- special cases

def _kadane_diagonals(A, B, mat):
    best = 0
    n, m = len(A), len(B)
    for d in range(-(n - 1), m):
        cur = 0
        for i in range(n):
            j = i + d
            if 0 <= j < m:
                cur = max(0, cur + int(mat[A[i]][B[j]]))
                best = max(best, cur)
    return best


def test_huge_gaps_reduce_to_max_subarray_on_diagonals():
    rng = np.random.default_rng(5)
    alphabet, mat = seqgen.PROTEIN_ALPHABET, seqgen.BLOSUM62
    for _ in range(6):
        a = seqgen.random_protein(rng, int(rng.integers(20, 120)))
        b = seqgen.random_protein(rng, int(rng.integers(20, 120)))
        S = oracle.sw_align(a, b, (alphabet, mat, 10**6, 10**6), want_cigar=False)["score"]
        A = [alphabet.index(chr(c)) for c in a]
        B = [alphabet.index(chr(c)) for c in b]
        assert S == _kadane_diagonals(A, B, mat)


def _longest_common_substring(a, b):
    best = 0
    prev = [0] * (len(b) + 1)
    for i in range(1, len(a) + 1):
        cur = [0] * (len(b) + 1)
        for j in range(1, len(b) + 1):
            if a[i - 1] == b[j - 1]:
                cur[j] = prev[j - 1] + 1
                best = max(best, cur[j])
        prev = cur
    return best


def test_match_only_scoring_is_longest_common_substring():
    rng = np.random.default_rng(6)
    sc = ("ACGT", _mat(4, 1, -127), 127, 127)
    for _ in range(8):
        a = seqgen.to_str(seqgen.random_dna(rng, int(rng.integers(10, 100))))
        b = seqgen.to_str(seqgen.random_dna(rng, int(rng.integers(10, 100))))
        assert oracle.sw_align(a, b, sc, want_cigar=False)["score"] == _longest_common_substring(a, b)


def _linear_gap_sw(A, B, mat, g):
    """Smith & Waterman (1981) with a linear gap cost g per residue."""
    H = [[0] * (len(B) + 1) for _ in range(len(A) + 1)]
    best = 0
    for i in range(1, len(A) + 1):
        for j in range(1, len(B) + 1):
            H[i][j] = max(0, H[i - 1][j - 1] + int(mat[A[i - 1]][B[j - 1]]),
                          H[i - 1][j] - g, H[i][j - 1] - g)
            best = max(best, H[i][j])
    return best


def test_open_equals_extend_is_linear_gap():
    rng = np.random.default_rng(7)
    mat = _mat(4, 2, -1)
    for g in (1, 2, 3):
        for _ in range(4):
            a = seqgen.random_dna(rng, int(rng.integers(5, 60)))
            b = seqgen.random_dna(rng, int(rng.integers(5, 60)))
            A = ["ACGT".index(chr(c)) for c in a]
            B = ["ACGT".index(chr(c)) for c in b]
            S = oracle.sw_align(a, b, ("ACGT", mat, g, g), want_cigar=False)["score"]
            assert S == _linear_gap_sw(A, B, mat, g)


def _self_condition(mat, codes):
    for x in codes:
        if mat[x][x] <= 0:
            return False
        for y in codes:
            if 2 * int(mat[x][y]) > int(mat[x][x]) + int(mat[y][y]):
                return False
    return True


def test_self_alignment_is_diagonal_sum():
    rng = np.random.default_rng(8)
    alphabet, mat, o, e = seqgen.protein_scoring()
    assert _self_condition(mat, range(20))
    for _ in range(4):
        a = seqgen.random_protein(rng, int(rng.integers(30, 300)))
        A = [alphabet.index(chr(c)) for c in a]
        assert oracle.sw_align(a, a, (alphabet, mat, o, e))["score"] == sum(int(mat[x][x]) for x in A)
    dna = seqgen.dna_scoring()
    assert _self_condition(dna[1], range(4))
    d = seqgen.random_dna(rng, 500)
    r = oracle.sw_align(d, d, dna)
    assert r["score"] == 500 and r["cigar"] == "500M"


def test_single_residue_query():
    rng = np.random.default_rng(9)
    alphabet, mat, o, e = seqgen.protein_scoring()
    for _ in range(10):
        a = seqgen.random_protein(rng, 1)
        b = seqgen.random_protein(rng, int(rng.integers(1, 50)))
        x = alphabet.index(chr(a[0]))
        want = max(0, max(int(mat[x][alphabet.index(chr(c))]) for c in b))
        assert oracle.sw_align(a, b, (alphabet, mat, o, e))["score"] == want


# ---------------------------------------------------------------- invariants

def _rescore(q, t, r, scoring):
    alphabet, mat, o, e = scoring
    A = [alphabet.index(chr(c) if not isinstance(c, str) else c) for c in q[r["q_begin"]:r["q_end"] + 1]]
    B = [alphabet.index(chr(c) if not isinstance(c, str) else c) for c in t[r["t_begin"]:r["t_end"] + 1]]
    ops = []
    num = ""
    for ch in r["cigar"]:
        if ch.isdigit():
            num += ch
        else:
            ops.append(ch * int(num))
            num = ""
    ops = "".join(ops)
    return brute.score_ops(ops, A, B, mat, o, e), ops, A, B


@pytest.mark.parametrize("which", ["dna", "protein"])
def test_invariants(which):
    rng = np.random.default_rng(10)
    sc = seqgen.dna_scoring() if which == "dna" else seqgen.protein_scoring()
    gen = seqgen.random_dna if which == "dna" else seqgen.random_protein
    smax = int(np.max(sc[1][:20, :20])) if which == "protein" else 1
    for _ in range(6):
        a = gen(rng, int(rng.integers(50, 300)))
        b = seqgen.mutate(rng, a, 0.1, 0.02, protein=(which == "protein")) if rng.random() < 0.5 \
            else gen(rng, int(rng.integers(50, 300)))
        a, b = bytes(a), bytes(b)
        r = oracle.sw_align(a, b, sc)
        assert r["score"] >= 0
        assert r["score"] <= min(len(a), len(b)) * smax
        assert oracle.sw_align(b, a, sc, want_cigar=False)["score"] == r["score"]
        assert oracle.sw_align(a + b"A", b, sc, want_cigar=False)["score"] >= r["score"]
        if r["score"] == 0:
            continue
        total, ops, A, B = _rescore(a, b, r, sc)
        assert total == r["score"]
        assert ops.count("M") + ops.count("I") == len(A)
        assert ops.count("M") + ops.count("D") == len(B)
        assert ops[0] == "M" and ops[-1] == "M"
        assert sc[1][A[0]][B[0]] > 0 and sc[1][A[-1]][B[-1]] > 0


def test_topk_is_stable_sort():
    rng = np.random.default_rng(11)
    scores = rng.integers(0, 5, size=(3, 40))
    idx, s = oracle.topk(scores, 7)
    for r in range(3):
        order = sorted(range(40), key=lambda c: (-scores[r, c], c))[:7]
        assert list(idx[r]) == order
        assert list(s[r]) == [scores[r, c] for c in order]
    idx, s = oracle.topk(scores[:, :3], 5)
    assert list(idx[0][3:]) == [-1, -1]


def test_db_scores_agree_with_pairwise():
    rng = np.random.default_rng(12)
    sc = seqgen.protein_scoring()
    qs = [bytes(seqgen.random_protein(rng, int(rng.integers(5, 60)))) for _ in range(3)]
    db = [bytes(seqgen.random_protein(rng, int(rng.integers(1, 80)))) for _ in range(17)]
    S = oracle.db_scores(qs, db, sc, threads=3)
    for i, q in enumerate(qs):
        for j, d in enumerate(db):
            assert S[i, j] == oracle.sw_end(q, d, sc)[0]


def test_bad_symbol_is_rejected():
    with pytest.raises(oracle.OracleError) as ei:
        oracle.sw_align("ACGN", "ACGT", seqgen.dna_scoring())
    assert ei.value.code == oracle.E_ALPHABET
