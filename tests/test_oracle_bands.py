"""The banded threaded form of the oracle's local pass (score, end, start of
one long pair), pinned against the plain single-threaded pass: both walk the
same recurrences, so every band height, chunk width and thread count must give
the same score and the same end and start cells -- including ragged last
bands and chunks, bands taller than the query, chunks wider than the target,
and tie-heavy inputs where the first-cell rule decides the end."""
import json
import os

import numpy as np
import pytest

import oracle
import seqgen

HERE = os.path.dirname(os.path.abspath(__file__))

SHAPES = [(1, 1, 3), (2, 3, 2), (7, 13, 4), (64, 100, 8), (1000, 1000, 2), (3, 5000, 5), (17, 1, 1)]


def _check(a, b, sc):
    want = oracle.sw_align(bytes(a), bytes(b), sc, want_cigar=False)
    for band, chunk, th in SHAPES:
        got = oracle.sw_coords_mt(bytes(a), bytes(b), sc, threads=th, band=band, chunk=chunk)
        for k in got:
            assert got[k] == want[k], (band, chunk, th, k, got, want)
        assert oracle.sw_end_mt(bytes(a), bytes(b), sc, threads=th, band=band, chunk=chunk) == \
            (want["score"], want["q_end"], want["t_end"])


@pytest.mark.parametrize("seed", range(12))
def test_random_and_related_dna(seed):
    rng = np.random.default_rng(seed)
    sc = seqgen.dna_scoring()
    n = int(rng.integers(1, 600))
    a = seqgen.random_dna(rng, n)
    if seed % 2:
        b = np.concatenate([seqgen.random_dna(rng, int(rng.integers(0, 60))), seqgen.mutate(rng, a, 0.05, 0.01),
                            seqgen.random_dna(rng, int(rng.integers(0, 60)))])
    else:
        b = seqgen.random_dna(rng, int(rng.integers(1, 700)))
    _check(a, b, sc)


@pytest.mark.parametrize("seed", range(6))
def test_tie_heavy(seed):
    # binary alphabet, +1/-1, o = e = 1: many co-optimal end cells
    rng = np.random.default_rng(50 + seed)
    alph = "AC"
    mat = np.array([[1, -1], [-1, 1]], dtype=np.int8)
    sc = (alph, mat, 1, 1)
    a = np.frombuffer(b"AC", np.uint8)[rng.integers(0, 2, size=int(rng.integers(1, 300)))]
    b = np.frombuffer(b"AC", np.uint8)[rng.integers(0, 2, size=int(rng.integers(1, 300)))]
    _check(a, b, sc)


def test_repeats_and_homopolymers():
    sc = seqgen.dna_scoring()
    _check(b"A" * 257, b"A" * 300, sc)
    _check(b"ACGT" * 70, b"ACGT" * 65 + b"TTTT" + b"ACGT" * 9, sc)
    _check(b"CCCC", b"GGGG", sc)          # score 0: no alignment


def test_protein():
    rng = np.random.default_rng(7)
    sc = seqgen.protein_scoring()
    q = seqgen.random_protein(rng, 400)
    t = np.concatenate([seqgen.random_protein(rng, 50), seqgen.homolog(rng, q), seqgen.random_protein(rng, 40)])
    _check(q, t, sc)


def test_high_score_scoring_reaches_near_limit():
    # the extreme scoring used by the high-score golden pair: self-alignment is
    # the diagonal sum, 127 per base
    sc = seqgen.high_score_dna_scoring()
    a = seqgen.random_dna(np.random.default_rng(3), 500)
    r = oracle.sw_coords_mt(bytes(a), bytes(a), sc, threads=4, band=32, chunk=64)
    assert r["score"] == 127 * 500 and (r["q_begin"], r["q_end"], r["t_begin"], r["t_end"]) == (0, 499, 0, 499)


def test_golden_long_pairs_file():
    # the stored values were written by tests/golden/make_long_pairs.py (oracle only)
    data = json.load(open(os.path.join(HERE, "golden", "long_pairs.json")))
    for name in ("long_pair_500k", "high_score_528k"):
        d = data[name]
        assert d["oracle"] == "sw_coords_mt"
        assert 0 <= d["q_begin"] <= d["q_end"] < d["query_len"]
        assert 0 <= d["t_begin"] <= d["t_end"] < d["target_len"]
        # S <= min(n, m) * s_max and the span covers at least S / s_max bases
        smax = 1 if d["scoring"] == "dna" else 127
        assert 0 < d["score"] <= smax * min(d["q_end"] - d["q_begin"] + 1, d["t_end"] - d["t_begin"] + 1)
    # the high-score pair sits just below the 2^26 input limit, its score near it
    hs = data["high_score_528k"]
    assert hs["query_len"] * 127 < 2 ** 26 and hs["score"] > 2 ** 25
