"""Bit-exact parity with the oracle at the benchmark's scale and score range.

tests/golden/long_pairs.json holds score, end and start of two long pairs
computed by the CPU oracle alone (tests/golden/make_long_pairs.py, the
banded threaded form of the oracle's local pass):

  long_pair_500k   the long-pair workload at 500,000 bp with 5,000 bp flanks
                   (the benchmark's 5 Mbp pair, reduced), +1/-3, open 5,
                   extend 2; about 2.5e11 cells per pass
  high_score_528k  a 528,000 bp related pair scored +127/-127, open 200,
                   extend 50: its score (about 6.6e7) is just below the 2^26
                   input limit, so the forward pass's end-cell keys
                   (H << log2 R) reach the top of the 32-bit range at every
                   strip height, including 32 rows per lane

The GPU must reproduce every value exactly, in every strip height and with
and without the rows kept for the band traceback; in CIGAR mode the path must
also rescore to the score and span the reported rectangle."""
import json
import os

import numpy as np
import pytest

import seqgen
from test_gpu_long import _rescore

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "long_pairs.json")))
KEYS = ("score", "q_begin", "q_end", "t_begin", "t_end")


@pytest.fixture(scope="module")
def eng():
    import paper_2211_10769_amd as swh
    return swh.Engine(0)


def _inputs(name):
    g = GOLD[name]
    q, t = getattr(seqgen, g["generator"])(**g["args"])
    sc = seqgen.dna_scoring() if g["scoring"] == "dna" else seqgen.high_score_dna_scoring()
    assert (len(q), len(t)) == (g["query_len"], g["target_len"])
    return bytes(q), bytes(t), sc, g


@pytest.fixture(scope="module")
def long500():
    return _inputs("long_pair_500k")


@pytest.fixture(scope="module")
def high528():
    return _inputs("high_score_528k")


@pytest.mark.parametrize("rows", [0, 8, 16, 20, 32])
def test_long_pair_500k_coords(eng, opt, long500, rows):
    q, t, sc, g = long500
    opt("rows_per_lane", rows)
    got = eng.align(q, t, sc, mode="coords")
    assert {k: got[k] for k in KEYS} == {k: g[k] for k in KEYS}


def test_long_pair_500k_cigar(eng, long500):
    q, t, sc, g = long500
    got = eng.align(q, t, sc, mode="cigar", stats=True)
    assert {k: got[k] for k in KEYS} == {k: g[k] for k in KEYS}
    assert got["stats"]["traceback_retries"] == 0
    assert _rescore(q, t, got, sc) == g["score"]


def test_long_pair_500k_unpruned_reverse(eng, opt, long500):
    q, t, sc, g = long500
    opt("prune", 0)
    got = eng.align(q, t, sc, mode="coords")
    assert {k: got[k] for k in KEYS} == {k: g[k] for k in KEYS}


@pytest.mark.parametrize("rows", [0, 16, 32])
def test_high_score_528k_coords(eng, opt, high528, rows):
    q, t, sc, g = high528
    opt("rows_per_lane", rows)
    got = eng.align(q, t, sc, mode="coords")
    assert {k: got[k] for k in KEYS} == {k: g[k] for k in KEYS}
    assert g["score"] > 2 ** 25


def test_high_score_528k_score_mode_device_inputs(eng, high528):
    import torch
    q, t, sc, g = high528
    qd = torch.from_numpy(np.frombuffer(q, np.uint8).copy()).cuda()
    td = torch.from_numpy(np.frombuffer(t, np.uint8).copy()).cuda()
    got = eng.align_dev(qd, td, sc, mode="score")
    assert (got["score"], got["q_end"], got["t_end"]) == (g["score"], g["q_end"], g["t_end"])


def test_million_score_pair_cigar_against_oracle(eng):
    # an 18 kbp related pair at +127/-127: score in the millions, rectangle
    # small enough (under 4e8 cells) for the oracle's full-matrix walk
    import oracle
    rng = np.random.default_rng(2026)
    a = seqgen.random_dna(rng, 18_000)
    b = np.concatenate([seqgen.random_dna(rng, 300), seqgen.mutate(rng, a, 0.01, 0.002),
                        seqgen.random_dna(rng, 300)])
    sc = seqgen.high_score_dna_scoring()
    want = oracle.sw_align(bytes(a), bytes(b), sc)
    assert want["score"] > 2_000_000
    got = eng.align(bytes(a), bytes(b), sc, mode="cigar")
    assert {k: got[k] for k in want} == want
