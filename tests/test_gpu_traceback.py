"""GPU parity of the CIGAR (linear-space traceback) against the oracle's
full-matrix greedy walk: byte-for-byte equal CIGARs."""
import numpy as np
import pytest

import oracle
import seqgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    import paper_2211_10769_amd as swh
    return swh.Engine(0)


def _cmp(eng, a, b, sc):
    got = eng.align(a, b, sc, mode="cigar")
    want = oracle.sw_align(a, b, sc, want_cigar=True)
    keys = ["score", "q_begin", "q_end", "t_begin", "t_end", "cigar"]
    g = {k: got[k] for k in keys}
    w = {k: want[k] for k in keys}
    assert g == w, (len(a), len(b), {k: (g[k], w[k]) for k in keys if g[k] != w[k]})
    return got


def test_small_cases(eng):
    sc = seqgen.dna_scoring()
    for a, b in [("A", "A"), ("ACGT", "ACGT"), ("AAAA", "CCCC"), ("ACGTTTACGT", "ACGT"),
                 ("ACACACACACGTGTGTGTGTG", "ACACACACACTGTGTGTGTG")]:
        _cmp(eng, a, b, sc)


def test_workload0_full(eng):
    a, b = seqgen.workload0()
    _cmp(eng, bytes(a), bytes(b), seqgen.dna_scoring())


@pytest.mark.parametrize("n", [300, 1500, 4000])
def test_similar_dna(eng, n):
    rng = np.random.default_rng(n)
    sc = seqgen.dna_scoring()
    a = seqgen.random_dna(rng, n)
    b = np.concatenate([seqgen.random_dna(rng, 50), seqgen.mutate(rng, a, 0.03, 0.01), seqgen.random_dna(rng, 70)])
    _cmp(eng, bytes(a), bytes(b), sc)


@pytest.mark.parametrize("leaf", [1, 7, 64, 1000])
def test_leaf_size_sweep(eng, leaf, opt):
    # tiny leaves force deep recursion on small inputs; tie-heavy scoring
    opt("tb_leaf", leaf)
    rng = np.random.default_rng(leaf)
    tie = ("AC", np.array([[1, -1], [-1, 1]], dtype=np.int8), 1, 1)
    for n in (40, 200):
        a = bytes(rng.choice(np.frombuffer(b"AC", np.uint8), n))
        b = bytes(rng.choice(np.frombuffer(b"AC", np.uint8), n + 13))
        _cmp(eng, a, b, tie)
    dna = seqgen.dna_scoring()
    a = seqgen.random_dna(rng, 700)
    b = seqgen.mutate(rng, a, 0.05, 0.02)
    _cmp(eng, bytes(a), bytes(b), dna)
    _cmp(eng, b"A" * 300 + b"C" * 5 + b"A" * 200, b"A" * 480 + b"C" * 3, dna)


def test_tandem_repeats_and_polya(eng):
    dna = seqgen.dna_scoring()
    unit = b"ACGTTGCA"
    _cmp(eng, unit * 120, unit * 117 + b"ACG" + unit * 5, dna)
    _cmp(eng, b"A" * 2000, b"A" * 1990, dna)
    lin = ("ACGT", np.array([[2 if i == j else -1 for j in range(4)] for i in range(4)], dtype=np.int8), 2, 2)
    rng = np.random.default_rng(5)
    a = seqgen.random_dna(rng, 1200)
    _cmp(eng, bytes(a), bytes(seqgen.mutate(rng, a, 0.1, 0.03)), lin)


def test_protein_homologs(eng):
    rng = np.random.default_rng(6)
    sc = seqgen.protein_scoring()
    for n in (150, 900, 2500):
        a = seqgen.random_protein(rng, n)
        b = np.concatenate([seqgen.random_protein(rng, 40), seqgen.homolog(rng, a), seqgen.random_protein(rng, 40)])
        _cmp(eng, bytes(a), bytes(b), sc)


def test_cigar_buffer_too_small(eng):
    import ctypes
    import paper_2211_10769_amd as swh
    from paper_2211_10769_amd import _lib
    sc = swh.Scoring(*seqgen.dna_scoring())
    a, b = b"ACGTACGTAAACGT", b"ACGTACGTACGT"
    out = _lib.swh_alignment()
    buf = ctypes.create_string_buffer(2)
    need = ctypes.c_int64()
    st = eng.L.swh_align(eng.h, a, len(a), b, len(b), ctypes.byref(sc.c), 2, ctypes.byref(out), buf, 2,
                         ctypes.byref(need), None)
    assert st == -4
    want = oracle.sw_align(a, b, seqgen.dna_scoring())["cigar"]
    assert need.value == len(want)
