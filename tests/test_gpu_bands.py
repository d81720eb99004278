"""GPU parity of the band traceback: the first split of the reconstruction
taken from rows kept by the two score passes.  The band-rows option forces kept
rows every few strips on inputs small enough for the oracle; the CIGAR must
equal the oracle's full-matrix greedy walk byte for byte, and the bands must
be used (no fall back to the plain divide and conquer)."""
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


def _cmp(eng, a, b, sc, min_bands=2):
    got = eng.align(a, b, sc, mode="cigar", stats=True)
    st = got["stats"]
    want = oracle.sw_align(a, b, sc, want_cigar=True)
    g = {k: got[k] for k in KEYS}
    w = {k: want[k] for k in KEYS}
    assert g == w, (len(a), len(b), {k: (g[k], w[k]) for k in KEYS if g[k] != w[k]})
    assert st["traceback_retries"] == 0
    assert st["traceback_bands"] >= min_bands, st
    return st


@pytest.fixture
def bands(opt):
    def set_(rows, R=None):
        opt("band_rows", rows)
        if R is not None:
            opt("rows_per_lane", R)
    return set_


@pytest.mark.parametrize("flank", [0, 1, 255, 700])
def test_flanks_move_the_cuts(eng, bands, flank):
    # the rectangle starts and ends at different offsets from the kept rows
    bands(256, R=4)
    rng = np.random.default_rng(100 + flank)
    sc = seqgen.dna_scoring()
    a = seqgen.random_dna(rng, 6000)
    q = np.concatenate([seqgen.random_dna(rng, flank), a, seqgen.random_dna(rng, 37)])
    t = np.concatenate([seqgen.random_dna(rng, 91), seqgen.mutate(rng, a, 0.03, 0.01), seqgen.random_dna(rng, flank)])
    _cmp(eng, bytes(q), bytes(t), sc, min_bands=10)


@pytest.mark.parametrize("rows,R", [(512, 8), (1024, 16), (2048, 8), (1280, 20), (1536, 24), (2048, 32)])
def test_strip_heights(eng, bands, rows, R):
    bands(rows, R=R)
    rng = np.random.default_rng(rows + R)
    sc = seqgen.dna_scoring()
    a = seqgen.random_dna(rng, 9000)
    b = np.concatenate([seqgen.random_dna(rng, 300), seqgen.mutate(rng, a, 0.02, 0.005), seqgen.random_dna(rng, 300)])
    _cmp(eng, bytes(a), bytes(b), sc, min_bands=3)


def test_long_gaps_cross_kept_rows(eng, bands):
    # a 900-residue insertion in the query and a 700-residue deletion: vertical
    # and horizontal gaps that span kept rows
    bands(256, R=4)
    rng = np.random.default_rng(7)
    sc = seqgen.dna_scoring()
    x, y, z = (seqgen.random_dna(rng, n) for n in (2500, 2500, 2500))
    ins = seqgen.random_dna(rng, 900)
    dele = seqgen.random_dna(rng, 700)
    q = np.concatenate([x, ins, y, z])
    t = np.concatenate([seqgen.mutate(rng, x, 0.01, 0.0), y, dele, seqgen.mutate(rng, z, 0.01, 0.0)])
    # nearly every kept row must be a clean cut, those inside the gaps included
    st = _cmp(eng, bytes(q), bytes(t), sc, min_bands=int(0.8 * len(q) / 256))
    assert st["cells_traceback"] < 0.5 * len(q) * len(t)


def test_tie_heavy(eng, bands):
    # binary alphabet with o = e = 1: many co-optimal paths, ambiguous kept rows join bands
    bands(256, R=4)
    tie = ("AC", np.array([[1, -1], [-1, 1]], dtype=np.int8), 1, 1)
    rng = np.random.default_rng(12)
    for n in (1500, 4000):
        a = rng.choice(np.frombuffer(b"AC", np.uint8), n)
        flip = rng.random(n) < 0.08
        b = np.where(flip, np.where(a == ord("A"), ord("C"), ord("A")), a).astype(np.uint8)
        got = eng.align(bytes(a), bytes(b), tie, mode="cigar", stats=True)
        st = got["stats"]
        want = oracle.sw_align(bytes(a), bytes(b), tie, want_cigar=True)
        assert {k: got[k] for k in KEYS} == {k: want[k] for k in KEYS}
        assert st["traceback_retries"] == 0


def test_repeats_and_homopolymers(eng, bands):
    bands(256, R=4)
    dna = seqgen.dna_scoring()
    unit = b"ACGTTGCA"
    for a, b in [(unit * 600, unit * 590 + b"ACG" + unit * 5), (b"A" * 3000, b"A" * 2990),
                 (b"AC" * 1500 + b"GT" * 700, b"AC" * 1480 + b"GT" * 720)]:
        got = eng.align(a, b, dna, mode="cigar", stats=True)
        st = got["stats"]
        want = oracle.sw_align(a, b, dna, want_cigar=True)
        assert {k: got[k] for k in KEYS} == {k: want[k] for k in KEYS}
        assert st["traceback_retries"] == 0


def test_several_optimal_starts(eng, bands):
    # the query's first half occurs twice in the target, so optimal alignments
    # ending at the same cell can start at different places
    bands(256, R=4)
    rng = np.random.default_rng(21)
    dna = seqgen.dna_scoring()
    h1, h2 = seqgen.random_dna(rng, 1500), seqgen.random_dna(rng, 2500)
    q = np.concatenate([h1, h2])
    t = np.concatenate([h1, seqgen.random_dna(rng, 3), h1, h2])
    got = eng.align(bytes(q), bytes(t), dna, mode="cigar", stats=True)
    st = got["stats"]
    want = oracle.sw_align(bytes(q), bytes(t), dna, want_cigar=True)
    assert {k: got[k] for k in KEYS} == {k: want[k] for k in KEYS}
    assert st["traceback_retries"] == 0


def test_protein(eng, bands):
    bands(256, R=4)
    rng = np.random.default_rng(31)
    sc = seqgen.protein_scoring()
    a = seqgen.random_protein(rng, 5000)
    b = np.concatenate([seqgen.random_protein(rng, 60), seqgen.homolog(rng, a), seqgen.random_protein(rng, 40)])
    _cmp(eng, bytes(a), bytes(b), sc, min_bands=2)


def test_disabled(eng, bands):
    rng = np.random.default_rng(41)
    sc = seqgen.dna_scoring()
    a = seqgen.random_dna(rng, 5000)
    b = seqgen.mutate(rng, a, 0.02, 0.005)
    bands(-1)
    st = _cmp(eng, bytes(a), bytes(b), sc, min_bands=0)
    assert st["traceback_bands"] == 0
