"""GPU parity of the pairwise path against the CPU oracle (bit-exact)."""
import numpy as np
import pytest

import oracle
import seqgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    import paper_2211_10769_amd as swh
    return swh.Engine(0)


def _cmp(eng, a, b, sc, mode="coords"):
    got = eng.align(a, b, sc, mode=mode)
    want = oracle.sw_align(a, b, sc, want_cigar=(mode == "cigar"))
    keys = ["score", "q_end", "t_end"] + (["q_begin", "t_begin"] if mode != "score" else [])
    if mode == "cigar":
        keys.append("cigar")
    g = {k: got[k] for k in keys}
    w = {k: want[k] for k in keys}
    assert g == w, (len(a), len(b), g, w)
    return got


def test_tiny_and_degenerate(eng):
    sc = seqgen.dna_scoring()
    cases = [("A", "A"), ("A", "C"), ("ACGT", "ACGT"), ("AAAA", "CCCC"), ("ACGTTTACGT", "ACGT"),
             ("ACGT", "ACGTTTACGT"), ("A" * 70, "A" * 130), ("ACGT" * 50, "TGCA" * 37)]
    for a, b in cases:
        _cmp(eng, a, b, sc)


def test_empty_inputs(eng):
    r = eng.align("", "ACGT", seqgen.dna_scoring(), mode="coords")
    assert r["score"] == 0 and r["q_begin"] == -1
    r = eng.align("ACGT", "", seqgen.dna_scoring(), mode="coords")
    assert r["score"] == 0 and r["t_end"] == -1


@pytest.mark.parametrize("n,m", [(1, 1000), (63, 65), (64, 64), (255, 257), (1000, 3),
                                 (1025, 4097), (4097, 1025), (5000, 7000)])
def test_random_dna_ragged(eng, n, m):
    rng = np.random.default_rng(n * 7919 + m)
    sc = seqgen.dna_scoring()
    a = seqgen.random_dna(rng, n)
    b = seqgen.mutate(rng, a, 0.05, 0.01) if n > 100 else seqgen.random_dna(rng, m)
    b = np.concatenate([seqgen.random_dna(rng, m // 3), b, seqgen.random_dna(rng, m // 3)])[:max(m, 1)]
    _cmp(eng, bytes(a), bytes(b), sc)


def test_tie_heavy(eng):
    mat = np.array([[1, -1], [-1, 1]], dtype=np.int8)
    sc = ("AC", mat, 1, 1)
    rng = np.random.default_rng(3)
    for n in (50, 300, 2000):
        a = bytes(rng.choice(np.frombuffer(b"AC", np.uint8), n))
        b = bytes(rng.choice(np.frombuffer(b"AC", np.uint8), n + 17))
        _cmp(eng, a, b, sc)
    _cmp(eng, b"A" * 3000, b"A" * 2000, sc)


def test_protein_blosum62(eng):
    rng = np.random.default_rng(4)
    sc = seqgen.protein_scoring()
    for n, m in ((120, 340), (1500, 900), (5000, 3000)):
        a = seqgen.random_protein(rng, n)
        b = np.concatenate([seqgen.random_protein(rng, m // 2), seqgen.homolog(rng, a[: n // 2]),
                            seqgen.random_protein(rng, m // 2)])
        _cmp(eng, bytes(a), bytes(b), sc)


def test_workload0_full(eng):
    a, b = seqgen.workload0()
    _cmp(eng, bytes(a), bytes(b), seqgen.dna_scoring())


def test_rows_per_lane_paths(eng):
    # strip heights of 64*4, 64*8 and 64*16 rows are picked by query length
    sc = seqgen.dna_scoring()
    for n, m in ((30_000, 3_000), (210_000, 1_500)):
        q, t = seqgen.workload1(n, flank=200)
        _cmp(eng, bytes(q), bytes(t[:m]), sc)


def test_bad_symbol(eng):
    import paper_2211_10769_amd as swh
    with pytest.raises(swh.SwhError) as ei:
        eng.align("ACGN", "ACGT", seqgen.dna_scoring(), mode="score")
    assert ei.value.status == -2
    assert "position 3" in str(ei.value)


@pytest.mark.parametrize("rows,grid", [(4, 0), (8, 0), (16, 0), (20, 0), (24, 0), (32, 0), (16, 1), (8, 3), (20, 3),
                                       (24, 2), (32, 2)])
def test_forced_strip_shapes(eng, rows, grid, opt):
    # every strip height and tiny persistent grids (one wave doing every strip in turn)
    opt("rows_per_lane", rows)
    opt("grid", grid)
    rng = np.random.default_rng(rows * 100 + grid)
    sc = seqgen.dna_scoring()
    a = seqgen.random_dna(rng, 6000)
    b = np.concatenate([seqgen.random_dna(rng, 700), seqgen.mutate(rng, a, 0.04, 0.01),
                        seqgen.random_dna(rng, 333)])
    _cmp(eng, bytes(a), bytes(b), sc)
    _cmp(eng, bytes(seqgen.random_dna(rng, 2100)), bytes(seqgen.random_dna(rng, 1900)), sc)
    q = seqgen.random_protein(rng, 1700)
    _cmp(eng, bytes(q), bytes(seqgen.homolog(rng, q)), seqgen.protein_scoring())
