"""The long DNA pair at full size (5,000,000 x 5,100,153, the size the
benchmark times): too big for the oracle, so the checks are properties that
hold at any size -- the CIGAR spans exactly the reported rectangle, starts
and ends with a pair, and rescored from the sequences gives the optimal
score -- plus agreement of the band traceback with the plain divide and
conquer on a 1 Mbp pair (the plain one is checked against the oracle at
small sizes)."""
import re

import numpy as np
import pytest

import seqgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    import paper_2211_10769_amd as swh
    return swh.Engine(0)


def _rescore(q, t, res, scoring):
    """Score of the alignment the CIGAR describes (gap of k costs o + (k-1) e)."""
    alphabet, mat, o, e = scoring
    lut = np.full(256, -1, dtype=np.int64)
    for k, ch in enumerate(alphabet):
        lut[ord(ch)] = k
    qc, tc = lut[np.frombuffer(q, np.uint8)], lut[np.frombuffer(t, np.uint8)]
    i, j, total, nq, nt = res["q_begin"], res["t_begin"], 0, 0, 0
    runs = re.findall(r"(\d+)([MID])", res["cigar"])
    assert "".join(n + op for n, op in runs) == res["cigar"]
    for n, op in runs:
        n = int(n)
        if op == "M":
            total += int(mat[qc[i:i + n], tc[j:j + n]].astype(np.int64).sum())
            i += n
            j += n
        elif op == "I":
            total -= o + (n - 1) * e
            i += n
        else:
            total -= o + (n - 1) * e
            j += n
    assert runs[0][1] == "M" and runs[-1][1] == "M"
    assert (i - 1, j - 1) == (res["q_end"], res["t_end"])
    return total


def test_full_size_pair(eng):
    q, t = seqgen.workload1()
    q, t = bytes(q), bytes(t)
    sc = seqgen.dna_scoring()
    res = eng.align(q, t, sc, mode="cigar", stats=True)
    st = res["stats"]
    assert res["score"] > 0.8 * len(q)
    assert st["traceback_bands"] > 100 and st["traceback_retries"] == 0, st
    assert st["cells_traceback"] < 0.05 * len(q) * len(t)
    assert _rescore(q, t, res, sc) == res["score"]


def test_bands_equal_plain_at_1mbp(eng, opt):
    q, t = seqgen.workload1(1_000_000, flank=10_000)
    q, t = bytes(q), bytes(t)
    sc = seqgen.dna_scoring()
    opt("band_rows", 8192)
    banded = eng.align(q, t, sc, mode="cigar", stats=True)
    opt("band_rows", -1)
    plain = eng.align(q, t, sc, mode="cigar", stats=True)
    assert banded["stats"]["traceback_bands"] > 50 and plain["stats"]["traceback_bands"] == 0
    keys = ["score", "q_begin", "q_end", "t_begin", "t_end", "cigar"]
    assert {k: banded[k] for k in keys} == {k: plain[k] for k in keys}
    assert _rescore(q, t, banded, sc) == banded["score"]
