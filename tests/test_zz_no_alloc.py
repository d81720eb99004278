"""swh_align_dev_noalloc (the entry point that allocates nothing) against
swh_align_dev through the C ABI: equal results on two calls in a row, the
second with a smaller input (the static array keeps the first call's
contents), in both modes; inputs beyond the array's size are refused."""
import ctypes

import numpy as np
import pytest

import oracle
import seqgen

pytestmark = pytest.mark.gpu

E_INVAL, E_RANGE = -1, -4


@pytest.fixture(scope="module")
def swh():
    import paper_2211_10769_amd as m
    return m


@pytest.fixture(scope="module")
def eng(swh):
    return swh.Engine(0)


def _noalloc(swh, qd, td, sc, mode, stream):
    out = swh._lib.swh_alignment()
    rc = swh._lib.load().swh_align_dev_noalloc(0, qd.data_ptr() if qd.numel() else None, qd.numel(),
                                               td.data_ptr() if td.numel() else None, td.numel(),
                                               ctypes.byref(sc.c), mode, stream, ctypes.byref(out))
    return rc, dict(score=out.score, q_begin=out.q_begin, q_end=out.q_end, t_begin=out.t_begin, t_end=out.t_end)


def _pair(rng, n, flank):
    a = seqgen.random_dna(rng, n)
    b = np.concatenate([seqgen.random_dna(rng, flank), seqgen.mutate(rng, a, 0.03, 0.005),
                        seqgen.random_dna(rng, flank)])
    return a, b


KEYS = ("score", "q_begin", "q_end", "t_begin", "t_end")


def test_two_calls_match_align_dev(swh, eng):
    import torch
    sc = swh.dna_scoring()
    rng = np.random.default_rng(77)
    stream = torch.cuda.current_stream().cuda_stream
    for n, flank in ((300_000, 20_000), (7_000, 900)):   # the second call is smaller
        a, b = _pair(rng, n, flank)
        qd = torch.from_numpy(a.copy()).cuda()
        td = torch.from_numpy(b.copy()).cuda()
        for mode, name in ((1, "coords"), (0, "score")):
            rc, got = _noalloc(swh, qd, td, sc, mode, stream)
            assert rc == 0
            want = eng.align_dev(qd, td, sc, mode=name, stream=stream)
            assert got == {k: want[k] for k in KEYS}, (n, name, got, want)
        if n < 10_000:
            o = oracle.sw_align(bytes(a), bytes(b), seqgen.dna_scoring(), want_cigar=False)
            assert got["score"] == o["score"]


def test_protein_and_no_hit(swh, eng):
    import torch
    sc = swh.Scoring(*seqgen.protein_scoring())
    rng = np.random.default_rng(78)
    q = seqgen.random_protein(rng, 900)
    t = np.concatenate([seqgen.random_protein(rng, 300), seqgen.homolog(rng, q), seqgen.random_protein(rng, 100)])
    qd = torch.from_numpy(q.copy()).cuda()
    td = torch.from_numpy(t.copy()).cuda()
    rc, got = _noalloc(swh, qd, td, sc, 1, None)
    want = oracle.sw_align(bytes(q), bytes(t), seqgen.protein_scoring(), want_cigar=False)
    assert rc == 0 and got == {k: want[k] for k in KEYS}
    dna = swh.dna_scoring()
    qd = torch.from_numpy(np.frombuffer(b"AAAA", np.uint8).copy()).cuda()
    td = torch.from_numpy(np.frombuffer(b"CCCC", np.uint8).copy()).cuda()
    rc, got = _noalloc(swh, qd, td, dna, 1, None)
    assert rc == 0 and got == dict(score=0, q_begin=-1, q_end=-1, t_begin=-1, t_end=-1)


def test_limits_and_arguments(swh):
    import torch
    sc = swh.dna_scoring()
    L = swh._lib.load()
    big = torch.zeros(8_000_000, dtype=torch.uint8, device="cuda") + ord("A")
    out = swh._lib.swh_alignment()
    # 2 * 8e6 + 10 * 8e6 bytes > 64 MiB: refused, nothing run
    assert L.swh_align_dev_noalloc(0, big.data_ptr(), big.numel(), big.data_ptr(), big.numel(),
                                   ctypes.byref(sc.c), 0, None, ctypes.byref(out)) == E_RANGE
    small = big[:100]
    assert L.swh_align_dev_noalloc(0, small.data_ptr(), 100, small.data_ptr(), 100, ctypes.byref(sc.c), 2, None,
                                   ctypes.byref(out)) == E_INVAL     # CIGAR mode is not offered
    assert L.swh_align_dev_noalloc(-1, small.data_ptr(), 100, small.data_ptr(), 100, ctypes.byref(sc.c), 0, None,
                                   ctypes.byref(out)) == E_INVAL
    assert L.swh_align_dev_noalloc(0, None, 100, small.data_ptr(), 100, ctypes.byref(sc.c), 0, None,
                                   ctypes.byref(out)) == E_INVAL
    # after the refusals a call works
    assert L.swh_align_dev_noalloc(0, small.data_ptr(), 100, small.data_ptr(), 100, ctypes.byref(sc.c), 1, None,
                                   ctypes.byref(out)) == 0
    assert (out.score, out.q_begin, out.q_end) == (100, 0, 99)
