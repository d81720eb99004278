"""Exhaustive enumeration on tiny inputs -- TEST INFRASTRUCTURE ONLY.

Independent of the DP in ``swh_oracle.c``: nothing here evaluates a
recurrence.  Scores are computed straight from the definition of an
alignment's score (paper: Background, Smith-Waterman; SW# suite paragraph for
affine open/extension penalties):

    score = sum of s(a_i, b_j) over aligned pairs
            - sum over maximal gap runs of  o + (k - 1) * e

and the local optimum is the maximum over every substring pair and every
alignment of it (0 for the empty alignment).  The canonical path is chosen by
enumerating every path through the three-state (H / E / F) alignment graph and
filtering, from the end backwards, by the preference order of the greedy
backward walk.
"""
from __future__ import annotations

import functools
from itertools import product


def _codes(s, alphabet):
    up = alphabet.upper()
    out = []
    for ch in (s.decode() if isinstance(s, (bytes, bytearray)) else s):
        out.append(up.index(ch.upper()))
    return out


@functools.lru_cache(maxsize=None)
def op_strings(p: int, q: int) -> tuple:
    """Every string over {M, I, D} consuming exactly p query and q target residues."""
    if p == 0 and q == 0:
        return ("",)
    res = []
    if p > 0 and q > 0:
        res += [s + "M" for s in op_strings(p - 1, q - 1)]
    if p > 0:
        res += [s + "I" for s in op_strings(p - 1, q)]
    if q > 0:
        res += [s + "D" for s in op_strings(p, q - 1)]
    return tuple(res)


def score_ops(ops: str, A, B, mat, o: int, e: int) -> int:
    """Score of one alignment of A vs B written as an op string (maximal gap runs)."""
    i = j = 0
    total = 0
    k = 0
    while k < len(ops):
        op = ops[k]
        if op == "M":
            total += int(mat[A[i]][B[j]])
            i += 1
            j += 1
            k += 1
            continue
        run = 0
        while k < len(ops) and ops[k] == op:
            run += 1
            k += 1
        total -= o + (run - 1) * e
        if op == "I":
            i += run
        else:
            j += run
    assert i == len(A) and j == len(B)
    return total


def local_all(a, b, scoring):
    """S and the list of optimal (i1, i2, j1, j2, ops), 1-based inclusive."""
    alphabet, mat, o, e = scoring
    A, B = _codes(a, alphabet), _codes(b, alphabet)
    n, m = len(A), len(B)
    best = 0
    opt = []
    for i1 in range(1, n + 1):
        for i2 in range(i1, n + 1):
            for j1 in range(1, m + 1):
                for j2 in range(j1, m + 1):
                    sa, sb = A[i1 - 1:i2], B[j1 - 1:j2]
                    for ops in op_strings(len(sa), len(sb)):
                        sc = score_ops(ops, sa, sb, mat, o, e)
                        if sc > best:
                            best = sc
                            opt = [(i1, i2, j1, j2, ops)]
                        elif sc == best and best > 0:
                            opt.append((i1, i2, j1, j2, ops))
    return best, opt


def local_result(a, b, scoring):
    """dict(score, q_begin, q_end, t_begin, t_end) by the end/start rules, 0-based."""
    S, opt = local_all(a, b, scoring)
    if S == 0:
        return dict(score=0, q_begin=-1, q_end=-1, t_begin=-1, t_end=-1)
    end = min((x[1], x[3]) for x in opt)                     # first in row-major order
    starts = [(x[0], x[2]) for x in opt if (x[1], x[3]) == end]
    start = max(starts)                                      # shortest co-optimal alignment
    return dict(score=S, q_begin=start[0] - 1, q_end=end[0] - 1,
                t_begin=start[1] - 1, t_end=end[1] - 1)


def _state_paths(A, B, mat, o, e):
    """Every path of the H/E/F graph from H(0,0) to H(p,q), walked backwards.

    Yields (score, ranks, ops_backward): ranks[k] is the preference rank of the
    predecessor chosen at the k-th node (0 = most preferred).
    Preferences: at H: diagonal(0) > F(1) > E(2); at F: open from H(0) > extend F(1);
    at E: open from H(0) > extend E(1).
    """
    p, q = len(A), len(B)

    def walk(kind, i, j):
        if kind == "H" and i == 0 and j == 0:
            yield 0, (), ""
            return
        if kind == "H":
            if i > 0 and j > 0:
                s = int(mat[A[i - 1]][B[j - 1]])
                for sc, r, ops in walk("H", i - 1, j - 1):
                    yield sc + s, (0,) + r, "M" + ops
            if i > 0:
                for sc, r, ops in walk("F", i, j):
                    yield sc, (1,) + r, ops
            if j > 0:
                for sc, r, ops in walk("E", i, j):
                    yield sc, (2,) + r, ops
        elif kind == "F":          # query residue A[i-1] against a gap
            for sc, r, ops in walk("H", i - 1, j):
                yield sc - o, (0,) + r, "I" + ops
            if i - 1 > 0:
                for sc, r, ops in walk("F", i - 1, j):
                    yield sc - e, (1,) + r, "I" + ops
        else:                      # target residue B[j-1] against a gap
            for sc, r, ops in walk("H", i, j - 1):
                yield sc - o, (0,) + r, "D" + ops
            if j - 1 > 0:
                for sc, r, ops in walk("E", i, j - 1):
                    yield sc - e, (1,) + r, "D" + ops

    yield from walk("H", p, q)


def cigar_of(ops_forward: str) -> str:
    out = []
    k = 0
    while k < len(ops_forward):
        c = ops_forward[k]
        r = 0
        while k < len(ops_forward) and ops_forward[k] == c:
            r += 1
            k += 1
        out.append(f"{r}{c}")
    return "".join(out)


def global_canonical(a, b, scoring):
    """(global optimum, canonical CIGAR) of a vs b by path enumeration."""
    alphabet, mat, o, e = scoring
    A, B = _codes(a, alphabet), _codes(b, alphabet)
    paths = list(_state_paths(A, B, mat, o, e))
    best = max(p[0] for p in paths)
    optimal = [p for p in paths if p[0] == best]
    chosen = min(optimal, key=lambda p: p[1])
    ops_backward = chosen[2]     # first character = the last op of the alignment
    return best, cigar_of(ops_backward[::-1])


def local_with_cigar(a, b, scoring):
    """Local result plus canonical CIGAR of the chosen rectangle."""
    r = local_result(a, b, scoring)
    if r["score"] == 0:
        r["cigar"] = ""
        return r
    sa = a[r["q_begin"]:r["q_end"] + 1]
    sb = b[r["t_begin"]:r["t_end"] + 1]
    g, cig = global_canonical(sa, sb, scoring)
    assert g == r["score"]
    r["cigar"] = cig
    return r


def all_strings(alphabet: str, n: int):
    for t in product(alphabet, repeat=n):
        yield "".join(t)


def hw_result(a, b, scoring):
    """Semi-global result by enumeration: the whole query against every target
    substring b[j1..j2] aligned end to end (or against no target residue at
    all), the residues around it unpenalised.  End = smallest j2 among the
    optima, start = largest j1 among those with that end; the CIGAR is the
    canonical path of the chosen rectangle."""
    alphabet, mat, o, e = scoring
    A, B = _codes(a, alphabet), _codes(b, alphabet)
    n, m = len(A), len(B)
    if n == 0:
        return dict(score=0, q_begin=-1, q_end=-1, t_begin=-1, t_end=-1, cigar="")
    cands = [(-(o + (n - 1) * e), 0, 0)]               # every query residue against a gap
    for j1 in range(1, m + 1):
        for j2 in range(j1, m + 1):
            sb = B[j1 - 1:j2]
            best = max(score_ops(ops, A, sb, mat, o, e) for ops in op_strings(n, len(sb)))
            cands.append((best, j1, j2))
    S = max(c[0] for c in cands)
    end = min(c[2] for c in cands if c[0] == S)
    if end == 0:
        return dict(score=S, q_begin=0, q_end=n - 1, t_begin=-1, t_end=-1, cigar=f"{n}I")
    start = max(c[1] for c in cands if c[0] == S and c[2] == end)
    g, cig = global_canonical(a, b[start - 1:end], scoring)
    assert g == S
    return dict(score=S, q_begin=0, q_end=n - 1, t_begin=start - 1, t_end=end - 1, cigar=cig)


def ov_result(a, b, scoring):
    """Overlap result by enumeration: every rectangle a[i1..i2] x b[j1..j2]
    that starts on the first row or column (i1 = 1 or j1 = 1) and ends on the
    last (i2 = n or j2 = m), aligned end to end, the residues outside it
    unpenalised; the empty overlap scores 0 and reports no alignment.  End =
    the smallest (i2, j2) among the optima, start = the largest (i1, j1)
    among those with that end; the CIGAR is the canonical path of the chosen
    rectangle."""
    alphabet, mat, o, e = scoring
    A, B = _codes(a, alphabet), _codes(b, alphabet)
    n, m = len(A), len(B)
    none = dict(score=0, q_begin=-1, q_end=-1, t_begin=-1, t_end=-1, cigar="")
    cands = []
    for i1 in range(1, n + 1):
        for j1 in range(1, m + 1):
            if i1 != 1 and j1 != 1:
                continue
            for i2 in range(i1, n + 1):
                for j2 in range(j1, m + 1):
                    if i2 != n and j2 != m:
                        continue
                    sa, sb = A[i1 - 1:i2], B[j1 - 1:j2]
                    best = max(score_ops(ops, sa, sb, mat, o, e) for ops in op_strings(len(sa), len(sb)))
                    cands.append((best, i1, j1, i2, j2))
    if not cands:
        return none
    S = max(c[0] for c in cands)
    if S <= 0:
        return none
    end = min((c[3], c[4]) for c in cands if c[0] == S)
    start = max((c[1], c[2]) for c in cands if c[0] == S and (c[3], c[4]) == end)
    g, cig = global_canonical(a[start[0] - 1:end[0]], b[start[1] - 1:end[1]], scoring)
    assert g == S
    return dict(score=S, q_begin=start[0] - 1, q_end=end[0] - 1, t_begin=start[1] - 1, t_end=end[1] - 1,
                cigar=cig)
