"""Throughput sweeps over the alignment forms, scoring schemes, query lengths
and strip shapes (the paper's Experimental Work: algorithm variants,
substitution matrices and gap penalties, query lengths and work-group sizes).

    python experiments.py [--pair-n 2000000] [--db-size 100000] [--out FILE]

Prints one markdown report (also written to --out).  Every input is seeded
and synthetic (the generators in seqgen); GCUPS = DP cells / kernel or call
time.  Needs the HIP library (paper_2211_10769_amd) and one GPU.
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np


def log(msg):
    print(f"[experiments] {msg}", file=sys.stderr, flush=True)


def forms(swh, eng, seqgen, n):
    """The four alignment forms on one related DNA pair, score only."""
    q, t = seqgen.workload1(n, flank=0)
    q, t = bytes(q), bytes(t)
    sc = swh.Scoring(*seqgen.dna_scoring())
    rows = []
    for form in ("local", "global", "semiglobal", "overlap"):
        eng.align(q[:200_000], t[:200_000], sc, mode="score", alignment=form)   # warm-up
        t0 = time.perf_counter()
        r = eng.align(q, t, sc, mode="score", stats=True, alignment=form)
        wall = time.perf_counter() - t0
        st = r["stats"]
        rows.append((form, r["score"], st["cells_forward"], st["ms_forward"], wall))
        log(f"form {form}: {st['ms_forward']:.1f} ms")
    out = [f"## Alignment forms (score only, {len(q):,} x {len(t):,} bp related DNA pair, +1/-3, 5/2)", "",
           "| form | score | DP cells | kernel ms | kernel GCUPS | call s | call GCUPS |", "|---|---|---|---|---|---|---|"]
    for form, s, cells, ms, wall in rows:
        out.append(f"| {form} | {s:,} | {cells:.3e} | {ms:,.1f} | {cells / ms / 1e6:,.0f} | {wall:.2f} | "
                   f"{cells / wall / 1e9:,.0f} |")
    return out


def dna_schemes(swh, eng, seqgen, n):
    """Local score pass under several DNA scoring schemes."""
    q, t = seqgen.workload1(n, flank=0)
    q, t = bytes(q), bytes(t)
    out = [f"## DNA scoring schemes (local score pass, {len(q):,} x {len(t):,} bp)", "",
           "| match | mismatch | open | extend | score | kernel ms | GCUPS |", "|---|---|---|---|---|---|---|"]
    for (ma, mi, o, e) in ((1, -3, 5, 2), (1, -1, 2, 1), (2, -3, 5, 2), (5, -4, 10, 1)):
        sc = swh.dna_scoring(ma, mi, o, e)
        eng.align(q[:100_000], t[:100_000], sc, mode="score")
        r = eng.align(q, t, sc, mode="score", stats=True)
        st = r["stats"]
        out.append(f"| {ma} | {mi} | {o} | {e} | {r['score']:,} | {st['ms_forward']:,.1f} | "
                   f"{st['cells_forward'] / st['ms_forward'] / 1e6:,.0f} |")
        log(f"dna scheme {ma}/{mi}/{o}/{e} done")
    return out


def protein_schemes(swh, eng, seqgen, db_size):
    """Database search under BLOSUM62, 50 and 45 with several gap penalties, and
    with BLOSUM62 doubled (a higher-scoring table: more 16-bit saturation)."""
    qs, (cat, off) = seqgen.workload2(n_db=db_size)
    alphabet, mat, _, _ = seqgen.protein_scoring()
    qcat, qoff = swh._concat(qs)
    out = [f"## Protein scoring schemes (database search, {len(qs)} queries vs {db_size:,} proteins, top-10)", "",
           "| matrix | open | extend | search ms | GCUPS | 16-bit saturated pairs |", "|---|---|---|---|---|---|"]
    doubled = np.clip(np.asarray(mat, dtype=np.int16) * 2, -128, 127).astype(np.int8)
    b50 = seqgen.blosum_scoring(50)
    b45 = seqgen.blosum_scoring(45)
    schemes = [("BLOSUM62", alphabet, mat, 10, 2), ("BLOSUM62", alphabet, mat, 10, 1),
               ("BLOSUM62", alphabet, mat, 11, 1), ("BLOSUM62", alphabet, mat, 12, 2),
               ("BLOSUM62", alphabet, mat, 6, 1), ("2 x BLOSUM62", alphabet, doubled, 20, 4),
               ("BLOSUM50", b50[0], b50[1], 10, 2), ("BLOSUM50", b50[0], b50[1], 13, 2),
               ("BLOSUM45", b45[0], b45[1], 10, 2), ("BLOSUM45", b45[0], b45[1], 14, 2)]
    for name, alph, m, o, e in schemes:
        db = swh.Database(eng, (cat, off), swh.Scoring(alph, m, o, e))
        db.search((qcat, qoff), k=10)
        t0 = time.perf_counter()
        reps = 2
        for _ in range(reps):
            _, _, st = db.search((qcat, qoff), k=10)
        dt = (time.perf_counter() - t0) / reps
        db.close()
        out.append(f"| {name} | {o} | {e} | {dt * 1e3:,.1f} | {st['cells'] / dt / 1e9:,.0f} | {st['saturated']:,} |")
        log(f"protein scheme {name} {o}/{e} done")
    return out


def query_lengths(swh, eng, seqgen, db_size):
    """Database search GCUPS against the length of a single query: the default
    launch (units shared by eight or twelve waves, oversize units on the
    single-pair kernel beside it) and one wave per unit with no routing."""
    _, (cat, off) = seqgen.workload2(n_db=db_size, n_queries=1)
    sc = swh.Scoring(*seqgen.protein_scoring())
    db = swh.Database(eng, (cat, off), sc)
    rng = seqgen.rng_for(2, 901)
    out = [f"## Query length (one query vs {db_size:,} proteins, BLOSUM62 10/2, top-10)", "",
           "| query residues | default ms | default GCUPS | one wave per unit ms | one wave per unit GCUPS |",
           "|---|---|---|---|---|"]
    for L in (100, 300, 1000, 3000, 5000):
        q = [bytes(seqgen.random_protein(rng, L))]
        row = []
        for waves, route in ((0, 0), (1, -1)):
            eng.set_option("db_waves", waves)
            eng.set_option("db_route", route)
            db.search(q, k=10)
            t0 = time.perf_counter()
            reps = 5
            for _ in range(reps):
                _, _, st = db.search(q, k=10)
            dt = (time.perf_counter() - t0) / reps
            row += [dt * 1e3, st["cells"] / dt / 1e9]
        eng.set_option("db_waves", 0)
        eng.set_option("db_route", 0)
        out.append(f"| {L:,} | {row[0]:,.2f} | {row[1]:,.0f} | {row[2]:,.2f} | {row[3]:,.0f} |")
        log(f"query length {L} done")
    db.close()
    return out


def strip_shapes(swh, eng, seqgen, n):
    """Local score pass with each strip height forced (rows per lane R, strip
    = 64 R rows), against the installed rule."""
    q, t = seqgen.workload1(n, flank=0)
    q, t = bytes(q), bytes(t)
    sc = swh.Scoring(*seqgen.dna_scoring())
    saved = eng.tune_table()
    out = [f"## Strip height (local score pass, {len(q):,} x {len(t):,} bp)", "",
           "| rows per lane | strips | kernel ms | GCUPS |", "|---|---|---|---|"]
    try:
        for R in (8, 16, 20, 24, 32):
            eng.set_tune_table([dict(max_rows=1 << 40, rows_per_lane=R, waves_per_simd=0)])
            eng.align(q[:100_000], t[:100_000], sc, mode="score")
            r = eng.align(q, t, sc, mode="score", stats=True)
            st = r["stats"]
            out.append(f"| {R} | {-(-len(q) // (64 * R)):,} | {st['ms_forward']:,.1f} | "
                       f"{st['cells_forward'] / st['ms_forward'] / 1e6:,.0f} |")
            log(f"strip height R={R} done")
    finally:
        eng.set_tune_table(saved)
    r = eng.align(q, t, sc, mode="score", stats=True)
    st = r["stats"]
    out.append(f"| rule ({saved[-1]['rows_per_lane'] if saved else 'default'}) | — | {st['ms_forward']:,.1f} | "
               f"{st['cells_forward'] / st['ms_forward'] / 1e6:,.0f} |")
    return out


def main():
    p = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    p.add_argument("--pair-n", type=int, default=2_000_000, help="query length of the DNA pair legs")
    p.add_argument("--db-size", type=int, default=100_000, help="database proteins of the search legs")
    p.add_argument("--out", default=None, help="also write the report here")
    p.add_argument("--only", default=None, help="comma list of legs: forms,dna,protein,qlen,shapes")
    args = p.parse_args()
    import paper_2211_10769_amd as swh
    import seqgen
    eng = swh.Engine(0)
    legs = {"forms": lambda: forms(swh, eng, seqgen, args.pair_n),
            "dna": lambda: dna_schemes(swh, eng, seqgen, args.pair_n // 2),
            "protein": lambda: protein_schemes(swh, eng, seqgen, args.db_size),
            "qlen": lambda: query_lengths(swh, eng, seqgen, args.db_size),
            "shapes": lambda: strip_shapes(swh, eng, seqgen, args.pair_n)}
    chosen = args.only.split(",") if args.only else list(legs)
    report = ["# Throughput sweeps", ""]
    for name in chosen:
        report += legs[name]() + [""]
    text = "\n".join(report)
    print(text, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text + "\n")
    eng.close()


if __name__ == "__main__":
    main()
