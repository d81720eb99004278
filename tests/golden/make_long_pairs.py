"""Write tests/golden/long_pairs.json: score, end and start of the long DNA
pairs that the GPU tests compare bit for bit.

Every value comes from the CPU oracle (``oracle.sw_coords_mt``, the banded
threaded form of the oracle's local pass, itself checked against the plain
single-threaded pass by the CPU tests) on inputs from ``seqgen``; nothing here
touches the GPU library.  Run from the repository root:

    python tests/golden/make_long_pairs.py [--threads T] [--only NAME]

Pairs:
  long_pair_500k  -- the long-pair workload at 500,000 bp with 5,000 bp flanks
                     (+1/-3, open 5, extend 2), about 2.5e11 cells per pass
  high_score_528k -- a 528,000 bp related pair scored +127/-127, open 200,
                     extend 50, whose score (about 6.6e7) sits just below the
                     2^26 limit on min(n, m) * max|s|
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import seqgen  # noqa: E402

OUT = os.path.join(HERE, "long_pairs.json")

PAIRS = {
    "long_pair_500k": dict(generator="workload1", args=dict(n=500_000, flank=5_000), scoring="dna"),
    "high_score_528k": dict(generator="workload1_high", args=dict(n=528_000, flank=5_000), scoring="high_score_dna"),
}


def inputs(spec):
    q, t = getattr(seqgen, spec["generator"])(**spec["args"])
    sc = seqgen.dna_scoring() if spec["scoring"] == "dna" else seqgen.high_score_dna_scoring()
    return q, t, sc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", default=None)
    args = ap.parse_args()
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name, spec in PAIRS.items():
        if args.only and name != args.only:
            continue
        q, t, sc = inputs(spec)
        t0 = time.time()
        res = oracle.sw_coords_mt(bytes(q), bytes(t), sc, threads=args.threads)
        dt = time.time() - t0
        data[name] = dict(spec, query_len=len(q), target_len=len(t), **res,
                          oracle="sw_coords_mt", threads=args.threads, seconds=round(dt, 1))
        print(name, res, f"{dt:.0f} s", flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main()
