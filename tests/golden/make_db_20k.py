"""Write tests/golden/db_20k_scores.npz: every local score of the 20 database
queries against 20,000 proteins, which the GPU tests compare bit for bit.

Every value comes from the CPU oracle (``oracle.db_scores``, the oracle's
plain Gotoh local pass per pair, threaded over pairs) on inputs from
``seqgen.workload2(n_db=20_000, n_queries=20)`` scored with BLOSUM62, gap open
10, extend 2; nothing here touches the GPU library.  About 2.3e11 cells: a few
minutes on eight threads.  Run from the repository root:

    python tests/golden/make_db_20k.py
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import seqgen  # noqa: E402

OUT = os.path.join(HERE, "db_20k_scores.npz")
N_DB, N_QUERIES = 20_000, 20


def main() -> None:
    qs, (cat, off) = seqgen.workload2(n_db=N_DB, n_queries=N_QUERIES)
    sc = seqgen.protein_scoring()
    t0 = time.time()
    scores = oracle.db_scores([bytes(q) for q in qs], (cat, off), sc)
    dt = time.time() - t0
    if scores.min() < 0 or scores.max() >= 2 ** 31:
        raise SystemExit("scores out of int32 range")
    np.savez_compressed(OUT, scores=scores.astype(np.int32),
                        query_lengths=np.array([len(q) for q in qs], dtype=np.int64),
                        db_residues=np.int64(off[-1] - off[0]))
    cells = sum(len(q) for q in qs) * int(off[-1] - off[0])
    print(f"wrote {OUT}: {scores.shape}, {cells:.3e} cells in {dt:.0f} s")


if __name__ == "__main__":
    main()
