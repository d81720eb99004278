"""Seeded synthetic inputs shaped like the paper's workloads.

This module is shared by the GPU tests/bench and by the oracle tests.  It holds
no alignment arithmetic at all: only random sequence generation, the scoring
*data* (substitution tables, gap values) and byte-level helpers.  Everything
is drawn from ``numpy.random.Generator(PCG64(seed))`` with

    seed = 221110769 + 1000 * workload + stream
    streams: 0 queries / query, 1 database / target, 2 mutations,
             3 planting positions, 4 training pairs, 5 audit sample

Workloads (the paper's data sets are public downloads that are not available
here; these stand in for them with the same shapes):

  0  two uniform ACGT sequences of 10,000 bp; +1/-3, open 5, extend 2
  1  uniform ACGT query of 5,000,000 bp; target = copy with 2% substitutions
     and 0.5% indel events (geometric length, mean 3) plus 50 kbp random
     flanks on both sides (stands in for the paper's 5 Mbp x 5 Mbp pair)
  2  20 protein queries (log-uniform 100..5,000 aa) vs 500,000 proteins with
     lognormal lengths (median 300, sigma 0.607, clipped 25..35,000),
     residues i.i.d. from background frequencies; BLOSUM62, open 10, extend 2
  3  same queries vs 2,000,000 proteins with 50 mutated homologs per query
     planted (30..90% identity, 5% indels), plus training pairs
  4  200,000 read/reference DNA pairs, reads log-uniform 150..20,000 bp,
     reference = read mutated at 1..15% divergence inside a random window of
     1.2x its length
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 221110769

DNA_ALPHABET = "ACGT"
DNA_MATRIX = np.array([[1 if i == j else -3 for j in range(4)] for i in range(4)], dtype=np.int8)
DNA_GAP_OPEN, DNA_GAP_EXTEND = 5, 2

PROTEIN_ALPHABET = "ARNDCQEGHILKMFPSTWYVBZX*"

# BLOSUM62 (Henikoff & Henikoff, PNAS 1992), rows/columns in PROTEIN_ALPHABET order.
_B62 = """
 4 -1 -2 -2  0 -1 -1  0 -2 -1 -1 -1 -1 -2 -1  1  0 -3 -2  0 -2 -1  0 -4
-1  5  0 -2 -3  1  0 -2  0 -3 -2  2 -1 -3 -2 -1 -1 -3 -2 -3 -1  0 -1 -4
-2  0  6  1 -3  0  0  0  1 -3 -3  0 -2 -3 -2  1  0 -4 -2 -3  3  0 -1 -4
-2 -2  1  6 -3  0  2 -1 -1 -3 -4 -1 -3 -3 -1  0 -1 -4 -3 -3  4  1 -1 -4
 0 -3 -3 -3  9 -3 -4 -3 -3 -1 -1 -3 -1 -2 -3 -1 -1 -2 -2 -1 -3 -3 -2 -4
-1  1  0  0 -3  5  2 -2  0 -3 -2  1  0 -3 -1  0 -1 -2 -1 -2  0  3 -1 -4
-1  0  0  2 -4  2  5 -2  0 -3 -3  1 -2 -3 -1  0 -1 -3 -2 -2  1  4 -1 -4
 0 -2  0 -1 -3 -2 -2  6 -2 -4 -4 -2 -3 -3 -2  0 -2 -2 -3 -3 -1 -2 -1 -4
-2  0  1 -1 -3  0  0 -2  8 -3 -3 -1 -2 -1 -2 -1 -2 -2  2 -3  0  0 -1 -4
-1 -3 -3 -3 -1 -3 -3 -4 -3  4  2 -3  1  0 -3 -2 -1 -3 -1  3 -3 -3 -1 -4
-1 -2 -3 -4 -1 -2 -3 -4 -3  2  4 -2  2  0 -3 -2 -1 -2 -1  1 -4 -3 -1 -4
-1  2  0 -1 -3  1  1 -2 -1 -3 -2  5 -1 -3 -1  0 -1 -3 -2 -2  0  1 -1 -4
-1 -1 -2 -3 -1  0 -2 -3 -2  1  2 -1  5  0 -2 -1 -1 -1 -1  1 -3 -1 -1 -4
-2 -3 -3 -3 -2 -3 -3 -3 -1  0  0 -3  0  6 -4 -2 -2  1  3 -1 -3 -3 -1 -4
-1 -2 -2 -1 -3 -1 -1 -2 -2 -3 -3 -1 -2 -4  7 -1 -1 -4 -3 -2 -2 -1 -2 -4
 1 -1  1  0 -1  0  0  0 -1 -2 -2  0 -1 -2 -1  4  1 -3 -2 -2  0  0  0 -4
 0 -1  0 -1 -1 -1 -1 -2 -2 -1 -1 -1 -1 -2 -1  1  5 -2 -2  0 -1 -1  0 -4
-3 -3 -4 -4 -2 -2 -3 -2 -2 -3 -2 -3 -1  1 -4 -3 -2 11  2 -3 -4 -3 -2 -4
-2 -2 -2 -3 -2 -1 -2 -3  2 -1 -1 -2 -1  3 -3 -2 -2  2  7 -1 -3 -2 -1 -4
 0 -3 -3 -3 -1 -2 -2 -3 -3  3  1 -2  1 -1 -2 -2  0 -3 -1  4 -3 -2 -1 -4
-2 -1  3  4 -3  0  1 -1  0 -3 -4  0 -3 -3 -2  0 -1 -4 -3 -3  4  1 -1 -4
-1  0  0  1 -3  3  4 -2  0 -3 -3  1 -1 -3 -1  0 -1 -3 -2 -2  1  4 -1 -4
 0 -1 -1 -1 -2 -1 -1 -1 -1 -1 -1 -1 -1 -1 -2  0  0 -2 -1 -1 -1 -1 -1 -4
-4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4  1
"""
BLOSUM62 = np.array([[int(x) for x in line.split()] for line in _B62.strip().splitlines()],
                    dtype=np.int8)
PROTEIN_GAP_OPEN, PROTEIN_GAP_EXTEND = 10, 2

# BLOSUM50 and BLOSUM45 (Henikoff & Henikoff, PNAS 1992; both in 1/3-bit
# units) over the 20 standard residues only, in PROTEIN_ALPHABET[:20] order:
# the protein generators emit no ambiguity codes.
_B50 = """
 5 -2 -1 -2 -1 -1 -1  0 -2 -1 -2 -1 -1 -3 -1  1  0 -3 -2  0
-2  7 -1 -2 -4  1  0 -3  0 -4 -3  3 -2 -3 -3 -1 -1 -3 -1 -3
-1 -1  7  2 -2  0  0  0  1 -3 -4  0 -2 -4 -2  1  0 -4 -2 -3
-2 -2  2  8 -4  0  2 -1 -1 -4 -4 -1 -4 -5 -1  0 -1 -5 -3 -4
-1 -4 -2 -4 13 -3 -3 -3 -3 -2 -2 -3 -2 -2 -4 -1 -1 -5 -3 -1
-1  1  0  0 -3  7  2 -2  1 -3 -2  2  0 -4 -1  0 -1 -1 -1 -3
-1  0  0  2 -3  2  6 -3  0 -4 -3  1 -2 -3 -1 -1 -1 -3 -2 -3
 0 -3  0 -1 -3 -2 -3  8 -2 -4 -4 -2 -3 -4 -2  0 -2 -3 -3 -4
-2  0  1 -1 -3  1  0 -2 10 -4 -3  0 -1 -1 -2 -1 -2 -3  2 -4
-1 -4 -3 -4 -2 -3 -4 -4 -4  5  2 -3  2  0 -3 -3 -1 -3 -1  4
-2 -3 -4 -4 -2 -2 -3 -4 -3  2  5 -3  3  1 -4 -3 -1 -2 -1  1
-1  3  0 -1 -3  2  1 -2  0 -3 -3  6 -2 -4 -1  0 -1 -3 -2 -3
-1 -2 -2 -4 -2  0 -2 -3 -1  2  3 -2  7  0 -3 -2 -1 -1  0  1
-3 -3 -4 -5 -2 -4 -3 -4 -1  0  1 -4  0  8 -4 -3 -2  1  4 -1
-1 -3 -2 -1 -4 -1 -1 -2 -2 -3 -4 -1 -3 -4 10 -1 -1 -4 -3 -3
 1 -1  1  0 -1  0 -1  0 -1 -3 -3  0 -2 -3 -1  5  2 -4 -2 -2
 0 -1  0 -1 -1 -1 -1 -2 -2 -1 -1 -1 -1 -2 -1  2  5 -3 -2  0
-3 -3 -4 -5 -5 -1 -3 -3 -3 -3 -2 -3 -1  1 -4 -4 -3 15  2 -3
-2 -1 -2 -3 -3 -1 -2 -3  2 -1 -1 -2  0  4 -3 -2 -2  2  8 -1
 0 -3 -3 -4 -1 -3 -3 -4 -4  4  1 -3  1 -1 -3 -2  0 -3 -1  5
"""
_B45 = """
 5 -2 -1 -2 -1 -1 -1  0 -2 -1 -1 -1 -1 -2 -1  1  0 -2 -2  0
-2  7  0 -1 -3  1  0 -2  0 -3 -2  3 -1 -2 -2 -1 -1 -2 -1 -2
-1  0  6  2 -2  0  0  0  1 -2 -3  0 -2 -2 -2  1  0 -4 -2 -3
-2 -1  2  7 -3  0  2 -1  0 -4 -3  0 -3 -4 -1  0 -1 -4 -2 -3
-1 -3 -2 -3 12 -3 -3 -3 -3 -3 -2 -3 -2 -2 -4 -1 -1 -5 -3 -1
-1  1  0  0 -3  6  2 -2  1 -2 -2  1  0 -4 -1  0 -1 -2 -1 -3
-1  0  0  2 -3  2  6 -2  0 -3 -2  1 -2 -3  0  0 -1 -3 -2 -3
 0 -2  0 -1 -3 -2 -2  7 -2 -4 -3 -2 -2 -3 -2  0 -2 -2 -3 -3
-2  0  1  0 -3  1  0 -2 10 -3 -2 -1  0 -2 -2 -1 -2 -3  2 -3
-1 -3 -2 -4 -3 -2 -3 -4 -3  5  2 -3  2  0 -2 -2 -1 -2  0  3
-1 -2 -3 -3 -2 -2 -2 -3 -2  2  5 -3  2  1 -3 -3 -1 -2  0  1
-1  3  0  0 -3  1  1 -2 -1 -3 -3  5 -1 -3 -1 -1 -1 -2 -1 -2
-1 -1 -2 -3 -2  0 -2 -2  0  2  2 -1  6  0 -2 -2 -1 -2  0  1
-2 -2 -2 -4 -2 -4 -3 -3 -2  0  1 -3  0  8 -3 -2 -1  1  3  0
-1 -2 -2 -1 -4 -1  0 -2 -2 -2 -3 -1 -2 -3  9 -1 -1 -3 -3 -3
 1 -1  1  0 -1  0  0  0 -1 -2 -3 -1 -2 -2 -1  4  2 -4 -2 -1
 0 -1  0 -1 -1 -1 -1 -2 -2 -1 -1 -1 -1 -1 -1  2  5 -3 -1  0
-2 -2 -4 -4 -5 -2 -3 -2 -3 -2 -2 -2 -2  1 -3 -4 -3 15  3 -3
-2 -1 -2 -2 -3 -1 -2 -3  2  0  0 -1  0  3 -3 -2 -1  3  8 -1
 0 -2 -3 -3 -1 -3 -3 -3 -3  3  1 -2  1  0 -3 -1  0 -3 -1  5
"""
BLOSUM50 = np.array([[int(x) for x in line.split()] for line in _B50.strip().splitlines()], dtype=np.int8)
BLOSUM45 = np.array([[int(x) for x in line.split()] for line in _B45.strip().splitlines()], dtype=np.int8)

# Background amino-acid frequencies (Robinson & Robinson, PNAS 1991) for the
# 20 standard residues, in PROTEIN_ALPHABET order (A R N D C Q E G H I L K M F
# P S T W Y V); renormalised to sum to one.
_BG_RAW = np.array([0.07805, 0.05129, 0.04487, 0.05364, 0.01925, 0.04264, 0.06295, 0.07377,
                    0.02199, 0.05142, 0.09019, 0.05744, 0.02243, 0.03856, 0.05203, 0.07120,
                    0.05841, 0.01330, 0.03216, 0.06441])
BACKGROUND = _BG_RAW / _BG_RAW.sum()

_DNA_BYTES = np.frombuffer(DNA_ALPHABET.encode(), dtype=np.uint8)
_AA_BYTES = np.frombuffer(PROTEIN_ALPHABET[:20].encode(), dtype=np.uint8)


def dna_scoring():
    """(alphabet, matrix, gap_open, gap_extend) for the DNA workloads."""
    return DNA_ALPHABET, DNA_MATRIX, DNA_GAP_OPEN, DNA_GAP_EXTEND


def protein_scoring():
    """(alphabet, matrix, gap_open, gap_extend) for the protein workloads."""
    return PROTEIN_ALPHABET, BLOSUM62, PROTEIN_GAP_OPEN, PROTEIN_GAP_EXTEND


def blosum_scoring(which: int, gap_open: int = PROTEIN_GAP_OPEN, gap_extend: int = PROTEIN_GAP_EXTEND):
    """(alphabet, matrix, gap_open, gap_extend) with BLOSUM62, 50 or 45 over the
    20 standard residues."""
    m = {62: BLOSUM62[:20, :20], 50: BLOSUM50, 45: BLOSUM45}[which]
    return PROTEIN_ALPHABET[:20], np.ascontiguousarray(m), gap_open, gap_extend


def rng_for(workload: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + 1000 * workload + stream))


# ---------------------------------------------------------------- residues

def random_dna(rng: np.random.Generator, n: int) -> np.ndarray:
    """n uniform ACGT bytes (ASCII) as uint8."""
    return _DNA_BYTES[rng.integers(0, 4, size=n)]


def random_protein(rng: np.random.Generator, n: int) -> np.ndarray:
    """n residues i.i.d. from the background frequencies, ASCII uint8."""
    return _AA_BYTES[rng.choice(20, size=n, p=BACKGROUND)]


def _substitute(rng, seq: np.ndarray, mask: np.ndarray, protein: bool) -> None:
    """Replace seq[mask] by a different residue (uniform for DNA, background for protein)."""
    k = int(mask.sum())
    if k == 0:
        return
    if protein:
        new = random_protein(rng, k)
        same = new == seq[mask]
        while same.any():
            new[same] = random_protein(rng, int(same.sum()))
            same = new == seq[mask]
    else:
        cur = np.searchsorted(_DNA_BYTES, seq[mask])   # ACGT is sorted
        new = _DNA_BYTES[(cur + rng.integers(1, 4, size=k)) % 4]
    seq[mask] = new


def mutate(rng: np.random.Generator, src: np.ndarray, p_sub: float, p_indel: float,
           protein: bool = False, mean_indel: float = 3.0) -> np.ndarray:
    """Copy of src with substitutions and indel events.

    Per position: substitution with probability p_sub; an indel event with
    probability p_indel, half insertions (random residues after the position)
    and half deletions (starting at the position), length ~ Geometric(1/mean)
    on {1, 2, ...}.
    """
    n = len(src)
    out = src.copy()
    u = rng.random(n)
    sub = u < p_sub
    _substitute(rng, out, sub, protein)
    ev = (u >= p_sub) & (u < p_sub + p_indel)
    pos = np.nonzero(ev)[0]
    lens = rng.geometric(1.0 / mean_indel, size=len(pos))
    is_ins = rng.random(len(pos)) < 0.5
    # deletions: mark removed ranges with a difference array
    diff = np.zeros(n + 1, dtype=np.int64)
    dpos, dlen = pos[~is_ins], lens[~is_ins]
    np.add.at(diff, dpos, 1)
    np.add.at(diff, np.minimum(dpos + dlen, n), -1)
    keep = np.cumsum(diff[:n]) == 0
    ins = np.zeros(n, dtype=np.int64)
    ins[pos[is_ins]] = lens[is_ins]
    counts = keep.astype(np.int64) + ins
    total = int(counts.sum())
    res = random_protein(rng, total) if protein else random_dna(rng, total)
    start = np.cumsum(counts) - counts
    res[start[keep]] = out[keep]
    return res


# ---------------------------------------------------------------- workloads

def workload0(n: int = 10_000, m: int = 10_000):
    """Pairwise DNA: (query, target) uniform ACGT."""
    return random_dna(rng_for(0, 0), n), random_dna(rng_for(0, 1), m)


def workload1(n: int = 5_000_000, flank: int = 50_000):
    """Long pairwise DNA: query and its mutated copy between random flanks."""
    q = random_dna(rng_for(1, 0), n)
    core = mutate(rng_for(1, 2), q, 0.02, 0.005)
    fr = rng_for(1, 1)
    t = np.concatenate([random_dna(fr, flank), core, random_dna(fr, flank)])
    return q, t


def high_score_dna_scoring():
    """DNA scoring with the extreme int8 scores (match +127, mismatch -127),
    gap open 200, extend 50: a related pair scores about 125 per base, so a
    pair of half a megabase reaches scores near 2^26."""
    m = np.full((4, 4), -127, dtype=np.int8)
    np.fill_diagonal(m, 127)
    return DNA_ALPHABET, m, 200, 50


def workload1_high(n: int = 528_000, flank: int = 5_000):
    """A related DNA pair for the high-score range: a uniform query and its
    copy with 1% substitutions and 0.2% indel events (geometric, mean 3)
    between random flanks (seed streams 10-12 of the long-pair workload, apart
    from the ones workload1 uses)."""
    q = random_dna(rng_for(1, 10), n)
    core = mutate(rng_for(1, 12), q, 0.01, 0.002)
    fr = rng_for(1, 11)
    t = np.concatenate([random_dna(fr, flank), core, random_dna(fr, flank)])
    return q, t


def query_lengths(rng, count: int = 20, lo: int = 100, hi: int = 5000) -> np.ndarray:
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)


def queries(count: int = 20, workload: int = 2):
    rng = rng_for(workload, 0)
    lens = query_lengths(rng, count)
    return [random_protein(rng, int(L)) for L in lens]


def db_lengths(rng, count: int, median: float = 300.0, sigma: float = 0.607,
               lo: int = 25, hi: int = 35_000) -> np.ndarray:
    L = np.rint(rng.lognormal(math.log(median), sigma, size=count)).astype(np.int64)
    return np.clip(L, lo, hi)


def protein_db(count: int, workload: int = 2):
    """(concatenated ASCII residues as uint8, int64 offsets)."""
    rng = rng_for(workload, 1)
    lens = db_lengths(rng, count)
    off = np.zeros(count + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    return random_protein(rng, int(off[-1])), off


def workload2(n_db: int = 500_000, n_queries: int = 20):
    return queries(n_queries, 2), protein_db(n_db, 2)


def homolog(rng, q: np.ndarray) -> np.ndarray:
    """Mutated copy at identity ~ U(0.30, 0.90) with ~5% of positions in indels."""
    ident = rng.uniform(0.30, 0.90)
    return mutate(rng, q, 1.0 - ident, 0.05 / 3.0, protein=True)


def workload3(n_db: int = 2_000_000, n_queries: int = 20, per_query: int = 50):
    """Queries, db with planted homologs, and the planted (query, db index) list."""
    qs = queries(n_queries, 2)
    cat, off = protein_db(n_db, 3)
    prng, mrng = rng_for(3, 3), rng_for(3, 2)
    where = prng.choice(n_db, size=n_queries * per_query, replace=False)
    seqs = {int(idx): homolog(mrng, qs[k // per_query]) for k, idx in enumerate(where)}
    # rebuild the concatenation with the planted sequences in place
    lens = np.diff(off).copy()
    for idx, h in seqs.items():
        lens[idx] = len(h)
    noff = np.zeros(n_db + 1, dtype=np.int64)
    noff[1:] = np.cumsum(lens)
    pieces, prev = [], 0
    for idx in sorted(seqs):
        pieces.append(cat[off[prev]:off[idx]])
        pieces.append(seqs[idx])
        prev = idx + 1
    pieces.append(cat[off[prev]:off[n_db]])
    ncat = np.concatenate(pieces)
    pairs = [(k // per_query, int(idx)) for k, idx in enumerate(where)]
    return qs, (ncat, noff), pairs


def training_pairs(count: int, workload: int = 3):
    """Half unrelated, half related (query-like x db-like lengths) protein pairs."""
    rng = rng_for(workload, 4)
    qs, ts = [], []
    for k in range(count):
        Lq = int(query_lengths(rng, 1)[0])
        q = random_protein(rng, Lq)
        if k % 2 == 0:
            t = random_protein(rng, int(db_lengths(rng, 1)[0]))
        else:
            t = homolog(rng, q)
        qs.append(q)
        ts.append(t)
    return qs, ts


def _concat_pool(seqs):
    off = np.zeros(len(seqs) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(x) for x in seqs])
    return np.concatenate(seqs) if seqs else np.zeros(0, np.uint8), off


def prefilter_training_set(n_pairs: int = 1_000_000, n_queries: int = 2_000, homologs: int = 25,
                           n_background: int = 100_000, workload: int = 3):
    """Labelled-pair inputs for the prefilter network: a sequence pool and
    (row, column) index pairs into it, half unrelated and half related.

    Pool: n_queries query-like sequences (log-uniform 100..5,000), for each
    `homologs` mutated copies (identity U(0.30, 0.90), 5% of positions in
    indels), and n_background database-like sequences (the db length law).
    Unrelated pairs: a query-like row against a background column.  Related
    pairs: two distinct members of one family (the query and its copies),
    drawn without repetition while the families hold enough pairs.  Seed streams are disjoint from the evaluation
    queries and database.
    """
    rng = rng_for(workload, 4)
    qlen = query_lengths(rng, n_queries)
    qres = random_protein(rng, int(qlen.sum()))
    qoff = np.concatenate([[0], np.cumsum(qlen)])
    qseqs = [qres[qoff[i]:qoff[i + 1]] for i in range(n_queries)]
    hseqs = [homolog(rng, q) for q in qseqs for _ in range(homologs)]
    blen = db_lengths(rng, n_background)
    bres = random_protein(rng, int(blen.sum()))
    boff = np.concatenate([[0], np.cumsum(blen)])
    bseqs = [bres[boff[i]:boff[i + 1]] for i in range(n_background)]
    cat, off = _concat_pool(qseqs + hseqs + bseqs)
    h0, b0 = n_queries, n_queries + n_queries * homologs
    n_unrel = n_pairs // 2
    n_rel = n_pairs - n_unrel
    ur = rng.integers(0, n_queries, size=n_unrel)
    uc = b0 + rng.integers(0, n_background, size=n_unrel)
    # family f: member 0 = query f, members 1..homologs = its copies
    fam = homologs + 1
    npf = fam * (fam - 1) // 2
    pick = rng.choice(n_queries * npf, size=n_rel, replace=n_rel > n_queries * npf)
    f, w = pick // npf, pick % npf
    iu, ju = np.triu_indices(fam, k=1)
    a, b = iu[w], ju[w]
    member = lambda fi, k: np.where(k == 0, fi, h0 + fi * homologs + (k - 1))
    rr, rc = member(f, a), member(f, b)
    rows = np.concatenate([ur, rr]).astype(np.int32)
    cols = np.concatenate([uc, rc]).astype(np.int32)
    perm = rng.permutation(n_pairs)
    return cat, off, rows[perm], cols[perm]


def read_pair(rng, L: int) -> tuple[np.ndarray, np.ndarray]:
    read = random_dna(rng, L)
    d = rng.uniform(0.01, 0.15)
    core = mutate(rng, read, 0.8 * d, 0.2 * d)
    total = int(round(1.2 * L))
    pad = max(total - len(core), 0)
    left = int(rng.integers(0, pad + 1))
    ref = np.concatenate([random_dna(rng, left), core, random_dna(rng, pad - left)])
    return read, ref


def workload4(n_pairs: int = 200_000, lo: int = 150, hi: int = 20_000):
    """Batched uneven DNA pairs: list of (read, reference)."""
    rng = rng_for(4, 0)
    lens = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_pairs))).astype(np.int64)
    mrng = rng_for(4, 2)
    return [read_pair(mrng, int(L)) for L in lens]


def to_str(x) -> str:
    return bytes(np.asarray(x, dtype=np.uint8)).decode("ascii")
