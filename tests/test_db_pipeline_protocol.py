"""Host-side model of the hand-over protocol of the pipelined database kernel
(several waves share one (query, group) unit, each taking every W-th 32-row
chunk of the query; a chunk's bottom row reaches the next chunk through a
small LDS ring between neighbouring waves, or through a ring in global
memory from the last wave back to the first).

The kernel's waits (ring data, ring space, unit-table publication and reuse)
are written out here as predicates over the same counters and the waves are
interleaved at random, one atomic step at a time.  The model checks that no
interleaving blocks every wave (the kernel's bounded waits would otherwise
expire) and that every chunk reads exactly the row its predecessor chunk
wrote, for any mix of unit lengths -- including units of one chunk, where a
wave can run many units ahead of its neighbours.
"""
import random

import pytest

RING = 8          # columns per LDS ring
TABLE = 32        # unit-table entries
PUB_LDS = 2       # an LDS producer publishes every 2 columns
PUB_WRAP = 16     # the wrap producer publishes every 16 columns


class Shared:
    def __init__(self, W, units, capg):
        self.W = W
        self.units = units            # [(nc, L)] in ticket order
        self.capg = capg
        self.ticket = 0
        self.prod = [0] * W
        self.cons = [0] * W
        self.wave_unit = [0] * W
        self.table = [None] * TABLE
        self.npub = 0
        self.ring = {}                # (ring id, slot) -> (unit, chunk, column)
        self.reads = []


def wave(sh, w):
    W = sh.W
    G, u, ug0, unc, uw = w, -1, 0, 0, 0
    in_seq = out_seq = 0
    inr = (w + W - 1) % W
    cap_out = sh.capg if w == W - 1 else RING
    cap_in = sh.capg if w == 0 else RING
    while True:
        while u < 0 or G >= ug0 + unc:
            nu = u + 1
            start = 0 if u < 0 else ug0 + unc
            if sh.npub > nu:
                e = sh.table[nu % TABLE]
                assert e[0] == nu
                u, uw, ug0, unc = nu, e[1], e[2], e[3]
                sh.wave_unit[w] = nu
                continue
            if G == start:
                tv = sh.ticket
                sh.ticket += 1
                work = tv if tv < len(sh.units) else -1
                nc = sh.units[work][0] if work >= 0 else 1 << 30
                yield lambda nu=nu: min(sh.wave_unit) >= nu - TABLE + 1
                sh.table[nu % TABLE] = (nu, work, start, nc)
                sh.npub = nu + 1
                continue
            yield lambda nu=nu: sh.npub > nu
        if uw < 0:
            return
        c = G - ug0
        nc, L = sh.units[uw]
        has_in, has_out = c > 0, c < nc - 1
        in_base, out_base = in_seq, out_seq
        nxt = None
        if has_in and L > 0:      # a group of empty sequences hands over no columns
            yield lambda: sh.prod[inr] >= in_base + 1
            nxt = sh.ring[(inr, in_base % cap_in)]
        for j in range(L):
            top = nxt
            if has_in and j + 1 < L:
                yield lambda j=j: sh.prod[inr] >= in_base + j + 2
                nxt = sh.ring[(inr, (in_base + j + 1) % cap_in)]
            if has_in:
                assert top == (uw, c - 1, j), (top, uw, c, j)
                sh.reads.append(top)
            if has_out:
                seq = out_base + j
                yield lambda seq=seq: seq - sh.cons[w] < cap_out
                sh.ring[(w, seq % cap_out)] = (uw, c, j)
                pub = PUB_WRAP if w == W - 1 else PUB_LDS
                if (j % pub) == pub - 1 or j == L - 1:
                    sh.prod[w] = seq + 1
            if has_in and ((j & 1) or j == L - 1):
                sh.cons[inr] = in_base + j + 1
            yield None
        if has_in:
            in_seq += L
        if has_out:
            out_seq += L
        G += W


def run(W, units, seed, capg):
    sh = Shared(W, units, capg)
    gens = {w: wave(sh, w) for w in range(W)}
    pending = {w: None for w in range(W)}
    rng = random.Random(seed)
    steps = 0
    while gens:
        ready = [w for w in gens if pending[w] is None or pending[w]()]
        assert ready, f"all waves blocked after {steps} steps"
        w = rng.choice(ready)
        try:
            pending[w] = next(gens[w])
        except StopIteration:
            del gens[w]
        steps += 1
    want = sum((nc - 1) * L for nc, L in units)
    assert len(sh.reads) == want
    return steps


@pytest.mark.parametrize("W", [2, 4, 8, 16])
@pytest.mark.parametrize("seed", range(6))
def test_random_interleavings_never_block_and_rows_match(W, seed):
    rng = random.Random(100 * W + seed)
    units = []
    for _ in range(rng.randint(1, 40)):
        kind = rng.random()
        nc = 1 if kind < 0.3 else rng.randint(1, 3 * W + 2)
        L = rng.choice([0, 1, 2, 3, rng.randint(1, 40)])
        units.append((nc, L))
    maxlen = max(1, max(L for _, L in units))
    run(W, units, seed, capg=maxlen + 64)


def test_single_chunk_units_let_waves_drift_without_overrunning_the_table():
    # 200 one-chunk units: no hand-over at all, only the unit table constrains
    # how far one wave can run ahead
    units = [(1, 1 + (i % 5)) for i in range(200)]
    for seed in range(4):
        run(4, units, seed, capg=70)


def test_long_units_use_the_wrap_ring():
    units = [(9, 50), (1, 3), (7, 64), (4, 2)]
    for seed in range(4):
        run(4, units, seed, capg=64 + 64)


def test_model_reports_a_wrap_ring_shorter_than_a_row():
    # the check is live: a global ring that cannot hold one chunk row blocks
    # (the first chunk of a round waits on a consumer still a round behind)
    with pytest.raises(AssertionError):
        for seed in range(10):
            run(4, [(9, 50), (7, 64)], seed, capg=3)
