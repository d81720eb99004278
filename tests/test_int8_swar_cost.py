"""Cost of a packed 8-bit Gotoh cell on a GPU that has no packed 8-bit
arithmetic (the int8 database search the paper lists as future work, Sec. 5).

CDNA4's vector ALU packs two 16-bit lanes per 32-bit register (add, subtract
and max with saturation, one instruction each) but has no 4 x 8-bit add, max
or saturation.  Four cells per register therefore need SWAR sequences of
32-bit logic and adds.  This file writes those sequences out (unsigned bytes
with a bias, the usual form for 8-bit Smith-Waterman), checks them against
per-byte scalar arithmetic, counts their 32-bit operations, and compares the
cost of one cell with the packed 16-bit and 32-bit kernels (about 10
operations per lane step: 5 per cell in 16 bits, 10 in 32 bits).  It is a
host-side design check; no GPU code follows it.
"""
import numpy as np

M7 = np.uint32(0x7F7F7F7F)
M8 = np.uint32(0x80808080)


class Ops:
    """Counts 32-bit vector operations; three-input forms that gfx9 has
    (v_and_or_b32, v_or3_b32, v_bfi_b32, v_add3_u32, v_lshl_or_b32) count once."""

    def __init__(self):
        self.n = 0

    def __call__(self, k=1):
        self.n += k


def sat_add(a, b, op):
    # per byte min(a + b, 255)
    t = (a & M7) + (b & M7); op(3)           # 2 ands + add
    r = t ^ ((a ^ b) & M8); op(3)            # xor, and, xor
    c = ((a & b) | ((a | b) & ~r)) & M8; op(4)   # and_or, or, andn(not folded), and
    m = (c >> np.uint32(7)) * np.uint32(0xFF); op(2)   # carry byte -> 0xFF mask
    return r | m, op(1)


def sat_sub(a, b, op):
    # per byte max(a - b, 0)
    t = (a | M8) - (b & M7); op(3)           # or, and, sub
    r = t ^ ((a ^ ~b) & M8); op(3)           # xnor, and, xor
    bw = ((~a & b) | ((~a | b) & r)) & M8; op(4)  # borrow out of bit 7
    m = (bw >> np.uint32(7)) * np.uint32(0xFF); op(2)
    return r & ~m, op(1)


def umax(a, b, op):
    # per byte max(a, b) = b + sat_sub(a, b): the sum cannot overflow
    d, _ = sat_sub(a, b, op)
    return b + d, op(1)


def _bytes(x):
    return np.stack([(x >> np.uint32(8 * k)) & np.uint32(0xFF) for k in range(4)]).astype(np.int64)


def test_swar_sequences_equal_per_byte_arithmetic():
    rng = np.random.default_rng(8)
    a = rng.integers(0, 2 ** 32, 20000, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 2 ** 32, 20000, dtype=np.uint64).astype(np.uint32)
    op = Ops()
    s, _ = sat_add(a, b, op)
    d, _ = sat_sub(a, b, op)
    m, _ = umax(a, b, op)
    A, B = _bytes(a), _bytes(b)
    assert (_bytes(s) == np.minimum(A + B, 255)).all()
    assert (_bytes(d) == np.maximum(A - B, 0)).all()
    assert (_bytes(m) == np.maximum(A, B)).all()


def gotoh_cell_ops():
    """32-bit operations for one SWAR step of four local Gotoh cells in biased
    unsigned bytes: H = max(Hdiag + s, E, F) (the zero floor is free in
    unsigned form, the bias is folded into the profile), E and F each
    max(prev - e, H - o), and the running maximum."""
    op = Ops()
    x = np.uint32(0x12345678)
    hd, _ = sat_add(x, x, op)      # diagonal + substitution (profile holds s + bias)
    hd, _ = sat_sub(hd, x, op)     # remove the bias
    h, _ = umax(hd, x, op)         # with E
    h, _ = umax(h, x, op)          # with F
    e1, _ = sat_sub(x, x, op)      # E - e
    e2, _ = sat_sub(h, x, op)      # H - o
    e, _ = umax(e1, e2, op)
    f1, _ = sat_sub(x, x, op)      # F - e
    f2, _ = sat_sub(h, x, op)      # H - o
    f, _ = umax(f1, f2, op)
    best, _ = umax(h, x, op)       # running maximum
    return op.n


def test_packed_int8_cell_costs_more_than_packed_int16():
    per_word = gotoh_cell_ops()
    per_cell_int8 = per_word / 4
    per_cell_int16 = 10 / 2
    per_cell_int32 = 10 / 1
    # the SWAR cell costs more than a 16-bit cell and even more than a 32-bit one
    assert per_word == 148      # 37 operations per cell
    assert per_cell_int8 > 2 * per_cell_int16 and per_cell_int8 > per_cell_int32
