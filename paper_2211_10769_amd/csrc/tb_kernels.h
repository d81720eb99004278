// tb_kernels.h -- device-side descriptors of the traceback kernels
// (tb_kernels.hip), shared with the host driver (traceback.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "engine.h"

namespace swh {

// dst[i] = i < first_pad ? pad : src[start + step * (i - first_pad)] for
// i - first_pad < count; pad up to padded.
struct GatherDesc {
    const uint8_t *src;
    uint8_t *dst;
    int64_t start;
    int64_t count;
    int64_t padded;
    int32_t step;        // +1 or -1
    int32_t first_pad;   // pad codes before the copy (the copy starts at dst[first_pad])
};

// Top row of one DP pass.  kind 0: copy count entries from src;
// kind 1: backward pass whose end is an H cell: G'(c) = c ? -o-(c-1)e : 0,
//         D'(c) = G'(c) - o;
// kind 2: backward pass whose end is an F cell: G' = -inf, D'(0) = -o,
//         D'(c>0) = -inf;
// kind 3: a single frontier node: entry 0 = (seed_h, seed_f), the rest -inf;
// kind 4: free leading target residues: G'(c) = 0, D'(c) = -o for every c.
// Entries from count to padded are (-inf, -inf).
struct BorderInit {
    Border *dst;
    const Border *src;
    int64_t count;
    int64_t padded;
    int32_t kind;
    int32_t seed_h, seed_f;
    int32_t pad_;
};

// Crossing scan of one split at mid row r (see traceback.cpp).
struct CrossDesc {
    const Border *fwd;      // fwd[k]: G(r, L+k), D(L+k) = F(r+1, L+k)
    const Border *bwd;      // bwd[k]: G'(row r+1 of the reversed pass, col k), D'
    const uint8_t *bpad;    // bpad[j] = code of B_j, bpad[0] = pad
    const uint8_t *arow;    // points at the code of A_{r+1}
    int64_t L, J;
    int32_t V;              // forward value of the end node
    int32_t pad_;
};

struct CrossOut {
    int32_t cmin;           // smallest frontier column a crossing needs (-1: none)
    int32_t count;          // number of crossing edges
    int32_t key;            // unique candidate: (column << 1) | vertical
    int32_t exit_col;       // unique candidate: node reached in row r (absolute column)
    int32_t exit_state;     // 0 = H, 1 = F
    int32_t exit_val;       // forward value of that node
    int32_t pad_[2];
};

// Crossing scan of one kept row of the two local score passes (the first
// split of the band traceback, engine.cpp).  For the cut between rows x and
// x+1 of the full matrix:
//   fwd[j] = (H(x, j), F(x+1, j))            forward local pass, j = 0..te
//   rev[c] = (H'(x+2, te-c), F'(x+1, te-c))  reverse local pass (reversed
//            columns; H'(i, j) and F'(i, j) are local values of the reversed
//            DP: the best alignment of A_i.., B_j.. that starts at row i)
// After a node in column j the path goes on with columns j+1 onwards, so an
// edge lies on an optimal local alignment iff forward + edge + reverse = S:
//   vertical into F(x+1, j):   F(x+1, j) + F'(x+1, j+1) + o               = S
//   diagonal into (x+1, j):    H(x, j-1) + s(A_{x+1}, B_j) + H'(x+2, j+1) = S
// (the open penalty of a gap through the cut is counted by both passes;
// H(x, -1) = 0 and H'(x+2, te+1) = 0 are the matrix borders, and no vertical
// edge in the last column can continue to the end cell).
struct CutDesc {
    const Border *fwd;
    const Border *rev;
    const uint8_t *arow;    // points at the code of A_{x+1}
    const uint8_t *tc;      // target codes, columns 0..te
    int64_t te;             // last column of the pair's rectangle
    int32_t S;              // the pair's optimum
    // global passes: fwd[-1] and rev[-1] are the records of the boundary
    // column (DP column 0 of each pass) instead of the local floor
    int32_t global;
};

// Resolved cut: clean = exactly one edge, and at a vertical edge the gap
// cannot close at row x (H(x, j) - o != F(x+1, j)), so that the node where
// the path meets row x is fixed.  That node is (x, col) in state H
// (diagonal edge, value H(x, col)) or F (vertical edge, value F(x+1, col) +
// e); the band below starts from it (seed record at column col).
struct CutOut {
    int32_t count;
    int32_t key;            // smallest (j << 1) | vertical
    int32_t clean;
    int32_t col;
    int32_t state;          // 0 = H, 1 = F
    int32_t val;
    int32_t seed_h, seed_f;
};

// One leaf: full DP with tie flags, then the greedy walk back to row 0 of
// the leaf (its frontier row).
struct LeafDesc {
    const uint8_t *arows;   // codes of the leaf rows (P)
    const uint8_t *bcols;   // codes of the leaf columns (w); pad for DP column 0
    const Border *front;    // front[k]: frontier row value at leaf column k
    uint8_t *gflags;        // large leaves: leaf_flag_bytes(P, w) bytes of global memory (else unused)
    char *ops;              // ops out, backward order
    int32_t P, w;
    int32_t end_state;      // 0 = H, 1 = F; the end is (P, w-1)
    int32_t ops_cap;
    int32_t V;              // forward value the end must have
    int32_t pad_;
};

// Large leaves (leaf_big_kernel): kLeafR rows per lane; tie flags in global
// memory, a nibble per cell, ceil(P / (64 kLeafR)) * (w + 63) * 64 dwords;
// LDS: matrix, per-lane profile, row buffer and column codes.
constexpr int kLeafR = 8;
inline int64_t leaf_flag_bytes(int64_t P, int64_t w) { return (P + 64 * kLeafR - 1) / (64 * kLeafR) * (w + 63) * 256; }
inline size_t leaf_big_lds(int asize, int64_t max_w)
{
    return (size_t)(1024 + (asize + 1) * 64 * (kLeafR / 4) * 4 + 9 * max_w + 16);
}

struct LeafOut {
    int32_t nops;
    int32_t exit_col;       // leaf column of the node reached in row 0
    int32_t exit_state;     // 0 = H, 1 = F
    int32_t exit_val;       // its forward value
    int32_t err;            // nonzero: the walk left the leaf, or the end value is not V
    int32_t pad_[3];
};

// One value picked from a row of border records row[0 .. count):
// mode 0: the largest h, at the smallest index; *out = ((h + 2^30) << 32) |
//         (0xFFFFFFFF - index) (zero on entry);
// mode 1: the smallest index >= 1 with h == target; *out = that index
//         (all ones on entry: none).
hipError_t launch_row_pick(const Border *row, int64_t count, int32_t target, int32_t mode, uint64_t *out,
                           hipStream_t st);

// The same reduction for many rows at once, one workgroup per row: out[k] =
// the key of descriptor k (mode 0: 0 when count is 0; mode 1: all ones when
// no entry matches).
struct RowPickDesc {
    const Border *row;
    int64_t count;
    int32_t target;
    int32_t mode;
};
hipError_t launch_row_pick_multi(const RowPickDesc *d, int32_t nd, uint64_t *out, hipStream_t st);

// Synthetic codes (timing runs of the autotuner): n codes in [0, asize), pad code up to padded.
hipError_t launch_random_codes(uint8_t *dst, int64_t n, int64_t padded, int32_t asize, uint64_t seed, hipStream_t st);
hipError_t launch_gather(const GatherDesc *d, int32_t nd, uint8_t pad, hipStream_t st);
hipError_t launch_border_init(const BorderInit *d, int32_t nd, int32_t o, int32_t e, hipStream_t st);
hipError_t launch_cross(const CrossDesc *d, int32_t nd, const int8_t *mat, int32_t asize, int32_t o, int32_t e,
                        CrossOut *out, hipStream_t st);
// counts[k] += edges of cut k, keys[k] = min key (counts zero, keys INT32_MAX
// or above on entry); one launch over all cuts (of any pairs); max_te = the
// largest te among them
hipError_t launch_cut_scan(const CutDesc *d, int32_t nd, int64_t max_te, const int8_t *mat, int32_t asize,
                           int32_t o, int32_t *counts, int32_t *keys, hipStream_t st);
hipError_t launch_cut_resolve(const CutDesc *d, int32_t nd, const int32_t *counts, const int32_t *keys, int32_t o,
                              int32_t e, CutOut *out, hipStream_t st);
hipError_t launch_leaf(const LeafDesc *d, int32_t nd, const int8_t *mat, int32_t asize, int32_t o, int32_t e,
                       size_t lds_bytes, LeafOut *out, hipStream_t st);
// large leaves; max_w = the widest leaf of the launch
hipError_t launch_leaf_big(const LeafDesc *d, int32_t nd, const int8_t *mat, int32_t asize, int32_t o, int32_t e,
                           int32_t max_w, LeafOut *out, hipStream_t st);

}  // namespace swh
