// tb_kernels.h -- device-side descriptors of the traceback kernels
// (tb_kernels.hip), shared with the host driver (traceback.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "engine.h"

namespace swh {

// dst[i] = first_pad && i == 0 ? pad : src[start + step * (i - first_pad)]
// for i < count; pad up to padded.
struct GatherDesc {
    const uint8_t *src;
    uint8_t *dst;
    int64_t start;
    int64_t count;
    int64_t padded;
    int32_t step;        // +1 or -1
    int32_t first_pad;   // 1: dst[0] is the pad code and the copy starts at dst[1]
};

// Top row of one DP pass.  kind 0: copy count entries from src;
// kind 1: backward pass whose end is an H cell: G'(c) = c ? -o-(c-1)e : 0,
//         D'(c) = G'(c) - o;
// kind 2: backward pass whose end is an F cell: G' = -inf, D'(0) = -o,
//         D'(c>0) = -inf.  Entries from count to padded are (-inf, -inf).
struct BorderInit {
    Border *dst;
    const Border *src;
    int64_t count;
    int64_t padded;
    int32_t kind;
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

// One leaf: full DP with tie flags, then the greedy walk back to row 0 of
// the leaf (its frontier row).
struct LeafDesc {
    const uint8_t *arows;   // codes of the leaf rows (P)
    const uint8_t *bcols;   // codes of the leaf columns (w); pad for DP column 0
    const Border *front;    // front[k]: frontier row value at leaf column k
    uint8_t *gflags;        // P*w bytes in global memory, or NULL to use LDS
    char *ops;              // ops out, backward order
    int32_t P, w;
    int32_t end_state;      // 0 = H, 1 = F; the end is (P, w-1)
    int32_t ops_cap;
};

struct LeafOut {
    int32_t nops;
    int32_t exit_col;       // leaf column of the node reached in row 0
    int32_t exit_state;     // 0 = H, 1 = F
    int32_t exit_val;       // its forward value
    int32_t err;            // nonzero: walk left the leaf (internal error)
    int32_t pad_[3];
};

// Synthetic codes (timing runs of the autotuner): n codes in [0, asize), pad code up to padded.
hipError_t launch_random_codes(uint8_t *dst, int64_t n, int64_t padded, int32_t asize, uint64_t seed, hipStream_t st);
hipError_t launch_gather(const GatherDesc *d, int32_t nd, uint8_t pad, hipStream_t st);
hipError_t launch_border_init(const BorderInit *d, int32_t nd, int32_t o, int32_t e, hipStream_t st);
hipError_t launch_cross(const CrossDesc *d, int32_t nd, const int8_t *mat, int32_t asize, int32_t o, int32_t e,
                        CrossOut *out, hipStream_t st);
hipError_t launch_leaf(const LeafDesc *d, int32_t nd, const int8_t *mat, int32_t asize, int32_t o, int32_t e,
                       size_t lds_bytes, LeafOut *out, hipStream_t st);

}  // namespace swh
