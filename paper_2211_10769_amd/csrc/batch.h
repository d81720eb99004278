// batch.h -- many pairwise alignments per call (batch.cpp).
#pragma once

#include <stdint.h>

#include <vector>

#include "context.h"

namespace swh {

// One local score pass: rows q[0..n) against columns t[0..m) (device codes);
// step -1 walks both backwards from the given pointers (reversed prefixes).
struct PairPass {
    const uint8_t *q;
    int64_t n;
    const uint8_t *t;
    int64_t m;
    int step;
    int R = 0, waves = 0;      // strip shape (R = 0: the shape rule for n rows)
    int64_t lead = 0;          // all-zero pad rows above row 0 (best rows count them)
    Border *keep = nullptr;    // kept rows (strips.h StripProblem), or NULL
    int32_t every = 0, phase = 0;
    int32_t prune = 0;         // known maximum of a reverse pass (block pruning), or 0
    bool int16 = false;        // packed 16-bit pass where the shape allows it (saturated passes are redone)
};
// Score, end row and end column of every pass (launches grouped by strip
// shape and precision, most expensive first, chunked to bound device memory).
// Passes asking for 16 bits run in the packed kernel when their strip height
// allows it; any whose maximum reaches sat16_limit is run again in 32 bits
// with the same strip height (so kept rows land on the same rows).
swh_status score_passes(swh_ctx *ctx, const std::vector<PairPass> &ps, const Scoring &sc, hipStream_t st,
                        std::vector<BestCell> &best, double &ms_total);

// Part of a pass's last row to reduce with the row-pick key (tb_kernels.h):
// entries first .. first+count-1 of the row (entry 0 = the pad column).
struct RowPick {
    int64_t first = 0, count = 0;
    int32_t target = 0, mode = 0;
};
inline int32_t row_key_value(uint64_t key) { return (int32_t)((uint32_t)(key >> 32) - (1u << 30)); }
inline int64_t row_key_index(uint64_t key) { return (int64_t)(0xFFFFFFFFu - (uint32_t)key); }

// Global-mode passes over [pad] + t, or t alone (both sequences read with the
// pass's step, n, m > 0) from a top border of BorderInit kind `kind`, with the
// free left border when free_left; keys[i] = the row pick of pass i's last
// row.  The device substitution table is used as it stands.
swh_status edge_scores(swh_ctx *ctx, const std::vector<PairPass> &ps, int32_t kind, const std::vector<RowPick> &picks,
                       const Scoring &sc, hipStream_t st, std::vector<uint64_t> &keys, double &ms_total,
                       bool pad_col = true, bool free_left = false);

// Upload the substitution table to the device, as given or transposed (passes
// that run the target down the rows score s(b, a)).
swh_status set_matrix(swh_ctx *ctx, const Scoring &sc, bool transposed, hipStream_t st);

// Global alignment scores G(n, m) of every pass (n, m > 0; step must be 1):
// the strip kernel in global mode over A against [pad] + B from the global
// top border G(0, j) = -(o + (j-1) e), G(0, 0) = 0.
swh_status global_scores(swh_ctx *ctx, const std::vector<PairPass> &ps, const Scoring &sc, hipStream_t st,
                         std::vector<int32_t> &scores, double &ms_total);

// dev: q_cat and t_cat are device pointers (encoded in place), else host pointers.
swh_status align_batch(swh_ctx *ctx, int64_t npairs, const char *q_cat, const int64_t *q_off, const char *t_cat,
                       const int64_t *t_off, const Scoring &sc, int mode, swh_alignment *out, char *cigar_cat,
                       int64_t cigar_cap, int64_t *cigar_off, swh_stats *stats, bool dev = false);

}  // namespace swh
