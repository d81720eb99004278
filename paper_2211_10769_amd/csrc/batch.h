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
};
// Score, end row and end column of every pass (launches grouped by strip
// shape, most expensive first, chunked to bound device memory).
swh_status score_passes(swh_ctx *ctx, const std::vector<PairPass> &ps, const Scoring &sc, hipStream_t st,
                        std::vector<BestCell> &best, double &ms_total);

// Global alignment scores G(n, m) of every pass (n, m > 0; step must be 1):
// the strip kernel in global mode over A against [pad] + B from the global
// top border G(0, j) = -(o + (j-1) e), G(0, 0) = 0.
swh_status global_scores(swh_ctx *ctx, const std::vector<PairPass> &ps, const Scoring &sc, hipStream_t st,
                         std::vector<int32_t> &scores, double &ms_total);

swh_status align_batch(swh_ctx *ctx, int64_t npairs, const char *q_cat, const int64_t *q_off, const char *t_cat,
                       const int64_t *t_off, const Scoring &sc, int mode, swh_alignment *out, char *cigar_cat,
                       int64_t cigar_cap, int64_t *cigar_off, swh_stats *stats);

}  // namespace swh
