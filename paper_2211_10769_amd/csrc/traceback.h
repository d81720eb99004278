// traceback.h -- reconstruction phase: linear-space traceback over the
// aligned rectangle (frontier-seeded divide and conquer).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "context.h"

namespace swh {

struct TracebackStats {
    double ms = 0.0;      // wall time
    double cells = 0.0;   // DP cells evaluated
    int64_t leaves = 0;
    int64_t splits = 0;
    bool inconsistent = false;   // a crossing or an end value did not check out
};

// One band of a rectangle (rectangle coordinates, rows and columns from 1):
// rows (r_top, r_bot], columns [L, J].  Its frontier on row r_top is the
// rectangle's top border (seeded = false: r_top = 0, L = 0) or a single node
// at column L with record (seed_h, seed_f) -- H there and the F it hands down,
// -inf for the transition the path does not take.  The end node (r_bot, J) is
// in state end_state (0 = H, 1 = F) with forward value V.
struct TbBand {
    int64_t r_top, r_bot, L, J;
    bool seeded;
    int32_t seed_h, seed_f;
    int end_state;
    int32_t V;
};

struct TbInput {
    const uint8_t *A;   // p codes on the device (rows of the aligned rectangle)
    int64_t p;
    const uint8_t *B;   // q codes on the device (columns)
    int64_t q;
    int32_t S;          // optimum of the rectangle (the local score)
    // top to bottom, the path's crossings between them known; empty = one
    // band, the whole rectangle ending at (p, q) in state H with value S
    std::vector<TbBand> bands = {};
};

// Canonical CIGARs of many rectangles; their subproblems share the launches
// of each level.
swh_status traceback_batch(swh_ctx *ctx, const std::vector<TbInput> &in, const Scoring &sc, hipStream_t st,
                           std::vector<std::string> &cigars, TracebackStats &ts);

// Canonical CIGAR of the global alignment of A (p codes, device) against
// B (q codes, device) whose optimum is S (the local score of the rectangle).
swh_status traceback(swh_ctx *ctx, const uint8_t *A, int64_t p, const uint8_t *B, int64_t q,
                     const Scoring &sc, int32_t S, hipStream_t st, std::string &cigar, TracebackStats &ts);

}  // namespace swh
