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
};

struct TbInput {
    const uint8_t *A;   // p codes on the device (rows of the aligned rectangle)
    int64_t p;
    const uint8_t *B;   // q codes on the device (columns)
    int64_t q;
    int32_t S;          // optimum of the rectangle (the local score)
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
