// tune.h -- strip shapes of the strip-wavefront kernel: built-in rule or a
// table measured on the device by the autotuner.
#pragma once

#include <stdint.h>

#include "context.h"

namespace swh {

struct StripShape {
    int R;       // rows per lane (strip height 64 R)
    int waves;   // waves per SIMD of the persistent grid (0: the rule for R)
};

// Shape for a problem of n rows: the context's tuned table when it has one,
// else the built-in rule.  The rows-per-lane option overrides R.
StripShape tuned_shape(swh_ctx *ctx, int64_t n);
inline int tuned_rows_per_lane(swh_ctx *ctx, int64_t n, int64_t) { return tuned_shape(ctx, n).R; }

// Time every (R, waves) candidate on synthetic problems for row buckets
// 1 Ki, 4 Ki, ... up to max_rows and install the fastest per bucket.
swh_status autotune(swh_ctx *ctx, const Scoring &sc, int64_t max_rows, double cells_per_trial);
// Measure the database length switch (swh_autotune_db).
swh_status autotune_db(swh_ctx *ctx, const Scoring &sc, const swh_scoring *raw, int32_t &inter_max);
swh_status tune_save(const swh_ctx *ctx, const char *path);
swh_status tune_load(swh_ctx *ctx, const char *path);

}  // namespace swh
