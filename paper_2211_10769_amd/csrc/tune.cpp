// tune.cpp -- the autotuner of the strip kernel's shape.  For each bucket of
// query rows it builds a synthetic batch of problems of that height, times
// one launch per candidate (rows per lane, waves per SIMD), and keeps the
// fastest.  Results are bit-identical for every shape; only speed differs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "context.h"
#include "strips.h"
#include "tb_kernels.h"
#include "tune.h"

namespace swh {

StripShape tuned_shape(swh_ctx *ctx, int64_t n)
{
    const int forced = ctx->opt.rows;
    if (forced == 4 || forced == 8 || forced == 16 || forced == 20 || forced == 24 || forced == 32)
        return StripShape{forced, 0};
    for (const swh_tune_entry &t : ctx->tune)
        if (n <= t.max_rows) return StripShape{t.rows_per_lane, t.waves_per_simd};
    if (!ctx->tune.empty()) return StripShape{ctx->tune.back().rows_per_lane, ctx->tune.back().waves_per_simd};
    return StripShape{pick_rows_per_lane(n, 4 * ctx->num_cu), 0};
}

swh_status autotune(swh_ctx *ctx, const Scoring &sc, int64_t max_rows, double cells_per_trial)
{
    hipStream_t st = ctx->own_stream;
    max_rows = std::max<int64_t>(max_rows, 1024);
    cells_per_trial = std::max(cells_per_trial, 1e8);
    std::vector<swh_tune_entry> table;
    swh_status s;
    hipError_t e;
    if ((s = ensure(ctx, ctx->mat, 32 * 32, "matrix")) != SWH_OK) return s;
    if ((e = hipMemcpyAsync(ctx->mat.p, sc.mat, (size_t)sc.asize * sc.asize, hipMemcpyHostToDevice, st)) !=
        hipSuccess)
        return hip_fail(ctx, e, "matrix upload");
    for (int64_t edge = 1024;; edge *= 4) {
        const int64_t n = std::max<int64_t>(64, edge * 3 / 4);
        const int64_t m = std::max<int64_t>(4096, std::min<int64_t>(n, 65536));
        const int64_t count = std::max<int64_t>(1, (int64_t)(cells_per_trial / ((double)n * (double)m)));
        const int64_t qpad = rows_padded(n, 32), tpad = cols_padded(m);
        if ((s = ensure(ctx, ctx->bq, (size_t)qpad + 256, "tuning rows")) != SWH_OK ||
            (s = ensure(ctx, ctx->bt, (size_t)tpad + 256, "tuning columns")) != SWH_OK ||
            (s = ensure(ctx, ctx->bborder, sizeof(Border) * (size_t)(tpad * count) + 256, "tuning borders")) !=
                SWH_OK)
            return s;
        if ((e = launch_random_codes((uint8_t *)ctx->bq.p, n, qpad, sc.asize, 0x5157u + (uint64_t)edge, st)) !=
                hipSuccess ||
            (e = launch_random_codes((uint8_t *)ctx->bt.p, m, tpad, sc.asize, 0x7a11u + (uint64_t)edge, st)) !=
                hipSuccess)
            return hip_fail(ctx, e, "tuning inputs");
        std::vector<StripProblem> probs;
        for (int64_t k = 0; k < count; ++k)
            probs.push_back(StripProblem{(const uint8_t *)ctx->bq.p, n, (const uint8_t *)ctx->bt.p, m,
                                         (Border *)ctx->bborder.p + k * tpad});
        swh_tune_entry best{edge >= max_rows ? INT64_MAX : edge, 4, 0};
        float best_ms = 1e30f;
        for (int R : {4, 8, 16, 20, 24, 32}) {
            if (64 * R > 4 * n && R > 4) continue;   // strips far taller than the problem
            for (int waves : {1, 2, 4, 8}) {
                if (waves * 4 * ctx->num_cu > strip_grid_limit(ctx->device, R, true, sc.asize)) continue;
                if ((e = hipMemsetAsync(ctx->bborder.p, 0, sizeof(Border) * (size_t)(tpad * count), st)) !=
                    hipSuccess)
                    return hip_fail(ctx, e, "tuning borders");
                std::vector<BestCell> b;
                float ms = 0.f;
                if ((s = run_strips(ctx, probs, sc, R, true, st, &b, &ms, waves)) != SWH_OK) return s;
                if (ms < best_ms) {
                    best_ms = ms;
                    best.rows_per_lane = R;
                    best.waves_per_simd = waves;
                }
            }
        }
        table.push_back(best);
        if (edge >= max_rows) break;
    }
    ctx->tune = table;
    return SWH_OK;
}

}  // namespace swh
