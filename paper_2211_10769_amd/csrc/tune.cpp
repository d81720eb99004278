// tune.cpp -- the autotuner of the strip kernel's shape.  For each bucket of
// query rows it builds a synthetic batch of problems of that height, times
// one launch per candidate (rows per lane, waves per SIMD), and keeps the
// fastest.  Results are bit-identical for every shape; only speed differs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "context.h"
#include "db.h"
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

swh_status autotune_db(swh_ctx *ctx, const Scoring &sc, const swh_scoring *raw, int32_t &inter_max)
{
    // synthetic sequences of uniform random symbols of the scoring's alphabet
    std::mt19937_64 rng(0x5EA5C4ull);
    std::uniform_int_distribution<int> sym(0, sc.asize - 1);
    std::vector<char> qcat;
    std::vector<int64_t> qoff{0};
    for (int q = 0; q < 4; ++q) {
        for (int i = 0; i < 400; ++i) qcat.push_back(raw->alphabet[sym(rng)]);
        qoff.push_back((int64_t)qcat.size());
    }
    const int32_t saved = ctx->opt.inter_max, saved_route = ctx->opt.db_route;
    ctx->opt.db_route = -1;   // time the kernels as chosen, unrouted
    int32_t best = 512;
    swh_status s = SWH_OK;
    for (int32_t T = 1024; T <= 8192; T *= 2) {
        // a bucket of lengths in (T/2, T]: on the inter-task kernel at switch T,
        // on the single-pair kernel at switch T/2
        const int64_t count = std::max<int64_t>(256, (int64_t)(2e10 / (1600.0 * 0.75 * T)));
        std::uniform_int_distribution<int> len(T / 2 + 1, T);
        std::vector<char> cat;
        std::vector<int64_t> off{0};
        for (int64_t i = 0; i < count; ++i) {
            const int L = len(rng);
            for (int j = 0; j < L; ++j) cat.push_back(raw->alphabet[sym(rng)]);
            off.push_back((int64_t)cat.size());
        }
        double ms[2] = {0.0, 0.0};
        for (int side = 0; side < 2 && s == SWH_OK; ++side) {
            ctx->opt.inter_max = side == 0 ? T : T / 2;
            swh_db *db = nullptr;
            if ((s = db_create(ctx, count, cat.data(), off.data(), sc, &db)) != SWH_OK) break;
            const size_t bytes = sizeof(int32_t) * 4 * (size_t)count + 64;
            s = ensure(ctx, ctx->db_scores, bytes, "score matrix");
            // one warm-up, then the faster of two timed runs
            double t = 1e30;
            for (int rep = 0; rep < 3 && s == SWH_OK; ++rep) {
                DbStats ds;
                s = db_scores_device(ctx, db, 4, qcat.data(), qoff.data(), (int32_t *)ctx->db_scores.p, ds);
                if (rep > 0) t = std::min(t, ds.ms_inter + ds.ms_intra);
            }
            ms[side] = t;
            db_destroy(db);
        }
        if (s != SWH_OK) break;
        if (ms[0] <= ms[1])
            best = T;
        else
            break;
    }
    ctx->opt.inter_max = saved;
    ctx->opt.db_route = saved_route;
    if (s != SWH_OK) return s;
    ctx->tuned_inter_max = best;
    inter_max = best;
    return SWH_OK;
}

swh_status tune_save(const swh_ctx *ctx, const char *path)
{
    FILE *f = std::fopen(path, "w");
    if (!f) return SWH_E_INVAL;
    std::fprintf(f, "swh-tune 1\ndevice %s\ninter_max %d\n", ctx->device_name.c_str(), (int)ctx->tuned_inter_max);
    for (const swh_tune_entry &t : ctx->tune)
        std::fprintf(f, "shape %lld %d %d\n", (long long)t.max_rows, (int)t.rows_per_lane, (int)t.waves_per_simd);
    const bool ok = std::fclose(f) == 0;
    return ok ? SWH_OK : SWH_E_INVAL;
}

swh_status tune_load(swh_ctx *ctx, const char *path)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(ctx, SWH_E_INVAL, std::string("cannot open ") + path);
    char line[512];
    std::vector<swh_tune_entry> table;
    int32_t inter = 0;
    bool header = false, device_ok = false;
    while (std::fgets(line, sizeof(line), f)) {
        int v = 0, r = 0, w = 0;
        long long mr = 0;
        if (std::strncmp(line, "swh-tune 1", 10) == 0) {
            header = true;
        } else if (std::strncmp(line, "device ", 7) == 0) {
            std::string name(line + 7);
            while (!name.empty() && (name.back() == '\n' || name.back() == '\r')) name.pop_back();
            device_ok = name == ctx->device_name;
        } else if (std::sscanf(line, "inter_max %d", &v) == 1) {
            inter = v;
        } else if (std::sscanf(line, "shape %lld %d %d", &mr, &r, &w) == 3) {
            table.push_back(swh_tune_entry{(int64_t)mr, r, w});
        }
    }
    std::fclose(f);
    if (!header) return fail(ctx, SWH_E_INVAL, "not a tuning file");
    if (!device_ok) return fail(ctx, SWH_E_INVAL, "tuning file was written on another device");
    if (inter != 0 && (inter < 32 || inter > 8192)) return fail(ctx, SWH_E_INVAL, "tuning file: bad length switch");
    for (size_t i = 0; i < table.size(); ++i) {
        const int R = table[i].rows_per_lane;
        if ((R != 4 && R != 8 && R != 16 && R != 20 && R != 24 && R != 32) || table[i].waves_per_simd < 0 ||
            table[i].waves_per_simd > 8 || table[i].max_rows < 1 ||
            (i > 0 && table[i].max_rows <= table[i - 1].max_rows))
            return fail(ctx, SWH_E_INVAL, "tuning file: bad shape entry");
    }
    ctx->tune = table;
    ctx->tuned_inter_max = inter;
    return SWH_OK;
}

}  // namespace swh
