// strips.cpp -- host side of the strip-wavefront kernel: runs one launch over
// a table of independent DP problems (one pairwise pass, the passes of one
// traceback level, or a batch of pairs).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "context.h"
#include "engine.h"
#include "strips.h"
#include "db_kernels.h"

namespace swh {

// A single chunk wait longer than this is a bug (the wavefront cannot
// deadlock); the kernel then drains and the call fails with SWH_E_TIMEOUT.
constexpr double kWaitSeconds = 30.0;

uint64_t wait_ticks(int device)
{
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || khz <= 0)
        khz = 100000;   // 100 MHz constant clock
    return (uint64_t)(kWaitSeconds * 1e3 * khz);
}

// Strip height for a launch whose problems hold n rows in all.  The strips of
// one problem form a chain that moves at the pace of its slowest wave, so a
// long problem runs with one wave per SIMD; each SIMD then runs
// ceil(strips / SIMDs) strips one after the other, and a step of a strip costs
// about 7.5 R + 24 instructions (7 per cell, half a max per cell for the
// end-cell tracker, and lane shifts and profile reads per step).  Long
// problems take the R in {8, 16, 20, 24, 32} that minimises
// ceil(strips / SIMDs) (7.5 R + 24).  Same-box measurements on the 5 Mbp pair
// (4,883 strips of 1,024 rows, 3,907 of 1,280, ...): R = 20 7.21 s, R = 16
// 7.45 s, R = 24 8.13 s; earlier R = 32 about 5% slower than R = 16, and two
// waves per SIMD 23% slower.
int pick_rows_per_lane(int64_t n, int simds)
{
    simds = std::max(simds, 1);
    auto strips = [&](int R) { return (n + 64 * R - 1) / (64 * R); };
    if (strips(8) >= (int64_t)simds) {
        // Every strip of a problem takes the same time and one wave keeps a
        // SIMD busy, so the pass takes ceil(strips / SIMDs) strip times.  A
        // strip time is proportional to the cycles one step (a 64-column
        // diagonal of 64 R cells) takes; measured per R on a 2 Mbp pair, one
        // wave per SIMD (R = 32 runs well above the linear trend of the others).
        static const struct { int R; int64_t cycles; } kStep[] = {{8, 428}, {16, 734}, {20, 844}, {24, 960},
                                                                   {32, 1581}};
        int best = 8;
        int64_t best_cost = INT64_MAX;
        for (const auto &k : kStep) {
            const int64_t cost = (strips(k.R) + simds - 1) / simds * k.cycles;
            if (cost < best_cost) {
                best_cost = cost;
                best = k.R;
            }
        }
        return best;
    }
    // shorter problems come in batches: 8 rows per lane costs fewer operations
    // per cell than 4 (sweep on 20,000 read pairs: 1.78 s against 2.01 s)
    return n >= 512 ? 8 : 4;
}

// Grid of single-wave workgroups (used when the balanced placement cannot be
// made, or the grid option forces it): a whole number of waves per SIMD on
// average, 8 for R=4, 4 for R=8 and 1 for taller strips.
int strip_grid(int64_t nstrips, int R, int limit, int num_cu, int waves, int forced)
{
    if (forced > 0) return (int)std::min<int64_t>(forced, nstrips);
    const int per_simd = waves > 0 ? waves : R <= 4 ? 8 : R <= 8 ? 4 : 1;
    const int want = std::min(limit, per_simd * 4 * std::max(num_cu, 1));
    return (int)std::max<int64_t>(1, std::min<int64_t>(nstrips, want));
}

bool int16_usable(const swh_ctx *ctx, const Scoring &sc, int R)
{
    return ctx->opt.int16 != 0 && (R == 4 || R == 8 || R == 16) && strip16_supported(2 * R, sc.asize, ctx->device);
}

swh_status prepare_strips(swh_ctx *ctx, const std::vector<StripProblem> &probs, const Scoring &sc, int R, bool local,
                          int waves, bool int16, PreparedStrips &out)
{
    const int np = (int)probs.size();
    if (int16 && (!local || (R != 4 && R != 8 && R != 16) || !strip16_supported(2 * R, sc.asize, ctx->device)))
        return fail(ctx, SWH_E_INVAL, "packed 16-bit pass requested for an unsupported shape");
    // the 16-bit kernel's strips hold two sub-strips of the nominal height
    const int RK = int16 ? 2 * R : R;
    out.R = R;
    out.local = local;
    out.int16 = int16;
    out.np = np;
    std::vector<Problem> &tab = out.tab;
    std::vector<int32_t> &sp = out.strip_prob;
    tab.resize(np);
    sp.clear();
    int64_t total_strips = 0, total_flags = 0;
    bool prune = false;
    for (int i = 0; i < np; ++i) {
        const StripProblem &q = probs[i];
        Problem &P = tab[i];
        P.qc = q.qc;
        P.tc = q.tc;
        P.border = q.border;
        P.n = (int32_t)q.n;
        P.m = (int32_t)q.m;
        P.nstrips = (int32_t)((q.n + 64 * RK - 1) / (64 * RK));
        // a strip waits for chunk 0 of the strip above, which a problem without
        // columns never publishes
        if (q.m <= 0 && P.nstrips > 1) return fail(ctx, SWH_E_INVAL, "strip problem with rows but no columns");
        P.nblocks = (int32_t)sweep_blocks(q.m) + (int16 ? 1 : 0);   // the 16-bit high halves trail by a block
        P.strip0 = (int32_t)total_strips;
        P.flags = (int32_t *)(intptr_t)total_flags;   // offset, fixed up below
        P.save = q.save;
        P.save_every = q.save ? q.save_every : 0;
        P.save_stride = q.save_stride;
        P.save_phase = q.save_phase;
        P.free_left = q.free_left;
        P.prune = local ? q.prune : 0;
        P.top_pass = local ? 0 : q.top_pass;
        prune = prune || P.prune > 0;
        total_strips += P.nstrips;
        total_flags += P.nblocks + 3;
        if (np > 1)
            for (int k = 0; k < P.nstrips; ++k) sp.push_back(i);
    }
    if (total_strips >= INT32_MAX) return fail(ctx, SWH_E_RANGE, "too many strips in one launch");
    swh_status s;
    if ((s = ensure(ctx, ctx->flags, (size_t)total_flags * 4, "chunk counters")) != SWH_OK) return s;
    if ((s = ensure(ctx, ctx->strip_best, (size_t)total_strips * sizeof(BestCell), "strip results")) != SWH_OK)
        return s;
    if ((s = ensure(ctx, ctx->probs, (size_t)np * sizeof(Problem), "problem table")) != SWH_OK) return s;
    if (np > 1 && (s = ensure(ctx, ctx->strip_prob, sp.size() * 4, "strip table")) != SWH_OK) return s;
    if (local && (s = ensure(ctx, ctx->prob_best, (size_t)np * sizeof(BestCell), "problem results")) != SWH_OK)
        return s;
    if ((s = ensure(ctx, ctx->sync, 64, "ticket")) != SWH_OK) return s;
    for (int i = 0; i < np; ++i)
        tab[i].flags = (int32_t *)ctx->flags.p + (intptr_t)tab[i].flags;
    out.total_strips = total_strips;
    out.total_flags = total_flags;
    out.prune = prune;

    // Strips of one problem form a chain that moves at the pace of its slowest
    // wave, so every SIMD must hold the same number of waves: a balanced
    // placement when it can be made (with fewer waves per SIMD when there are
    // few strips), else single-wave workgroups (the grid option forces those).
    const size_t wave_lds = int16 ? strip16_lds_bytes(RK, sc.asize) : strip_lds_bytes(R, sc.asize);
    StripLaunch grid{0, 1, wave_lds};
    const int forced = ctx->opt.grid;
    // long chains of a few big problems want one wave per SIMD (their strips
    // come in rounds of one per SIMD); problems at least as many as the SIMDs
    // fill the GPU with independent chains whatever their length and want
    // several waves to hide latency (read-pair batch: 4 for R = 8)
    const bool long_chains = total_strips >= 16 * (int64_t)np && np < 4 * ctx->num_cu;
    int per_simd = waves > 0 ? waves : long_chains ? 1 : (RK <= 4 ? 8 : 4);
    while (per_simd > 1 && (int64_t)per_simd / 2 * 4 * ctx->num_cu >= total_strips) per_simd /= 2;
    const bool balanced = int16 ? strip16_balanced_launch(ctx->device, RK, sc.asize, per_simd, ctx->num_cu, grid)
                                : strip_balanced_launch(ctx->device, R, local, sc.asize, per_simd, ctx->num_cu, grid);
    if (forced > 0 || !balanced) {
        const int limit = int16 ? strip16_grid_limit(ctx->device, RK, sc.asize)
                                : strip_grid_limit(ctx->device, R, local, sc.asize);
        grid = StripLaunch{strip_grid(total_strips, RK, limit, ctx->num_cu, waves, forced), 1, wave_lds};
    }
    out.grid = grid;

    // With problems enough to fill the GPU the tickets go level by level: strip
    // 0 of every problem (in the caller's order), then strip 1 of every problem
    // with two or more, and so on.  By the time a strip is taken the strip above
    // has long had the head start of a few blocks it waits for, so no wave sits
    // idle building it up; the tickets of one problem keep increasing.  Measured
    // on 200,000 read pairs (score-mode forward): consecutive tickets 2.12 s,
    // strip k about k G tickets after strip 0: G = 512 2.01 s, 4,096 1.87 s,
    // 16,384 1.80 s, level by level 1.78 s.
    out.strip_order.clear();
    if (np >= 4 * ctx->num_cu && total_strips > np) {
        int32_t levels = 0;
        for (int i = 0; i < np; ++i) levels = std::max(levels, tab[i].nstrips);
        std::vector<int64_t> start((size_t)levels + 1, 0);   // tickets before level k
        for (int i = 0; i < np; ++i)
            for (int32_t k = 0; k < tab[i].nstrips; ++k) ++start[(size_t)k + 1];
        for (int32_t k = 0; k < levels; ++k) start[(size_t)k + 1] += start[(size_t)k];
        out.strip_order.resize((size_t)total_strips);
        for (int i = 0; i < np; ++i)
            for (int32_t k = 0; k < tab[i].nstrips; ++k) out.strip_order[(size_t)start[(size_t)k]++] = tab[i].strip0 + k;
        if ((s = ensure(ctx, ctx->strip_order, out.strip_order.size() * 4, "strip order")) != SWH_OK) return s;
    }
    return SWH_OK;
}

hipError_t enqueue_strips(swh_ctx *ctx, const PreparedStrips &ps, const Scoring &sc, const Problem *tab_src,
                          const int32_t *sp_src, hipStream_t st, bool timed)
{
    hipError_t e;
    // counters and ticket cleared by kernels (no memset node in a captured graph)
    if ((e = launch_fill_i32((int32_t *)ctx->flags.p, ps.total_flags, 0, st)) != hipSuccess ||
        (e = launch_fill_i32((int32_t *)ctx->sync.p, 2, 0, st)) != hipSuccess ||
        (e = hipMemcpyAsync(ctx->probs.p, tab_src, (size_t)ps.np * sizeof(Problem), hipMemcpyHostToDevice, st)) !=
            hipSuccess ||
        (ps.np > 1 && (e = hipMemcpyAsync(ctx->strip_prob.p, sp_src, ps.strip_prob.size() * 4,
                                          hipMemcpyHostToDevice, st)) != hipSuccess) ||
        (!ps.strip_order.empty() && (e = hipMemcpyAsync(ctx->strip_order.p, ps.strip_order.data(),
                                                        ps.strip_order.size() * 4, hipMemcpyHostToDevice, st)) !=
                                        hipSuccess))
        return e;
    StripArgs a;
    a.probs = (const Problem *)ctx->probs.p;
    a.strip_prob = ps.np > 1 ? (const int32_t *)ctx->strip_prob.p : nullptr;
    a.strip_order = ps.strip_order.empty() ? nullptr : (const int32_t *)ctx->strip_order.p;
    a.total_strips = (int32_t)ps.total_strips;
    a.mat = (const int8_t *)ctx->mat.p;
    a.asize = sc.asize;
    a.o = sc.o;
    a.e = sc.e;
    a.smax = sc.smax;
    a.ticket = (int32_t *)ctx->sync.p;
    a.abort_flag = (int32_t *)ctx->sync.p + 1;
    a.cancel = ctx->cancel_dev;
    a.strip_best = (BestCell *)ctx->strip_best.p;
    a.wait_ticks = wait_ticks(ctx->device);
    const int RK = ps.int16 ? 2 * ps.R : ps.R;
    if (timed) hipEventRecord(ctx->ev[0], st);
    if ((e = ps.int16 ? launch_strip16(a, RK, ps.grid, st, ps.prune)
                      : launch_strip(a, ps.R, ps.local, ps.grid, st, ps.prune)) != hipSuccess)
        return e;
    if (timed) hipEventRecord(ctx->ev[1], st);
    if (ps.local && (e = launch_reduce_best_multi(a.strip_best, a.probs, ps.np, (BestCell *)ctx->prob_best.p, st)) !=
                        hipSuccess)
        return e;
    return hipSuccess;
}

swh_status run_strips(swh_ctx *ctx, const std::vector<StripProblem> &probs, const Scoring &sc, int R, bool local,
                      hipStream_t st, std::vector<BestCell> *best, float *ms, int waves, bool int16)
{
    const int np = (int)probs.size();
    if (np == 0) return SWH_OK;
    PreparedStrips &ps = ctx->strips;
    swh_status s = prepare_strips(ctx, probs, sc, R, local, waves, int16, ps);
    if (s != SWH_OK) return s;
    hipError_t e;
    if ((e = enqueue_strips(ctx, ps, sc, ps.tab.data(), ps.strip_prob.data(), st, true)) != hipSuccess)
        return hip_fail(ctx, e, "strip pass launch");
    int32_t flags_host[2] = {0, 0};
    if ((e = hipMemcpyAsync(flags_host, ctx->sync.p, 8, hipMemcpyDeviceToHost, st)) != hipSuccess)
        return hip_fail(ctx, e, "hipMemcpyAsync(abort flag)");
    if (local && best) {
        best->resize(np);
        if ((e = hipMemcpyAsync(best->data(), ctx->prob_best.p, (size_t)np * sizeof(BestCell), hipMemcpyDeviceToHost,
                                st)) != hipSuccess)
            return hip_fail(ctx, e, "hipMemcpyAsync(results)");
    }
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(ctx, e, "strip pass");
    if (ms) hipEventElapsedTime(ms, ctx->ev[0], ctx->ev[1]);
    if (flags_host[1]) {
        if (cancelled(ctx)) return cancel_status(ctx);
        return fail(ctx, SWH_E_TIMEOUT, "strip wavefront wait expired");
    }
    if (cancelled(ctx)) return cancel_status(ctx);
    return SWH_OK;
}

}  // namespace swh
