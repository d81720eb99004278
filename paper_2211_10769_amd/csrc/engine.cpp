// engine.cpp -- host orchestration of one pairwise alignment:
// encode -> forward local pass (score, end) -> reverse local pass on the
// reversed prefixes (start) -> linear-space traceback (CIGAR).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <string>

#include "context.h"
#include "engine.h"
#include "traceback.h"

namespace swh {

namespace {

// misc buffer layout (int32 words)
enum { kTicket = 0, kAbort = 1, kBadQ = 2, kBadT = 3, kResult = 4, kMiscWords = 8 };

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

// Tuning knobs (environment): SWH_ROWS forces the rows per lane (4, 8, 16,
// 32), SWH_GRID the persistent grid of the strip kernel.
int env_int(const char *name, int dflt)
{
    const char *v = std::getenv(name);
    if (!v || !*v) return dflt;
    return std::atoi(v);
}

int pick_rows_per_lane(int64_t n)
{
    const int forced = env_int("SWH_ROWS", 0);
    if (forced == 4 || forced == 8 || forced == 16 || forced == 32) return forced;
    if (n >= 200000) return 16;
    if (n >= 20000) return 8;
    return 4;
}

// Persistent grid: a whole number of waves per SIMD (every strip waits on the
// previous one, so the wavefront runs at the pace of the most loaded SIMD and
// an uneven spread of waves over SIMDs slows everything down).  Waves per
// SIMD by strip height, from sweeps on the long DNA pair: 8 for R=4, 4 for
// R=8, 2 for R=16 and R=32.
int strip_grid(int nstrips, int R, int limit, int num_cu)
{
    const int forced = env_int("SWH_GRID", 0);
    if (forced > 0) return std::min(forced, nstrips);
    const int per_simd = R <= 4 ? 8 : R <= 8 ? 4 : 2;
    const int want = std::min(limit, per_simd * 4 * std::max(num_cu, 1));
    return std::max(1, std::min(nstrips, want));
}

struct LocalPass {
    BestCell best{0, 0, 0, 0};
    float ms = 0.f;
};

// One local score pass over encoded inputs already on the device.
// qc must hold nstrips*64*R codes (pad beyond n), tc 64*(sweep_blocks(m)+3) codes.
swh_status local_pass(swh_ctx *ctx, const uint8_t *qc, int64_t n, const uint8_t *tc, int64_t m,
                      const Scoring &sc, int R, hipStream_t st, LocalPass &res)
{
    const int32_t nstrips = (int32_t)((n + 64 * R - 1) / (64 * R));
    const int32_t nblocks = (int32_t)sweep_blocks(m);
    const size_t bcount = (size_t)64 * (nblocks + 3);
    swh_status s;
    if ((s = ensure(ctx, ctx->border, bcount * sizeof(Border), "border buffer")) != SWH_OK) return s;
    if ((s = ensure(ctx, ctx->flags, (size_t)(nblocks + 3) * 4, "chunk counters")) != SWH_OK) return s;
    if ((s = ensure(ctx, ctx->strip_best, (size_t)nstrips * sizeof(BestCell), "strip results")) != SWH_OK)
        return s;
    int32_t *misc = (int32_t *)ctx->misc.p;
    hipError_t e;
    if ((e = hipMemsetAsync(ctx->border.p, 0, bcount * sizeof(Border), st)) != hipSuccess)
        return hip_fail(ctx, e, "hipMemsetAsync(border)");
    if ((e = hipMemsetAsync(ctx->flags.p, 0, (size_t)(nblocks + 3) * 4, st)) != hipSuccess)
        return hip_fail(ctx, e, "hipMemsetAsync(flags)");
    if ((e = hipMemsetAsync(misc + kTicket, 0, 8, st)) != hipSuccess)
        return hip_fail(ctx, e, "hipMemsetAsync(ticket)");

    StripArgs a;
    a.qc = qc;
    a.tc = tc;
    a.n = (int32_t)n;
    a.m = (int32_t)m;
    a.nstrips = nstrips;
    a.nblocks = nblocks;
    a.mat = (const int8_t *)ctx->mat.p;
    a.asize = sc.asize;
    a.o = sc.o;
    a.e = sc.e;
    a.border = (Border *)ctx->border.p;
    a.flags = (int32_t *)ctx->flags.p;
    a.ticket = misc + kTicket;
    a.abort_flag = misc + kAbort;
    a.strip_best = (BestCell *)ctx->strip_best.p;
    a.wait_ticks = wait_ticks(ctx->device);
    const int grid = strip_grid(nstrips, R, strip_grid_limit(ctx->device, R, true, sc.asize), ctx->num_cu);

    hipEventRecord(ctx->ev[0], st);
    if ((e = launch_strip(a, R, true, grid, st)) != hipSuccess) return hip_fail(ctx, e, "strip kernel launch");
    hipEventRecord(ctx->ev[1], st);
    if ((e = launch_reduce_best(a.strip_best, nstrips, (BestCell *)(misc + kResult), st)) != hipSuccess)
        return hip_fail(ctx, e, "reduce kernel launch");
    int32_t host[kMiscWords];
    if ((e = hipMemcpyAsync(host, misc, sizeof(host), hipMemcpyDeviceToHost, st)) != hipSuccess)
        return hip_fail(ctx, e, "hipMemcpyAsync(result)");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(ctx, e, "strip pass");
    hipEventElapsedTime(&res.ms, ctx->ev[0], ctx->ev[1]);
    if (host[kAbort]) return fail(ctx, SWH_E_TIMEOUT, "strip wavefront wait expired");
    std::memcpy(&res.best, host + kResult, sizeof(BestCell));
    return SWH_OK;
}

}  // namespace

swh_status align_device(swh_ctx *ctx, const char *q_dev, int64_t qlen, const char *t_dev, int64_t tlen,
                        const Scoring &sc, int mode, hipStream_t st, swh_alignment *out, char *cigar,
                        int64_t cigar_cap, int64_t *cigar_len, swh_stats *stats)
{
    out->score = 0;
    out->flags = SWH_F_NONE;
    out->q_begin = out->q_end = out->t_begin = out->t_end = -1;
    if (cigar_len) *cigar_len = 0;
    if (cigar && cigar_cap > 0) cigar[0] = '\0';
    if (qlen == 0 || tlen == 0) return SWH_OK;

    const int R = pick_rows_per_lane(qlen);
    const int64_t qpad = ((qlen + 64 * R - 1) / (64 * R)) * 64 * R;
    const int64_t tpad = 64 * (sweep_blocks(tlen) + 3);
    swh_status s;
    if ((s = ensure(ctx, ctx->qc, (size_t)qpad, "query codes")) != SWH_OK) return s;
    if ((s = ensure(ctx, ctx->tc, (size_t)tpad, "target codes")) != SWH_OK) return s;
    if ((s = ensure(ctx, ctx->misc, kMiscWords * 4, "scratch words")) != SWH_OK) return s;
    if ((s = ensure(ctx, ctx->mat, 32 * 32, "matrix")) != SWH_OK) return s;
    if ((s = ensure(ctx, ctx->lut, 256, "symbol table")) != SWH_OK) return s;

    hipError_t e;
    static const int32_t init[kMiscWords] = {0, 0, INT32_MAX, INT32_MAX, 0, 0, 0, 0};
    if ((e = hipMemcpyAsync(ctx->misc.p, init, sizeof(init), hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(ctx->mat.p, sc.mat, (size_t)sc.asize * sc.asize, hipMemcpyHostToDevice, st)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(ctx->lut.p, sc.lut, 256, hipMemcpyHostToDevice, st)) != hipSuccess)
        return hip_fail(ctx, e, "hipMemcpyAsync(scoring)");
    int32_t *misc = (int32_t *)ctx->misc.p;
    const uint8_t pad = (uint8_t)sc.asize;
    if ((e = launch_encode(q_dev, qlen, (uint8_t *)ctx->qc.p, qpad, (const uint8_t *)ctx->lut.p, pad,
                           misc + kBadQ, st)) != hipSuccess ||
        (e = launch_encode(t_dev, tlen, (uint8_t *)ctx->tc.p, tpad, (const uint8_t *)ctx->lut.p, pad,
                           misc + kBadT, st)) != hipSuccess)
        return hip_fail(ctx, e, "encode kernel launch");
    int32_t bad[2];
    if ((e = hipMemcpyAsync(bad, misc + kBadQ, 8, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, "encode");
    if (bad[0] != INT32_MAX)
        return fail(ctx, SWH_E_ALPHABET, "query byte at position " + std::to_string(bad[0]) +
                                             " is not in the alphabet");
    if (bad[1] != INT32_MAX)
        return fail(ctx, SWH_E_ALPHABET, "target byte at position " + std::to_string(bad[1]) +
                                             " is not in the alphabet");

    // ---- resolution: forward local pass
    LocalPass fwd;
    if ((s = local_pass(ctx, (const uint8_t *)ctx->qc.p, qlen, (const uint8_t *)ctx->tc.p, tlen, sc, R, st, fwd)) !=
        SWH_OK)
        return s;
    if (stats) {
        stats->cells_forward = (double)qlen * (double)tlen;
        stats->ms_forward = fwd.ms;
    }
    out->score = fwd.best.score;
    if (fwd.best.score == 0) return SWH_OK;
    out->q_end = fwd.best.row - 1;
    out->t_end = fwd.best.col - 1;
    if (mode == SWH_MODE_SCORE) return SWH_OK;

    // ---- reverse local pass on the prefixes ending at the end cell
    const int64_t rn = out->q_end + 1, rm = out->t_end + 1;
    const int Rr = pick_rows_per_lane(rn);
    const int64_t rqpad = ((rn + 64 * Rr - 1) / (64 * Rr)) * 64 * Rr;
    const int64_t rtpad = 64 * (sweep_blocks(rm) + 3);
    if ((s = ensure(ctx, ctx->qr, (size_t)rqpad, "reversed query")) != SWH_OK) return s;
    if ((s = ensure(ctx, ctx->tr, (size_t)rtpad, "reversed target")) != SWH_OK) return s;
    if ((e = launch_reverse((const uint8_t *)ctx->qc.p, rn, (uint8_t *)ctx->qr.p, rqpad, pad, st)) != hipSuccess ||
        (e = launch_reverse((const uint8_t *)ctx->tc.p, rm, (uint8_t *)ctx->tr.p, rtpad, pad, st)) != hipSuccess)
        return hip_fail(ctx, e, "reverse kernel launch");
    LocalPass rev;
    if ((s = local_pass(ctx, (const uint8_t *)ctx->qr.p, rn, (const uint8_t *)ctx->tr.p, rm, sc, Rr, st, rev)) !=
        SWH_OK)
        return s;
    if (stats) stats->ms_reverse = rev.ms;
    if (rev.best.score != fwd.best.score)
        return fail(ctx, SWH_E_DEVICE, "reverse pass maximum " + std::to_string(rev.best.score) +
                                           " differs from the forward score " + std::to_string(fwd.best.score));
    out->q_begin = out->q_end - (rev.best.row - 1);
    out->t_begin = out->t_end - (rev.best.col - 1);
    if (mode == SWH_MODE_COORDS) return SWH_OK;

    // ---- reconstruction: linear-space traceback over the rectangle
    std::string cg;
    TracebackStats ts;
    if ((s = traceback(ctx, (const uint8_t *)ctx->qc.p + out->q_begin, out->q_end - out->q_begin + 1,
                       (const uint8_t *)ctx->tc.p + out->t_begin, out->t_end - out->t_begin + 1, sc,
                       fwd.best.score, st, cg, ts)) != SWH_OK)
        return s;
    if (stats) {
        stats->ms_traceback = ts.ms;
        stats->cells_traceback = ts.cells;
    }
    if (cigar_len) *cigar_len = (int64_t)cg.size();
    if (!cigar || (int64_t)cg.size() + 1 > cigar_cap)
        return fail(ctx, SWH_E_RANGE, "CIGAR needs " + std::to_string(cg.size() + 1) + " bytes");
    std::memcpy(cigar, cg.c_str(), cg.size() + 1);
    return SWH_OK;
}

}  // namespace swh
