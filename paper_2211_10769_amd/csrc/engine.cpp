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
#include "strips.h"
#include "traceback.h"
#include "tune.h"

namespace swh {

namespace {

// misc buffer layout (int32 words)
enum { kBadQ = 0, kBadT = 1, kMiscWords = 4 };

struct LocalPass {
    BestCell best{0, 0, 0, 0};
    float ms = 0.f;
};

// One local score pass over encoded inputs already on the device.
swh_status local_pass(swh_ctx *ctx, const uint8_t *qc, int64_t n, const uint8_t *tc, int64_t m,
                      const Scoring &sc, StripShape shape, hipStream_t st, LocalPass &res)
{
    const size_t bcount = (size_t)cols_padded(m);
    swh_status s;
    if ((s = ensure(ctx, ctx->border, bcount * sizeof(Border), "border buffer")) != SWH_OK) return s;
    hipError_t e;
    if ((e = hipMemsetAsync(ctx->border.p, 0, bcount * sizeof(Border), st)) != hipSuccess)
        return hip_fail(ctx, e, "hipMemsetAsync(border)");
    std::vector<StripProblem> pr{{qc, n, tc, m, (Border *)ctx->border.p}};
    std::vector<BestCell> best;
    if ((s = run_strips(ctx, pr, sc, shape.R, true, st, &best, &res.ms, shape.waves)) != SWH_OK) return s;
    res.best = best[0];
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

    const StripShape shape = tuned_shape(ctx, qlen);
    const int64_t qpad = rows_padded(qlen, shape.R);
    const int64_t tpad = cols_padded(tlen);
    swh_status s;
    if ((s = ensure(ctx, ctx->qc, (size_t)qpad, "query codes")) != SWH_OK) return s;
    if ((s = ensure(ctx, ctx->tc, (size_t)tpad, "target codes")) != SWH_OK) return s;
    if ((s = ensure(ctx, ctx->misc, kMiscWords * 4, "scratch words")) != SWH_OK) return s;
    if ((s = ensure(ctx, ctx->mat, 32 * 32, "matrix")) != SWH_OK) return s;
    if ((s = ensure(ctx, ctx->lut, 256, "symbol table")) != SWH_OK) return s;

    hipError_t e;
    static const int32_t init[kMiscWords] = {INT32_MAX, INT32_MAX, 0, 0};
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
    if ((s = local_pass(ctx, (const uint8_t *)ctx->qc.p, qlen, (const uint8_t *)ctx->tc.p, tlen, sc, shape, st, fwd)) !=
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
    const StripShape rshape = tuned_shape(ctx, rn);
    const int64_t rqpad = rows_padded(rn, rshape.R);
    const int64_t rtpad = cols_padded(rm);
    if ((s = ensure(ctx, ctx->qr, (size_t)rqpad, "reversed query")) != SWH_OK) return s;
    if ((s = ensure(ctx, ctx->tr, (size_t)rtpad, "reversed target")) != SWH_OK) return s;
    if ((e = launch_reverse((const uint8_t *)ctx->qc.p, rn, (uint8_t *)ctx->qr.p, rqpad, pad, st)) != hipSuccess ||
        (e = launch_reverse((const uint8_t *)ctx->tc.p, rm, (uint8_t *)ctx->tr.p, rtpad, pad, st)) != hipSuccess)
        return hip_fail(ctx, e, "reverse kernel launch");
    LocalPass rev;
    if ((s = local_pass(ctx, (const uint8_t *)ctx->qr.p, rn, (const uint8_t *)ctx->tr.p, rm, sc, rshape, st, rev)) !=
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
