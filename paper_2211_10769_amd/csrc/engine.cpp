// engine.cpp -- host orchestration of one pairwise alignment:
// encode -> forward local pass (score, end) -> reverse local pass on the
// reversed prefixes (start) -> linear-space traceback (CIGAR).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <string>

#include "bands.h"
#include "batch.h"
#include "context.h"
#include "engine.h"
#include "strips.h"
#include "tb_kernels.h"
#include "traceback.h"
#include "tune.h"

namespace swh {

namespace {

// misc buffer layout (int32 words)
enum { kBadQ = 0, kBadT = 1, kPick = 2, kMiscWords = 4 };   // kPick: 8-byte row pick key

struct LocalPass {
    BestCell best{0, 0, 0, 0};
    float ms = 0.f;
};

// Rows the pass keeps (band traceback): strip s with (s + 1 + phase) % every
// == 0 writes its last row to keep + slot * cols_padded(m).
struct KeepRows {
    Border *keep = nullptr;
    int32_t every = 0, phase = 0;
};

// One local score pass over encoded inputs already on the device.
swh_status local_pass(swh_ctx *ctx, const uint8_t *qc, int64_t n, const uint8_t *tc, int64_t m,
                      const Scoring &sc, StripShape shape, hipStream_t st, LocalPass &res, const KeepRows &kr = {},
                      int32_t prune = 0, bool int16 = false)
{
    const size_t bcount = (size_t)cols_padded(m);
    swh_status s;
    if ((s = ensure(ctx, ctx->border, bcount * sizeof(Border), "border buffer")) != SWH_OK) return s;
    hipError_t e;
    if ((e = hipMemsetAsync(ctx->border.p, 0, bcount * sizeof(Border), st)) != hipSuccess)
        return hip_fail(ctx, e, "hipMemsetAsync(border)");
    StripProblem sp{qc, n, tc, m, (Border *)ctx->border.p};
    sp.prune = prune;
    if (kr.keep) {
        sp.save = kr.keep;
        sp.save_stride = (int64_t)bcount;
        sp.save_every = kr.every;
        sp.save_phase = kr.phase;
    }
    std::vector<StripProblem> pr{sp};
    std::vector<BestCell> best;
    if ((s = run_strips(ctx, pr, sc, shape.R, true, st, &best, &res.ms, shape.waves, int16)) != SWH_OK) return s;
    res.best = best[0];
    if (int16) ++ctx->passes16;
    return SWH_OK;
}

// Band traceback (bands.cpp): in CIGAR mode both score passes keep rows for
// the traceback's first split; budget per pass, and the smallest number of
// kept rows worth keeping.
constexpr int64_t kKeepBudget = (int64_t)16 << 30;   // bytes of kept rows per pass
constexpr int64_t kKeepMinRows = 8;                  // fewer kept rows: not worth it

// Strips between kept rows for a forward pass over n x m, or 0 (plain traceback).
int band_stride(swh_ctx *ctx, int64_t n, int64_t m, int R)
{
    const int64_t H = 64 * (int64_t)R;
    const int64_t nstrips = (n + H - 1) / H;
    const int forced = ctx->opt.band_rows;
    if (forced < 0) return 0;
    if (forced > 0) return (int)std::max<int64_t>(1, (forced + H - 1) / H);
    if (nstrips < 32) return 0;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    const int64_t budget = std::min<int64_t>(std::min<int64_t>(kKeepBudget, (int64_t)(free_b / 4)),
                                             (int64_t)std::min<size_t>(cap_room(ctx) / 4, INT64_MAX));
    const int64_t row_bytes = cols_padded(m) * (int64_t)sizeof(Border);
    const int64_t max_rows = budget / row_bytes;
    if (max_rows < kKeepMinRows) return 0;
    return (int)std::max<int64_t>(1, (nstrips + max_rows - 1) / max_rows);
}

// Copy a finished CIGAR string out (SWH_E_RANGE when it does not fit).
swh_status put_cigar(swh_ctx *ctx, const std::string &cg, char *cigar, int64_t cigar_cap, int64_t *cigar_len)
{
    if (cigar_len) *cigar_len = (int64_t)cg.size();
    if (!cigar || (int64_t)cg.size() + 1 > cigar_cap)
        return fail(ctx, SWH_E_RANGE, "CIGAR needs " + std::to_string(cg.size() + 1) + " bytes");
    std::memcpy(cigar, cg.c_str(), cg.size() + 1);
    return SWH_OK;
}

// One global-mode pass of the semi-global and overlap forms: rows = the n
// row codes (read backwards from rc[n-1] when rstep < 0), columns = an
// optional pad column, then count codes cc[cstart + k * cstep]; top row of
// BorderInit kind `kind`; free_left: H = 0 left of the first column.  Leaves
// the last row in ctx->bborder (entry k = column k, the pad column first).
// Options of an edge pass: a fixed strip shape (R = 0: the rule), `lead`
// pass-through rows above the rows (their strip boundaries then fall `lead`
// rows lower), and kept rows.
struct EdgeOpts {
    StripShape shape{0, 0};
    int64_t lead = 0;
    KeepRows keep;
};

swh_status edge_pass(swh_ctx *ctx, const uint8_t *rc, int64_t n, int32_t rstep, const uint8_t *cc, int64_t cstart,
                     int64_t count, int32_t cstep, int32_t kind, bool pad_col, bool free_left, const Scoring &sc,
                     hipStream_t st, double &ms, const EdgeOpts &opt = {})
{
    const StripShape sh = opt.shape.R ? opt.shape : tuned_shape(ctx, n);
    const int64_t cols = count + (pad_col ? 1 : 0);
    const int64_t qpad = rows_padded(n + opt.lead, sh.R), tpad = cols_padded(cols);
    swh_status s;
    if ((s = ensure(ctx, ctx->bq, (size_t)qpad + 256, "edge pass row codes")) != SWH_OK ||
        (s = ensure(ctx, ctx->bt, (size_t)tpad + 256, "edge pass column codes")) != SWH_OK ||
        (s = ensure(ctx, ctx->bborder, sizeof(Border) * (size_t)tpad + 256, "edge pass border")) != SWH_OK ||
        (s = ensure(ctx, ctx->tb_misc, 2 * sizeof(GatherDesc), "gather table")) != SWH_OK ||
        (s = ensure(ctx, ctx->tb_leaf, sizeof(BorderInit), "border table")) != SWH_OK)
        return s;
    uint8_t *qp = (uint8_t *)ctx->bq.p, *tp = (uint8_t *)ctx->bt.p;
    Border *bp = (Border *)ctx->bborder.p;
    const GatherDesc gd[2] = {GatherDesc{rc, qp, rstep > 0 ? 0 : n - 1, n, qpad, rstep, (int32_t)opt.lead},
                              GatherDesc{cc, tp, cstart, count, tpad, cstep, pad_col ? 1 : 0}};
    const BorderInit bi{bp, nullptr, cols, tpad, kind, 0, 0, 0};
    hipError_t e;
    if ((e = hipMemcpyAsync(ctx->tb_misc.p, gd, sizeof(gd), hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(ctx->tb_leaf.p, &bi, sizeof(bi), hipMemcpyHostToDevice, st)) != hipSuccess)
        return hip_fail(ctx, e, "edge pass tables");
    if ((e = launch_gather((const GatherDesc *)ctx->tb_misc.p, 2, (uint8_t)sc.asize, st)) != hipSuccess ||
        (e = launch_border_init((const BorderInit *)ctx->tb_leaf.p, 1, sc.o, sc.e, st)) != hipSuccess)
        return hip_fail(ctx, e, "edge pass setup launch");
    // the host tables above are stack copies: finish the copies before returning
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(ctx, e, "edge pass setup");
    StripProblem sp{qp, n + opt.lead, tp, cols, bp};
    sp.free_left = free_left ? 1 : 0;
    sp.top_pass = (int32_t)opt.lead;
    if (opt.keep.keep) {
        sp.save = opt.keep.keep;
        sp.save_stride = tpad;
        sp.save_every = opt.keep.every;
        sp.save_phase = opt.keep.phase;
    }
    std::vector<StripProblem> pr{sp};
    float t = 0.f;
    if ((s = run_strips(ctx, pr, sc, sh.R, false, st, nullptr, &t, sh.waves)) != SWH_OK) return s;
    ms += t;
    return SWH_OK;
}

// launch_row_pick over the first `entries` records of ctx->bborder; returns the key.
swh_status pick_row(swh_ctx *ctx, int64_t entries, int32_t target, int32_t mode, hipStream_t st, uint64_t &key)
{
    uint64_t *slot = (uint64_t *)((int32_t *)ctx->misc.p + kPick);
    const uint64_t init = mode == 0 ? 0ull : ~0ull;
    key = init;
    if (entries <= 0) return SWH_OK;
    hipError_t e;
    if ((e = hipMemcpyAsync(slot, &init, sizeof(init), hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = launch_row_pick((const Border *)ctx->bborder.p, entries, target, mode, slot, st)) != hipSuccess ||
        (e = hipMemcpyAsync(&key, slot, sizeof(key), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, "row pick");
    return SWH_OK;
}

// mode-0 key -> (value, index)
inline int32_t key_value(uint64_t key) { return (int32_t)((uint32_t)(key >> 32) - (1u << 30)); }
inline int64_t key_index(uint64_t key) { return (int64_t)(0xFFFFFFFFu - (uint32_t)key); }


// Global alignment in CIGAR mode with band cuts (as for the local path): the
// forward global pass keeps every `every`-th strip's last row, a global pass
// over the reversed sequences from the corner keeps the matching rows (lead
// pass-through rows put its strip ends on them), and the crossings found at
// those rows cut the traceback into bands.  done = false (with S set when the
// forward pass ran) when there is nothing to gain or no room for the rows.
swh_status global_banded(swh_ctx *ctx, const uint8_t *qc, int64_t n, const uint8_t *tc, int64_t m, const Scoring &sc,
                         hipStream_t st, int32_t &S, std::string &cg, TracebackStats &ts, double &ms_f, double &ms_r,
                         int64_t &nbands, int64_t &retries, bool &done)
{
    done = false;
    const StripShape shape = tuned_shape(ctx, n);
    const int every = band_stride(ctx, n, m + 1, shape.R);
    if (every <= 0) return SWH_OK;
    BandKeep bk;
    const int64_t frecs = band_forward_layout(shape.R, every, n, m + 1, bk);
    if (bk.every <= 0) return SWH_OK;
    if (ensure(ctx, ctx->keep_f, (size_t)frecs * sizeof(Border), "kept rows") != SWH_OK) {
        ctx->err.clear();
        return SWH_OK;
    }
    swh_status s;
    hipError_t e;
    EdgeOpts fo;
    fo.shape = shape;
    fo.keep = KeepRows{(Border *)ctx->keep_f.p, bk.every, 0};
    if ((s = edge_pass(ctx, qc, n, 1, tc, 0, m, 1, 1, true, false, sc, st, ms_f, fo)) != SWH_OK) return s;
    Border corner;
    if ((e = hipMemcpyAsync(&corner, (const Border *)ctx->bborder.p + m, sizeof(Border), hipMemcpyDeviceToHost,
                            st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, "global score");
    S = corner.h;
    const int64_t rrecs = band_reverse_layout(n - 1, m, bk, shape.R);
    if (bk.kr < 1 || ensure(ctx, ctx->keep_r, (size_t)rrecs * sizeof(Border), "kept rows") != SWH_OK) {
        ctx->err.clear();
        return SWH_OK;
    }
    EdgeOpts ro;
    ro.shape = StripShape{bk.Rr, bk.Rr == shape.R ? shape.waves : 0};
    ro.lead = bk.lead;
    ro.keep = KeepRows{(Border *)ctx->keep_r.p, bk.every_r, bk.phase};
    if ((s = edge_pass(ctx, qc, n, -1, tc, m - 1, m, -1, 1, true, false, sc, st, ms_r, ro)) != SWH_OK) return s;
    if ((e = hipMemcpyAsync(&corner, (const Border *)ctx->bborder.p + m, sizeof(Border), hipMemcpyDeviceToHost,
                            st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, "global score");
    if (corner.h != S)
        return fail(ctx, SWH_E_DEVICE, "global reverse pass gives " + std::to_string(corner.h) +
                                           ", the forward pass " + std::to_string(S));
    // the records of both passes start with the boundary column (DP column 0)
    bk.keep_f = (const Border *)ctx->keep_f.p + 1;
    bk.keep_r = (const Border *)ctx->keep_r.p + 1;
    bk.global = true;
    swh_alignment al{};
    al.score = S;
    al.q_begin = 0;
    al.q_end = n - 1;
    al.t_begin = 0;
    al.t_end = m - 1;
    std::vector<CutDesc> cd;
    std::vector<int64_t> rows;
    std::vector<CutOut> co;
    band_cuts(bk, al, S, qc, tc, cd, rows);
    if ((s = resolve_cuts(ctx, sc, st, cd, co)) != SWH_OK) return s;
    TbInput tin{qc, n, tc, m, S};
    bands_from_cuts(co.data(), rows.data(), (int)co.size(), al, S, tin.bands);
    std::vector<std::string> cgs;
    s = traceback_batch(ctx, {tin}, sc, st, cgs, ts);
    if (s != SWH_OK && ts.inconsistent && !tin.bands.empty()) {
        // a band did not check out: the plain divide and conquer
        ++retries;
        ctx->err.clear();
        tin.bands.clear();
        ts = TracebackStats{};
        s = traceback_batch(ctx, {tin}, sc, st, cgs, ts);
    }
    if (s != SWH_OK) return s;
    nbands = retries ? 0 : (int64_t)tin.bands.size();
    cg.swap(cgs[0]);
    done = true;
    return SWH_OK;
}

}  // namespace

swh_status align_device(swh_ctx *ctx, const char *q_dev, int64_t qlen, const char *t_dev, int64_t tlen,
                        const Scoring &sc, int mode, hipStream_t st, swh_alignment *out, char *cigar,
                        int64_t cigar_cap, int64_t *cigar_len, swh_stats *stats)
{
    if (stats) {
        const uint32_t size = stats->struct_size;
        *stats = swh_stats{};
        stats->struct_size = size;
    }
    const bool global = (mode & SWH_GLOBAL) != 0;
    const bool semi = (mode & SWH_SEMIGLOBAL) != 0;
    const bool overlap = (mode & SWH_OVERLAP) != 0;
    mode &= ~(SWH_GLOBAL | SWH_SEMIGLOBAL | SWH_OVERLAP);
    out->score = 0;
    out->flags = SWH_F_NONE;
    out->q_begin = out->q_end = out->t_begin = out->t_end = -1;
    if (cigar_len) *cigar_len = 0;
    if (cigar && cigar_cap > 0) cigar[0] = '\0';
    if (global) {
        out->q_begin = qlen ? 0 : -1;
        out->q_end = qlen - 1;
        out->t_begin = tlen ? 0 : -1;
        out->t_end = tlen - 1;
        if (qlen == 0 || tlen == 0) {
            // one sequence against nothing: a single gap (or the empty alignment)
            const int64_t len = qlen + tlen;
            out->score = len ? -(int32_t)(sc.o + (len - 1) * (int64_t)sc.e) : 0;
            if (mode != SWH_MODE_CIGAR) return SWH_OK;
            const std::string cg = len ? std::to_string(len) + (qlen ? "I" : "D") : std::string();
            if (cigar_len) *cigar_len = (int64_t)cg.size();
            if (!cigar || (int64_t)cg.size() + 1 > cigar_cap)
                return fail(ctx, SWH_E_RANGE, "CIGAR needs " + std::to_string(cg.size() + 1) + " bytes");
            std::memcpy(cigar, cg.c_str(), cg.size() + 1);
            return SWH_OK;
        }
    }
    if (semi && qlen > 0) {
        out->q_begin = 0;
        out->q_end = qlen - 1;
        if (tlen == 0) {
            // nothing to align against: the whole query as one insertion run
            out->score = -(int32_t)(sc.o + (qlen - 1) * (int64_t)sc.e);
            if (mode != SWH_MODE_CIGAR) return SWH_OK;
            return put_cigar(ctx, std::to_string(qlen) + "I", cigar, cigar_cap, cigar_len);
        }
    }
    if (qlen == 0 || tlen == 0) return SWH_OK;

    StripShape shape = tuned_shape(ctx, qlen);
    // One pass of at most one strip per SIMD is bound by its chain of strips,
    // whose every step takes the strip's rows: 4 rows per lane while those
    // strips still fit in one round (10 kbp pair: forward 2.51 ms against 2.65
    // at 8; 250 kbp: 71.4 against 75.5 ms), unless a height is forced or tuned.
    if (shape.R == 8 && ctx->opt.rows == 0 && ctx->tune.empty() &&
        (qlen + 255) / 256 <= 4 * (int64_t)std::max(ctx->num_cu, 1))
        shape.R = 4;
    const int64_t qpad = rows_padded(qlen, 2 * shape.R);   // room for 16-bit strips of twice the height
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

    if (semi) {
        // ---- semi-global alignment (whole query, free target ends).  Forward:
        // G(0, j) = 0 over a pad column and the target, the last row gives the
        // score and the smallest end column; backward: the reversed query
        // against the target reversed from that end with both starts penalised,
        // the smallest column of the last row holding the score is the
        // largest start.
        const uint8_t *qc = (const uint8_t *)ctx->qc.p, *tc = (const uint8_t *)ctx->tc.p;
        double ms_f = 0.0, ms_r = 0.0;
        uint64_t key = 0;
        if ((s = edge_pass(ctx, qc, qlen, 1, tc, 0, tlen, 1, 4, true, false, sc, st, ms_f)) != SWH_OK ||
            (s = pick_row(ctx, tlen + 1, 0, 0, st, key)) != SWH_OK)
            return s;
        const int32_t S = key_value(key);
        const int64_t je = key_index(key);
        out->score = S;
        if (stats) {
            stats->cells_forward = (double)qlen * (double)(tlen + 1);
            stats->ms_forward = ms_f;
        }
        if (je < 0 || je > tlen) return fail(ctx, SWH_E_DEVICE, "semi-global end column out of range");
        if (je == 0) {
            // no target residue pays: the query as one insertion run
            if (mode != SWH_MODE_CIGAR) return SWH_OK;
            return put_cigar(ctx, std::to_string(qlen) + "I", cigar, cigar_cap, cigar_len);
        }
        out->t_end = je - 1;
        if (mode == SWH_MODE_SCORE) return SWH_OK;
        if ((s = edge_pass(ctx, qc, qlen, -1, tc, je - 1, je, -1, 1, true, false, sc, st, ms_r)) != SWH_OK ||
            (s = pick_row(ctx, je + 1, S, 1, st, key)) != SWH_OK)
            return s;
        if (stats) stats->ms_reverse = ms_r;
        if (key < 1 || key > (uint64_t)je)
            return fail(ctx, SWH_E_DEVICE, "semi-global backward pass does not reach the score " + std::to_string(S));
        out->t_begin = je - (int64_t)key;
        if (mode == SWH_MODE_COORDS) return SWH_OK;
        std::string cg;
        TracebackStats ts;
        if ((s = traceback(ctx, qc, qlen, tc + out->t_begin, out->t_end - out->t_begin + 1, sc, S, st, cg, ts)) !=
            SWH_OK)
            return s;
        if (stats) {
            stats->ms_traceback = ts.ms;
            stats->cells_traceback = ts.cells;
        }
        return put_cigar(ctx, cg, cigar, cigar_cap, cigar_len);
    }

    if (overlap) {
        // ---- overlap alignment (end gaps of both sequences free).  The last
        // row of the DP with both borders free, and its last column as the
        // last row of the same DP with the sequences swapped (transposed
        // scores); the end is the first border cell in row-major order holding
        // the maximum.  The start: the same two edges of the DP on the
        // reversed prefixes entered at its corner (both borders penalised).
        const uint8_t *qc = (const uint8_t *)ctx->qc.p, *tc = (const uint8_t *)ctx->tc.p;
        double ms_f = 0.0, ms_r = 0.0;
        uint64_t krow = 0, kcol = 0;
        if ((s = edge_pass(ctx, qc, qlen, 1, tc, 0, tlen, 1, 4, false, true, sc, st, ms_f)) != SWH_OK ||
            (s = pick_row(ctx, tlen, 0, 0, st, krow)) != SWH_OK ||          // G(n, 1..m)
            (s = set_matrix(ctx, sc, true, st)) != SWH_OK ||
            (s = edge_pass(ctx, tc, tlen, 1, qc, 0, qlen, 1, 4, false, true, sc, st, ms_f)) != SWH_OK ||
            (s = pick_row(ctx, qlen - 1, 0, 0, st, kcol)) != SWH_OK ||      // G(1..n-1, m)
            (s = set_matrix(ctx, sc, false, st)) != SWH_OK)
            return s;
        if (stats) {
            stats->cells_forward = 2.0 * (double)qlen * (double)tlen;
            stats->ms_forward = ms_f;
        }
        const int32_t srow = key_value(krow);
        const int32_t scol = qlen > 1 ? key_value(kcol) : INT32_MIN;
        const int32_t S = std::max(0, std::max(srow, scol));
        out->score = S;
        if (S == 0) return SWH_OK;   // only the empty overlap: no alignment
        const int64_t ie = scol == S ? key_index(kcol) + 1 : qlen;
        const int64_t je = scol == S ? tlen : key_index(krow) + 1;
        if (ie < 1 || ie > qlen || je < 1 || je > tlen)
            return fail(ctx, SWH_E_DEVICE, "overlap end cell out of range");
        out->q_end = ie - 1;
        out->t_end = je - 1;
        if (mode == SWH_MODE_SCORE) return SWH_OK;
        uint64_t kr = 0, kc = 0;
        if ((s = set_matrix(ctx, sc, true, st)) != SWH_OK ||
            (s = edge_pass(ctx, tc, je, -1, qc, ie - 1, ie, -1, 1, true, false, sc, st, ms_r)) != SWH_OK ||
            (s = pick_row(ctx, ie, S, 1, st, kr)) != SWH_OK ||              // G'(1..ie-1, je)
            (s = set_matrix(ctx, sc, false, st)) != SWH_OK ||
            (s = edge_pass(ctx, qc, ie, -1, tc, je - 1, je, -1, 1, true, false, sc, st, ms_r)) != SWH_OK ||
            (s = pick_row(ctx, je + 1, S, 1, st, kc)) != SWH_OK)            // G'(ie, 1..je)
            return s;
        if (stats) stats->ms_reverse = ms_r;
        int64_t is, js;
        if (kr >= 1 && kr < (uint64_t)ie) {
            is = ie - (int64_t)kr;
            js = 0;
        } else if (kc >= 1 && kc <= (uint64_t)je) {
            is = 0;
            js = je - (int64_t)kc;
        } else {
            return fail(ctx, SWH_E_DEVICE, "overlap backward passes do not reach the score " + std::to_string(S));
        }
        out->q_begin = is;
        out->t_begin = js;
        if (mode == SWH_MODE_COORDS) return SWH_OK;
        std::string cg;
        TracebackStats ts;
        if ((s = traceback(ctx, qc + is, ie - is, tc + js, je - js, sc, S, st, cg, ts)) != SWH_OK) return s;
        if (stats) {
            stats->ms_traceback = ts.ms;
            stats->cells_traceback = ts.cells;
        }
        return put_cigar(ctx, cg, cigar, cigar_cap, cigar_len);
    }

    if (global && mode == SWH_MODE_CIGAR && ctx->opt.band_rows >= 0) {
        std::string cg;
        TracebackStats ts;
        int32_t S = 0;
        double ms_f = 0.0, ms_r = 0.0;
        int64_t nbands = 0, retries = 0;
        bool done = false;
        const auto t0 = std::chrono::steady_clock::now();
        if ((s = global_banded(ctx, (const uint8_t *)ctx->qc.p, qlen, (const uint8_t *)ctx->tc.p, tlen, sc, st, S, cg,
                               ts, ms_f, ms_r, nbands, retries, done)) != SWH_OK)
            return s;
        if (done) {
            out->score = S;
            if (stats) {
                stats->cells_forward = (double)qlen * (double)tlen;
                stats->ms_forward = ms_f;
                stats->ms_reverse = ms_r;
                stats->ms_traceback =
                    std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() - ms_f -
                    ms_r;
                stats->cells_traceback = ts.cells;
                stats->traceback_bands = nbands;
                stats->traceback_retries = retries;
            }
            return put_cigar(ctx, cg, cigar, cigar_cap, cigar_len);
        }
    }
    if (global) {
        // ---- global alignment: the forward pass in global mode gives G(n, m),
        // the reconstruction is the divide and conquer over the whole matrix
        std::vector<int32_t> gs;
        double ms = 0.0;
        if ((s = global_scores(ctx, {PairPass{(const uint8_t *)ctx->qc.p, qlen, (const uint8_t *)ctx->tc.p, tlen, 1}},
                               sc, st, gs, ms)) != SWH_OK)
            return s;
        out->score = gs[0];
        if (stats) {
            stats->cells_forward = (double)qlen * (double)tlen;
            stats->ms_forward = ms;
        }
        if (mode != SWH_MODE_CIGAR) return SWH_OK;
        std::string cg;
        TracebackStats ts;
        if ((s = traceback(ctx, (const uint8_t *)ctx->qc.p, qlen, (const uint8_t *)ctx->tc.p, tlen, sc, gs[0], st, cg,
                           ts)) != SWH_OK)
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

    // ---- resolution: forward local pass (keeping rows for the band traceback in
    // CIGAR mode), in packed 16-bit arithmetic when no cell can reach its limit
    // (the 16-bit kernel runs strips of two sub-strips of the nominal height; a
    // short pair keeps 512-row strips, as its 32-bit pass would).  A pass with
    // fewer strips than the GPU has SIMDs is bound by its dependency chain,
    // whose steps are shorter in 32 bits: 16 bits only for passes that fill
    // the GPU, unless the option asks for them everywhere.
    const int R16 = shape.R == 8 && ctx->opt.rows == 0 ? 4 : shape.R;
    auto fills = [&](int64_t rows, int R) { return (rows + 64 * R - 1) / (64 * R) >= 4 * (int64_t)ctx->num_cu; };
    const bool f16 = never_saturates(qlen, tlen, sc) && int16_usable(ctx, sc, R16) &&
                     (ctx->opt.int16 == 2 || fills(qlen, R16));
    const StripShape fshape = f16 ? StripShape{R16, 0} : shape;
    BandKeep bk;
    KeepRows kfwd;
    {
        const int every = mode == SWH_MODE_CIGAR ? band_stride(ctx, qlen, tlen, fshape.R) : 0;
        const int64_t recs = band_forward_layout(fshape.R, every, qlen, tlen, bk);
        if (bk.every > 0) {
            if (ensure(ctx, ctx->keep_f, (size_t)recs * sizeof(Border), "kept rows") != SWH_OK) {
                bk.every = 0;
                ctx->err.clear();
            } else {
                bk.keep_f = (const Border *)ctx->keep_f.p;
                kfwd = KeepRows{(Border *)ctx->keep_f.p, bk.every, 0};
            }
        }
    }
    LocalPass fwd;
    if ((s = local_pass(ctx, (const uint8_t *)ctx->qc.p, qlen, (const uint8_t *)ctx->tc.p, tlen, sc, fshape, st, fwd,
                        kfwd, 0, f16)) != SWH_OK)
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

    // ---- reverse local pass on the prefixes ending at the end cell.  With kept
    // rows it runs with a strip height H that divides the distance C between the
    // forward kept rows and `lead` pad rows on top (all-zero rows of the local
    // DP, like the border) so that its strip boundaries fall on the rows the
    // cuts need: reversed strip s' ends at row q_end - (s'+1) H + 1 + lead,
    // which is x + 2 for the forward cut row x = k C - 1 when (s'+1) = T - k
    // every_r, T = (q_end + lead) / H, every_r = C / H.
    const int64_t rn = out->q_end + 1, rm = out->t_end + 1;
    // The reverse pass knows its maximum (the forward score) and is block
    // pruned; what remains is bound by its diagonal dependency chain, whose
    // steps are shortest at 8 rows per lane (long pair: 1.70 s against 2.41 s
    // at 20).  With kept rows the reverse strips must still end on the cut rows.
    const bool prune_rev = ctx->opt.prune != 0;
    const int64_t rrecs = band_reverse_layout(out->q_end, out->t_end, bk, prune_rev ? 8 : fshape.R);
    const StripShape rshape = bk.every > 0 ? StripShape{bk.Rr, bk.Rr == fshape.R ? fshape.waves : 0}
                              : (prune_rev && rn >= 512) ? StripShape{8, 0}
                                                         : tuned_shape(ctx, rn);
    const int64_t lead = bk.every > 0 ? bk.lead : 0;
    // the reverse pass's maximum is the forward score: 16 bits are exact below the limit
    const bool r16 = fwd.best.score < sat16_limit(sc.smax) && int16_usable(ctx, sc, rshape.R) &&
                     (ctx->opt.int16 == 2 || fills(rn + lead, rshape.R));
    const int64_t rqpad = rows_padded(rn + lead, r16 ? 2 * rshape.R : rshape.R);
    const int64_t rtpad = cols_padded(rm);
    if ((s = ensure(ctx, ctx->qr, (size_t)rqpad, "reversed query")) != SWH_OK) return s;
    if ((s = ensure(ctx, ctx->tr, (size_t)rtpad, "reversed target")) != SWH_OK) return s;
    if ((e = launch_reverse((const uint8_t *)ctx->qc.p, rn, (uint8_t *)ctx->qr.p, rqpad, pad, st, lead)) !=
            hipSuccess ||
        (e = launch_reverse((const uint8_t *)ctx->tc.p, rm, (uint8_t *)ctx->tr.p, rtpad, pad, st)) != hipSuccess)
        return hip_fail(ctx, e, "reverse kernel launch");
    KeepRows krev;
    if (bk.every > 0) {
        if (bk.kr < 1 || ensure(ctx, ctx->keep_r, (size_t)rrecs * sizeof(Border), "kept rows") != SWH_OK) {
            bk.every = 0;
            ctx->err.clear();
        } else {
            bk.keep_r = (const Border *)ctx->keep_r.p;
            krev = KeepRows{(Border *)ctx->keep_r.p, bk.every_r, bk.phase};
        }
    }
    const int32_t prune = prune_rev ? fwd.best.score : 0;
    LocalPass rev;
    if ((s = local_pass(ctx, (const uint8_t *)ctx->qr.p, rn + lead, (const uint8_t *)ctx->tr.p, rm, sc, rshape, st,
                        rev, krev, prune, r16)) != SWH_OK)
        return s;
    if (stats) stats->ms_reverse = rev.ms;
    if (rev.best.score != fwd.best.score)
        return fail(ctx, SWH_E_DEVICE, "reverse pass maximum " + std::to_string(rev.best.score) +
                                           " differs from the forward score " + std::to_string(fwd.best.score));
    out->q_begin = out->q_end - (rev.best.row - lead - 1);
    out->t_begin = out->t_end - (rev.best.col - 1);
    if (mode == SWH_MODE_COORDS) return SWH_OK;

    // ---- reconstruction: linear-space traceback over the rectangle, cut into
    // bands at the kept rows where the path's crossing is known
    std::string cg;
    TracebackStats ts;
    TbInput tin{(const uint8_t *)ctx->qc.p + out->q_begin, out->q_end - out->q_begin + 1,
                (const uint8_t *)ctx->tc.p + out->t_begin, out->t_end - out->t_begin + 1, fwd.best.score};
    int64_t retries = 0;
    const auto t_cut = std::chrono::steady_clock::now();
    if (bk.every > 0) {
        std::vector<CutDesc> cd;
        std::vector<int64_t> rows;
        std::vector<CutOut> co;
        band_cuts(bk, *out, fwd.best.score, (const uint8_t *)ctx->qc.p, (const uint8_t *)ctx->tc.p, cd, rows);
        if ((s = resolve_cuts(ctx, sc, st, cd, co)) != SWH_OK) return s;
        bands_from_cuts(co.data(), rows.data(), (int)co.size(), *out, fwd.best.score, tin.bands);
    }
    const double cut_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_cut).count();
    std::vector<std::string> cgs;
    s = traceback_batch(ctx, {tin}, sc, st, cgs, ts);
    if (s != SWH_OK && ts.inconsistent && !tin.bands.empty()) {
        // a band did not check out: the plain divide and conquer over the rectangle
        ++retries;
        ctx->err.clear();
        tin.bands.clear();
        ts = TracebackStats{};
        s = traceback_batch(ctx, {tin}, sc, st, cgs, ts);
    }
    if (s != SWH_OK) return s;
    cg.swap(cgs[0]);
    if (stats) {
        stats->ms_traceback = ts.ms + cut_ms;
        stats->cells_traceback = ts.cells;
        stats->traceback_bands = retries ? 0 : (int64_t)tin.bands.size();
        stats->traceback_retries = retries;
    }
    if (cigar_len) *cigar_len = (int64_t)cg.size();
    if (!cigar || (int64_t)cg.size() + 1 > cigar_cap)
        return fail(ctx, SWH_E_RANGE, "CIGAR needs " + std::to_string(cg.size() + 1) + " bytes");
    std::memcpy(cigar, cg.c_str(), cg.size() + 1);
    return SWH_OK;
}

}  // namespace swh
