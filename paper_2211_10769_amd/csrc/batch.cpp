// batch.cpp -- many independent pairwise alignments in few launches.
//
// All pairs of a call share each phase: one forward local pass over every
// pair (the strip kernel's problem table, strips of all pairs in one ticket
// space, the most expensive pairs first), one reverse pass over the reversed
// prefixes of every pair with a positive score, and one level-synchronous
// traceback whose levels hold the subproblems of all pairs.  Pairs are cut
// into chunks only to bound the device memory of one launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "bands.h"
#include "batch.h"
#include "context.h"
#include "strips.h"
#include "tb_kernels.h"
#include "traceback.h"
#include "tune.h"

namespace swh {

namespace {

// device bytes of the per-pair copies and border rows of one launch
constexpr int64_t kChunkBytes = (int64_t)3 << 30;
// total rectangle columns of one traceback batch (arena: ~9 bytes per column)
constexpr int64_t kTracebackCols = (int64_t)64 << 20;
// band traceback of a batch: rows between kept rows, and the device bytes the
// kept rows of one group of pairs may take (both passes; an eighth of the free
// memory caps it, 35 GiB on a 288 GB device).  Every group is one launch per
// score pass, whose last strips leave SIMDs idle: 200,000 read pairs in 19
// groups at 16 GiB, forward 2.04 s, reverse 0.81 s; in 9 at 35 GiB, 1.92 s and
// 0.72 s, the traceback unchanged (0.87 s)
constexpr int64_t kBatchBandRows = 512;
constexpr int64_t kBatchKeepBytes = (int64_t)64 << 30;

template <typename T>
swh_status upload(swh_ctx *ctx, DevBuf &buf, const std::vector<T> &v, hipStream_t st, const char *what)
{
    swh_status s = ensure(ctx, buf, v.size() * sizeof(T) + 16, what);
    if (s != SWH_OK) return s;
    hipError_t e = hipMemcpyAsync(buf.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(ctx, e, what);
    return SWH_OK;
}

}  // namespace

swh_status score_passes(swh_ctx *ctx, const std::vector<PairPass> &ps, const Scoring &sc, hipStream_t st,
                        std::vector<BestCell> &best, double &ms_total)
{
    const size_t np = ps.size();
    best.assign(np, BestCell{0, 0, 0, 0});
    std::vector<StripShape> sh(np);
    std::vector<char> w16(np, 0);
    for (size_t i = 0; i < np; ++i) {
        sh[i] = ps[i].R ? StripShape{ps[i].R, ps[i].waves} : tuned_shape(ctx, ps[i].n);
        w16[i] = ps[i].int16 && int16_usable(ctx, sc, sh[i].R);
        if (w16[i]) sh[i].waves = 0;   // the rule for the 16-bit kernel's strips
    }
    auto same = [&](size_t a, size_t b) {
        return sh[a].R == sh[b].R && sh[a].waves == sh[b].waves && w16[a] == w16[b];
    };
    // by precision and strip shape, then most expensive first
    std::vector<size_t> order(np);
    std::iota(order.begin(), order.end(), (size_t)0);
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
        if (w16[a] != w16[b]) return w16[a] > w16[b];
        if (sh[a].R != sh[b].R) return sh[a].R > sh[b].R;
        if (sh[a].waves != sh[b].waves) return sh[a].waves > sh[b].waves;
        return (double)ps[a].n * (double)ps[a].m > (double)ps[b].n * (double)ps[b].m;
    });
    const uint8_t pad = (uint8_t)sc.asize;
    size_t k = 0;
    while (k < np) {
        while (k < np && (ps[order[k]].n == 0 || ps[order[k]].m == 0)) ++k;
        if (k == np) break;
        const size_t lead = order[k];
        const int Rk = sh[lead].R;
        const int Rpad = w16[lead] ? 2 * Rk : Rk;   // the 16-bit kernel reads rows of strips twice as tall
        // a chunk: one strip shape, bounded bytes
        size_t end = k;
        int64_t bytes = 0, nb = 0, nq = 0, nt = 0;
        while (end < np && same(order[end], lead)) {
            const PairPass &p = ps[order[end]];
            if (p.n == 0 || p.m == 0) {
                ++end;
                continue;
            }
            const int64_t b = rows_padded(p.n + p.lead, Rpad) + cols_padded(p.m) * (1 + (int64_t)sizeof(Border));
            if (bytes && bytes + b > kChunkBytes) break;
            bytes += b;
            nq += rows_padded(p.n + p.lead, Rpad);
            nt += cols_padded(p.m);
            nb += cols_padded(p.m);
            ++end;
        }
        swh_status s;
        if ((s = ensure(ctx, ctx->bq, (size_t)nq + 256, "batch row codes")) != SWH_OK ||
            (s = ensure(ctx, ctx->bt, (size_t)nt + 256, "batch column codes")) != SWH_OK ||
            (s = ensure(ctx, ctx->bborder, sizeof(Border) * (size_t)nb + 256, "batch borders")) != SWH_OK)
            return s;
        std::vector<GatherDesc> gd;
        std::vector<StripProblem> probs;
        std::vector<size_t> idx;
        uint8_t *qp = (uint8_t *)ctx->bq.p, *tp = (uint8_t *)ctx->bt.p;
        Border *bp = (Border *)ctx->bborder.p;
        for (size_t i = k; i < end; ++i) {
            const PairPass &p = ps[order[i]];
            if (p.n == 0 || p.m == 0) continue;
            const int64_t qpad = rows_padded(p.n + p.lead, Rpad), tpad = cols_padded(p.m);
            gd.push_back(GatherDesc{p.q, qp, 0, p.n, qpad, p.step, (int32_t)p.lead});
            gd.push_back(GatherDesc{p.t, tp, 0, p.m, tpad, p.step, 0});
            StripProblem sp{qp, p.n + p.lead, tp, p.m, bp};
            sp.prune = p.prune;
            if (p.keep) {
                sp.save = p.keep;
                sp.save_stride = tpad;
                sp.save_every = p.every;
                sp.save_phase = p.phase;
            }
            probs.push_back(sp);
            idx.push_back(order[i]);
            qp += qpad;
            tp += tpad;
            bp += tpad;
        }
        hipError_t e;
        if ((s = upload(ctx, ctx->tb_misc, gd, st, "gather table")) != SWH_OK) return s;
        if ((e = launch_gather((const GatherDesc *)ctx->tb_misc.p, (int32_t)gd.size(), pad, st)) != hipSuccess ||
            (e = hipMemsetAsync(ctx->bborder.p, 0, sizeof(Border) * (size_t)nb, st)) != hipSuccess)
            return hip_fail(ctx, e, "batch setup");
        std::vector<BestCell> b;
        float ms = 0.f;
        const bool i16 = w16[lead] != 0;
        if ((s = run_strips(ctx, probs, sc, Rk, true, st, &b, &ms, sh[lead].waves, i16)) != SWH_OK) return s;
        ms_total += ms;
        for (size_t i = 0; i < idx.size(); ++i) best[idx[i]] = b[i];
        if (i16) ctx->passes16 += (int64_t)idx.size();
        k = end;
    }
    // 16-bit passes whose maximum reached the limit may have saturated: again in
    // 32 bits, same strip height and kept rows
    const int32_t lim = sat16_limit(sc.smax);
    std::vector<PairPass> redo;
    std::vector<size_t> ridx;
    for (size_t i = 0; i < np; ++i)
        if (w16[i] && best[i].score >= lim) {
            PairPass p = ps[i];
            p.R = sh[i].R;
            p.waves = 0;
            p.int16 = false;
            redo.push_back(p);
            ridx.push_back(i);
        }
    if (!redo.empty()) {
        std::vector<BestCell> b;
        swh_status s = score_passes(ctx, redo, sc, st, b, ms_total);
        if (s != SWH_OK) return s;
        for (size_t j = 0; j < ridx.size(); ++j) best[ridx[j]] = b[j];
        ctx->saturated16 += (int64_t)redo.size();
    }
    return SWH_OK;
}

swh_status edge_scores(swh_ctx *ctx, const std::vector<PairPass> &ps, int32_t kind, const std::vector<RowPick> &picks,
                       const Scoring &sc, hipStream_t st, std::vector<uint64_t> &keys, double &ms_total, bool pad_col,
                       bool free_left)
{
    const int64_t pc = pad_col ? 1 : 0;
    const size_t np = ps.size();
    keys.assign(np, 0);
    std::vector<StripShape> sh(np);
    for (size_t i = 0; i < np; ++i) sh[i] = tuned_shape(ctx, ps[i].n);
    std::vector<size_t> order(np);
    std::iota(order.begin(), order.end(), (size_t)0);
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
        if (sh[a].R != sh[b].R) return sh[a].R > sh[b].R;
        if (sh[a].waves != sh[b].waves) return sh[a].waves > sh[b].waves;
        return (double)ps[a].n * (double)ps[a].m > (double)ps[b].n * (double)ps[b].m;
    });
    const uint8_t pad = (uint8_t)sc.asize;
    size_t k = 0;
    while (k < np) {
        const size_t lead = order[k];
        const int Rk = sh[lead].R;
        size_t end = k;
        int64_t bytes = 0, nq = 0, nt = 0;
        while (end < np && sh[order[end]].R == Rk && sh[order[end]].waves == sh[lead].waves) {
            const PairPass &p = ps[order[end]];
            const int64_t b = rows_padded(p.n, Rk) + cols_padded(p.m + pc) * (1 + (int64_t)sizeof(Border));
            if (bytes && bytes + b > kChunkBytes) break;
            bytes += b;
            nq += rows_padded(p.n, Rk);
            nt += cols_padded(p.m + pc);
            ++end;
        }
        const size_t nc = end - k;
        swh_status s;
        if ((s = ensure(ctx, ctx->bq, (size_t)nq + 256, "batch row codes")) != SWH_OK ||
            (s = ensure(ctx, ctx->bt, (size_t)nt + 256, "batch column codes")) != SWH_OK ||
            (s = ensure(ctx, ctx->bborder, sizeof(Border) * (size_t)nt + 256, "batch borders")) != SWH_OK ||
            (s = ensure(ctx, ctx->gscores, sizeof(uint64_t) * nc + 256, "row keys")) != SWH_OK)
            return s;
        std::vector<GatherDesc> gd;
        std::vector<BorderInit> bi;
        std::vector<StripProblem> probs;
        std::vector<RowPickDesc> rd;
        uint8_t *qp = (uint8_t *)ctx->bq.p, *tp = (uint8_t *)ctx->bt.p;
        Border *bp = (Border *)ctx->bborder.p;
        for (size_t i = k; i < end; ++i) {
            const PairPass &p = ps[order[i]];
            const RowPick &pk = picks[order[i]];
            const int64_t qpad = rows_padded(p.n, Rk), tpad = cols_padded(p.m + pc);
            gd.push_back(GatherDesc{p.q, qp, 0, p.n, qpad, p.step, 0});
            // with a pad column first, column 0 is the border (DP column 0)
            gd.push_back(GatherDesc{p.t, tp, 0, p.m, tpad, p.step, (int32_t)pc});
            bi.push_back(BorderInit{bp, nullptr, p.m + pc, tpad, kind, 0, 0, 0});
            StripProblem sp{qp, p.n, tp, p.m + pc, bp};
            sp.free_left = free_left ? 1 : 0;
            probs.push_back(sp);
            rd.push_back(RowPickDesc{bp + pk.first, pk.count, pk.target, pk.mode});
            qp += qpad;
            tp += tpad;
            bp += tpad;
        }
        hipError_t e;
        if ((s = upload(ctx, ctx->tb_misc, gd, st, "gather table")) != SWH_OK) return s;
        if ((e = launch_gather((const GatherDesc *)ctx->tb_misc.p, (int32_t)gd.size(), pad, st)) != hipSuccess)
            return hip_fail(ctx, e, "gather launch");
        if ((s = upload(ctx, ctx->tb_leaf, bi, st, "border table")) != SWH_OK) return s;
        if ((e = launch_border_init((const BorderInit *)ctx->tb_leaf.p, (int32_t)bi.size(), sc.o, sc.e, st)) !=
            hipSuccess)
            return hip_fail(ctx, e, "border init launch");
        // the tables above are read by launches already queued on st before
        // the buffers are reused: synchronise before run_strips rewrites them
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(ctx, e, "edge pass setup");
        float ms = 0.f;
        if ((s = run_strips(ctx, probs, sc, Rk, false, st, nullptr, &ms, sh[lead].waves)) != SWH_OK) return s;
        ms_total += ms;
        if ((s = upload(ctx, ctx->tb_misc, rd, st, "row pick table")) != SWH_OK) return s;
        std::vector<uint64_t> res(nc);
        if ((e = launch_row_pick_multi((const RowPickDesc *)ctx->tb_misc.p, (int32_t)rd.size(),
                                       (uint64_t *)ctx->gscores.p, st)) != hipSuccess ||
            (e = hipMemcpyAsync(res.data(), ctx->gscores.p, sizeof(uint64_t) * nc, hipMemcpyDeviceToHost, st)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess)
            return hip_fail(ctx, e, "row pick");
        for (size_t i = k; i < end; ++i) keys[order[i]] = res[i - k];
        k = end;
    }
    return SWH_OK;
}

swh_status set_matrix(swh_ctx *ctx, const Scoring &sc, bool transposed, hipStream_t st)
{
    int8_t m[32 * 32];
    const int A = sc.asize;
    for (int x = 0; x < A; ++x)
        for (int y = 0; y < A; ++y) m[x * A + y] = transposed ? sc.mat[y * A + x] : sc.mat[x * A + y];
    hipError_t e;
    if ((e = hipMemcpyAsync(ctx->mat.p, m, (size_t)A * A, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, "substitution table");
    return SWH_OK;
}

swh_status global_scores(swh_ctx *ctx, const std::vector<PairPass> &ps, const Scoring &sc, hipStream_t st,
                         std::vector<int32_t> &scores, double &ms_total)
{
    // G(n, m) is the last row's record of column m: a pick over that entry alone
    std::vector<RowPick> picks(ps.size());
    for (size_t i = 0; i < ps.size(); ++i) picks[i] = RowPick{ps[i].m, 1, 0, 0};
    std::vector<uint64_t> keys;
    swh_status s = edge_scores(ctx, ps, 1, picks, sc, st, keys, ms_total);
    if (s != SWH_OK) return s;
    scores.resize(ps.size());
    for (size_t i = 0; i < ps.size(); ++i) scores[i] = row_key_value(keys[i]);
    return SWH_OK;
}

swh_status align_batch(swh_ctx *ctx, int64_t npairs, const char *q_cat, const int64_t *q_off, const char *t_cat,
                       const int64_t *t_off, const Scoring &sc, int mode, swh_alignment *out, char *cigar_cat,
                       int64_t cigar_cap, int64_t *cigar_off, swh_stats *stats, bool dev)
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
    for (int64_t i = 0; i < npairs; ++i) {
        out[i].score = 0;
        out[i].flags = SWH_F_NONE;
        out[i].q_begin = out[i].q_end = out[i].t_begin = out[i].t_end = -1;
    }
    if (mode == SWH_MODE_CIGAR && cigar_off)
        for (int64_t i = 0; i <= npairs; ++i) cigar_off[i] = 0;
    if (npairs == 0) return SWH_OK;
    hipStream_t st = ctx->own_stream;
    const int64_t qbase = q_off[0], tbase = t_off[0];
    const int64_t qtot = q_off[npairs] - qbase, ttot = t_off[npairs] - tbase;
    swh_status s;
    hipError_t e;

    // ---- encode both concatenations once (host inputs through a device copy,
    // device inputs in place)
    if ((!dev && (s = ensure(ctx, ctx->qraw, (size_t)qtot + 1, "query copy")) != SWH_OK) ||
        (!dev && (s = ensure(ctx, ctx->traw, (size_t)ttot + 1, "target copy")) != SWH_OK) ||
        (s = ensure(ctx, ctx->qc, (size_t)qtot + 1, "query codes")) != SWH_OK ||
        (s = ensure(ctx, ctx->tc, (size_t)ttot + 1, "target codes")) != SWH_OK ||
        (s = ensure(ctx, ctx->misc, 64, "scratch words")) != SWH_OK ||
        (s = ensure(ctx, ctx->mat, 32 * 32, "matrix")) != SWH_OK ||
        (s = ensure(ctx, ctx->lut, 256, "symbol table")) != SWH_OK)
        return s;
    static const int32_t init[2] = {INT32_MAX, INT32_MAX};
    int32_t *misc = (int32_t *)ctx->misc.p;
    const uint8_t pad = (uint8_t)sc.asize;
    if ((!dev && qtot &&
         (e = hipMemcpyAsync(ctx->qraw.p, q_cat + qbase, (size_t)qtot, hipMemcpyHostToDevice, st)) != hipSuccess) ||
        (!dev && ttot &&
         (e = hipMemcpyAsync(ctx->traw.p, t_cat + tbase, (size_t)ttot, hipMemcpyHostToDevice, st)) != hipSuccess) ||
        (e = hipMemcpyAsync(misc, init, sizeof(init), hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(ctx->mat.p, sc.mat, (size_t)sc.asize * sc.asize, hipMemcpyHostToDevice, st)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(ctx->lut.p, sc.lut, 256, hipMemcpyHostToDevice, st)) != hipSuccess)
        return hip_fail(ctx, e, "batch upload");
    const char *qsrc = dev ? q_cat + qbase : (const char *)ctx->qraw.p;
    const char *tsrc = dev ? t_cat + tbase : (const char *)ctx->traw.p;
    if ((e = launch_encode(qsrc, qtot, (uint8_t *)ctx->qc.p, qtot, (const uint8_t *)ctx->lut.p, pad, misc, st)) !=
            hipSuccess ||
        (e = launch_encode(tsrc, ttot, (uint8_t *)ctx->tc.p, ttot, (const uint8_t *)ctx->lut.p, pad, misc + 1,
                           st)) != hipSuccess)
        return hip_fail(ctx, e, "encode kernel launch");
    int32_t bad[2];
    if ((e = hipMemcpyAsync(bad, misc, 8, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, "encode");
    for (int side = 0; side < 2; ++side) {
        if (bad[side] == INT32_MAX) continue;
        const int64_t *off = side ? t_off : q_off;
        const int64_t pos = bad[side] + (side ? tbase : qbase);
        const int64_t pr = (int64_t)(std::upper_bound(off, off + npairs + 1, pos) - off) - 1;
        return fail(ctx, SWH_E_ALPHABET, std::string(side ? "target" : "query") + " of pair " + std::to_string(pr) +
                                             ": byte at position " + std::to_string(pos - off[pr]) +
                                             " is not in the alphabet");
    }
    const uint8_t *qc = (const uint8_t *)ctx->qc.p, *tc = (const uint8_t *)ctx->tc.p;

    // ---- the pairs' passes, in groups: in CIGAR mode both score passes keep
    // rows for the band traceback (bands.cpp), and a group is sized so that
    // its kept rows fit the budget; otherwise one group holds every pair
    std::vector<PairPass> ps((size_t)npairs);
    double cells = 0.0;
    for (int64_t i = 0; i < npairs; ++i) {
        ps[i] = PairPass{qc + (q_off[i] - qbase), q_off[i + 1] - q_off[i], tc + (t_off[i] - tbase),
                         t_off[i + 1] - t_off[i], 1};
        cells += (double)ps[i].n * (double)ps[i].m;
    }
    if (stats) stats->cells_forward = cells;
    std::vector<std::string> cig((size_t)npairs);
    if (overlap) {
        // ---- overlap alignments (end gaps of both sequences free): the last
        // row of A x B and, from the swapped passes (transposed table), the
        // last column; the reversed corner-anchored passes give the start; then
        // the divide and conquer between start and end
        std::vector<PairPass> fr, fc;
        std::vector<RowPick> prow, pcol;
        std::vector<int64_t> fi;
        for (int64_t i = 0; i < npairs; ++i) {
            const int64_t n = ps[i].n, m = ps[i].m;
            if (n == 0 || m == 0) continue;   // only the empty overlap
            fr.push_back(ps[i]);
            prow.push_back(RowPick{0, m, 0, 0});                  // G(n, 1..m)
            fc.push_back(PairPass{ps[i].t, m, ps[i].q, n, 1});
            pcol.push_back(RowPick{0, n - 1, 0, 0});              // G(1..n-1, m)
            fi.push_back(i);
        }
        std::vector<uint64_t> krow, kcol;
        double ms_f = 0.0, ms_r = 0.0;
        if ((s = edge_scores(ctx, fr, 4, prow, sc, st, krow, ms_f, false, true)) != SWH_OK ||
            (s = set_matrix(ctx, sc, true, st)) != SWH_OK ||
            (s = edge_scores(ctx, fc, 4, pcol, sc, st, kcol, ms_f, false, true)) != SWH_OK ||
            (s = set_matrix(ctx, sc, false, st)) != SWH_OK)
            return s;
        std::vector<PairPass> rr, rc;
        std::vector<RowPick> prr, prc;
        std::vector<int64_t> ri;
        for (size_t j = 0; j < fi.size(); ++j) {
            const int64_t i = fi[j], n = ps[i].n, m = ps[i].m;
            const int32_t srow = row_key_value(krow[j]);
            const int32_t scol = n > 1 ? row_key_value(kcol[j]) : INT32_MIN;
            const int32_t S = std::max(0, std::max(srow, scol));
            out[i].score = S;
            if (S == 0) continue;
            const int64_t ie = scol == S ? row_key_index(kcol[j]) + 1 : n;
            const int64_t je = scol == S ? m : row_key_index(krow[j]) + 1;
            if (ie < 1 || ie > n || je < 1 || je > m) return fail(ctx, SWH_E_DEVICE, "overlap end cell out of range");
            out[i].q_end = ie - 1;
            out[i].t_end = je - 1;
            rr.push_back(PairPass{ps[i].t + je - 1, je, ps[i].q + ie - 1, ie, -1});   // swapped: G'(1..ie-1, je)
            prr.push_back(RowPick{0, ie, S, 1});
            rc.push_back(PairPass{ps[i].q + ie - 1, ie, ps[i].t + je - 1, je, -1});   // G'(ie, 1..je)
            prc.push_back(RowPick{0, je + 1, S, 1});
            ri.push_back(i);
        }
        if (stats) stats->ms_forward = ms_f;
        if (mode == SWH_MODE_SCORE) return SWH_OK;
        if ((s = set_matrix(ctx, sc, true, st)) != SWH_OK ||
            (s = edge_scores(ctx, rr, 1, prr, sc, st, krow, ms_r)) != SWH_OK ||
            (s = set_matrix(ctx, sc, false, st)) != SWH_OK ||
            (s = edge_scores(ctx, rc, 1, prc, sc, st, kcol, ms_r)) != SWH_OK)
            return s;
        for (size_t k = 0; k < ri.size(); ++k) {
            const int64_t i = ri[k], ie = out[i].q_end + 1, je = out[i].t_end + 1;
            if (krow[k] >= 1 && krow[k] < (uint64_t)ie) {
                out[i].q_begin = ie - (int64_t)krow[k];
                out[i].t_begin = 0;
            } else if (kcol[k] >= 1 && kcol[k] <= (uint64_t)je) {
                out[i].q_begin = 0;
                out[i].t_begin = je - (int64_t)kcol[k];
            } else {
                return fail(ctx, SWH_E_DEVICE, "overlap backward passes of pair " + std::to_string(i) +
                                                   " do not reach its score");
            }
        }
        if (stats) stats->ms_reverse = ms_r;
        if (mode != SWH_MODE_CIGAR) return SWH_OK;
        TracebackStats ts;
        size_t k = 0;
        while (k < ri.size()) {
            std::vector<TbInput> in;
            std::vector<int64_t> ids;
            int64_t cols = 0;
            while (k < ri.size()) {
                const int64_t i = ri[k], w = out[i].t_end - out[i].t_begin + 1;
                if (!in.empty() && cols + w > kTracebackCols) break;
                in.push_back(TbInput{ps[i].q + out[i].q_begin, out[i].q_end - out[i].q_begin + 1,
                                     ps[i].t + out[i].t_begin, w, out[i].score});
                ids.push_back(i);
                cols += w;
                ++k;
            }
            std::vector<std::string> cg;
            if ((s = traceback_batch(ctx, in, sc, st, cg, ts)) != SWH_OK) return s;
            for (size_t j = 0; j < ids.size(); ++j) cig[ids[j]].swap(cg[j]);
        }
        if (stats) {
            stats->ms_traceback = ts.ms;
            stats->cells_traceback = ts.cells;
        }
    } else if (semi) {
        // ---- semi-global alignments (whole query, free target ends): forward
        // passes from the free top border, the row pick gives the score and the
        // smallest end column; reverse passes from the end give the largest
        // start; then the divide and conquer over each read's rectangle
        std::vector<PairPass> fp;
        std::vector<RowPick> fpk;
        std::vector<int64_t> fi;
        for (int64_t i = 0; i < npairs; ++i) {
            const int64_t n = ps[i].n, m = ps[i].m;
            if (n == 0) continue;   // no query: score 0, no alignment
            out[i].q_begin = 0;
            out[i].q_end = n - 1;
            if (m == 0) {
                out[i].score = -(int32_t)(sc.o + (n - 1) * (int64_t)sc.e);
                cig[i] = std::to_string(n) + "I";
                continue;
            }
            fp.push_back(ps[i]);
            fpk.push_back(RowPick{0, m + 1, 0, 0});
            fi.push_back(i);
        }
        std::vector<uint64_t> keys;
        double ms_f = 0.0, ms_r = 0.0;
        if ((s = edge_scores(ctx, fp, 4, fpk, sc, st, keys, ms_f)) != SWH_OK) return s;
        std::vector<PairPass> rp;
        std::vector<RowPick> rpk;
        std::vector<int64_t> ri;
        for (size_t j = 0; j < fi.size(); ++j) {
            const int64_t i = fi[j], n = ps[i].n;
            const int32_t S = row_key_value(keys[j]);
            const int64_t je = row_key_index(keys[j]);
            if (je < 0 || je > ps[i].m) return fail(ctx, SWH_E_DEVICE, "semi-global end column out of range");
            out[i].score = S;
            if (je == 0) {
                cig[i] = std::to_string(n) + "I";
                continue;
            }
            out[i].t_end = je - 1;
            rp.push_back(PairPass{ps[i].q + n - 1, n, ps[i].t + je - 1, je, -1});
            rpk.push_back(RowPick{0, je + 1, S, 1});
            ri.push_back(i);
        }
        if (stats) stats->ms_forward = ms_f;
        if (mode == SWH_MODE_SCORE) return SWH_OK;
        if ((s = edge_scores(ctx, rp, 1, rpk, sc, st, keys, ms_r)) != SWH_OK) return s;
        for (size_t k = 0; k < ri.size(); ++k) {
            const int64_t i = ri[k], je = out[i].t_end + 1;
            if (keys[k] < 1 || keys[k] > (uint64_t)je)
                return fail(ctx, SWH_E_DEVICE, "semi-global backward pass of pair " + std::to_string(i) +
                                                   " does not reach its score");
            out[i].t_begin = je - (int64_t)keys[k];
        }
        if (stats) stats->ms_reverse = ms_r;
        if (mode != SWH_MODE_CIGAR) return SWH_OK;
        TracebackStats ts;
        size_t k = 0;
        while (k < ri.size()) {
            std::vector<TbInput> in;
            std::vector<int64_t> ids;
            int64_t cols = 0;
            while (k < ri.size()) {
                const int64_t i = ri[k], w = out[i].t_end - out[i].t_begin + 1;
                if (!in.empty() && cols + w > kTracebackCols) break;
                in.push_back(TbInput{ps[i].q, ps[i].n, ps[i].t + out[i].t_begin, w, out[i].score});
                ids.push_back(i);
                cols += w;
                ++k;
            }
            std::vector<std::string> cg;
            if ((s = traceback_batch(ctx, in, sc, st, cg, ts)) != SWH_OK) return s;
            for (size_t j = 0; j < ids.size(); ++j) cig[ids[j]].swap(cg[j]);
        }
        if (stats) {
            stats->ms_traceback = ts.ms;
            stats->cells_traceback = ts.cells;
        }
    } else if (global) {
        // ---- global alignments: G(n, m) per pair, then the plain divide and
        // conquer over each whole matrix (an empty side: a single gap)
        std::vector<PairPass> gp;
        std::vector<int64_t> gi;
        for (int64_t i = 0; i < npairs; ++i) {
            out[i].q_begin = ps[i].n ? 0 : -1;
            out[i].q_end = ps[i].n - 1;
            out[i].t_begin = ps[i].m ? 0 : -1;
            out[i].t_end = ps[i].m - 1;
            if (ps[i].n && ps[i].m) {
                gp.push_back(ps[i]);
                gi.push_back(i);
                continue;
            }
            const int64_t len = ps[i].n + ps[i].m;
            out[i].score = len ? -(int32_t)(sc.o + (len - 1) * (int64_t)sc.e) : 0;
            if (len) cig[i] = std::to_string(len) + (ps[i].n ? "I" : "D");
        }
        std::vector<int32_t> gs;
        double ms = 0.0;
        if ((s = global_scores(ctx, gp, sc, st, gs, ms)) != SWH_OK) return s;
        for (size_t j = 0; j < gi.size(); ++j) out[gi[j]].score = gs[j];
        if (stats) stats->ms_forward = ms;
        if (mode != SWH_MODE_CIGAR) return SWH_OK;
        TracebackStats ts;
        size_t k = 0;
        while (k < gi.size()) {
            std::vector<TbInput> in;
            std::vector<int64_t> ids;
            int64_t cols = 0;
            while (k < gi.size()) {
                const int64_t i = gi[k];
                if (!in.empty() && cols + ps[i].m > kTracebackCols) break;
                in.push_back(TbInput{ps[i].q, ps[i].n, ps[i].t, ps[i].m, out[i].score});
                ids.push_back(i);
                cols += ps[i].m;
                ++k;
            }
            std::vector<std::string> cg;
            if ((s = traceback_batch(ctx, in, sc, st, cg, ts)) != SWH_OK) return s;
            for (size_t j = 0; j < ids.size(); ++j) cig[ids[j]].swap(cg[j]);
        }
        if (stats) {
            stats->ms_traceback = ts.ms;
            stats->cells_traceback = ts.cells;
        }
    } else {
    const int forced = ctx->opt.band_rows;
    const bool banded = mode == SWH_MODE_CIGAR && forced >= 0;
    const bool want16 = ctx->opt.int16 != 0;
    std::vector<BandKeep> bk((size_t)npairs);
    std::vector<int64_t> frecs((size_t)npairs, 0);
    for (int64_t i = 0; i < npairs; ++i) ps[i].int16 = want16;
    if (banded)
        for (int64_t i = 0; i < npairs; ++i) {
            const StripShape sh = tuned_shape(ctx, ps[i].n);
            const int64_t H = 64 * (int64_t)sh.R;
            const int64_t want = forced > 0 ? forced : kBatchBandRows;
            const int every = (int)std::max<int64_t>(1, (want + H - 1) / H);
            frecs[i] = band_forward_layout(sh.R, every, ps[i].n, ps[i].m, bk[i]);
            ps[i].R = sh.R;
            ps[i].waves = sh.waves;
        }
    int64_t budget = kBatchKeepBytes / (int64_t)sizeof(Border);
    {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess)
            budget = std::min<int64_t>(budget, (int64_t)(free_b / 8 / sizeof(Border)));
        else
            (void)hipGetLastError();
        budget = std::min<int64_t>(budget, (int64_t)std::min<size_t>(cap_room(ctx) / 4 / sizeof(Border), INT64_MAX));
    }
    TracebackStats ts;
    double ms_fwd = 0.0, ms_rev = 0.0;
    int64_t nbands = 0, retries = 0;
    int64_t g0 = 0;
    while (g0 < npairs) {
        // a group: kept rows of both passes within the budget (a pair whose
        // rows do not fit alone runs without them)
        int64_t g1 = g0, recs = 0;
        while (g1 < npairs) {
            const int64_t r = 2 * frecs[(size_t)g1];
            if (g1 > g0 && recs + r > budget) break;
            recs += r;
            ++g1;
        }
        std::vector<PairPass> gps(ps.begin() + g0, ps.begin() + g1);
        if (banded) {
            int64_t off = 0;
            const bool fits = recs <= budget && ensure(ctx, ctx->keep_f, (size_t)std::max<int64_t>(recs / 2, 1) *
                                                                             sizeof(Border), "kept rows") == SWH_OK;
            if (!fits) ctx->err.clear();
            for (int64_t i = g0; i < g1; ++i) {
                BandKeep &k = bk[(size_t)i];
                if (!fits || k.every == 0) {
                    k.every = 0;
                    continue;
                }
                k.keep_f = (const Border *)ctx->keep_f.p + off;
                PairPass &p = gps[(size_t)(i - g0)];
                p.keep = (Border *)ctx->keep_f.p + off;
                p.every = k.every;
                p.phase = 0;
                off += frecs[(size_t)i];
            }
        }

        // ---- resolution: forward local pass of every pair of the group
        std::vector<BestCell> fwd;
        if ((s = score_passes(ctx, gps, sc, st, fwd, ms_fwd)) != SWH_OK) return s;
        std::vector<int64_t> pos_pairs;
        for (int64_t i = g0; i < g1; ++i) {
            const BestCell &f = fwd[(size_t)(i - g0)];
            out[i].score = f.score;
            if (f.score > 0) {
                out[i].q_end = f.row - 1;
                out[i].t_end = f.col - 1;
                pos_pairs.push_back(i);
            }
        }
        if (mode == SWH_MODE_SCORE) {
            g0 = g1;
            continue;
        }

        // ---- reverse pass over the reversed prefixes ending at each end cell
        // (with kept rows: the forward strip height and the lead rows that put
        // its strip boundaries on the forward cuts)
        std::vector<PairPass> rp;
        rp.reserve(pos_pairs.size());
        int64_t rrecs = 0;
        const bool prune = ctx->opt.prune != 0;
        for (int64_t i : pos_pairs) {
            PairPass p{ps[i].q + out[i].q_end, out[i].q_end + 1, ps[i].t + out[i].t_end, out[i].t_end + 1, -1};
            p.prune = prune ? out[i].score : 0;   // the reverse maximum is the forward score
            p.int16 = want16 && out[i].score < sat16_limit(sc.smax);
            BandKeep &k = bk[(size_t)i];
            if (k.every > 0) {
                rrecs += band_reverse_layout(out[i].q_end, out[i].t_end, k);
                p.R = k.Rr;
                p.waves = ps[i].waves;
                p.lead = k.lead;
            }
            rp.push_back(p);
        }
        if (rrecs > 0) {
            if (ensure(ctx, ctx->keep_r, (size_t)rrecs * sizeof(Border), "kept rows") != SWH_OK) {
                ctx->err.clear();
                for (int64_t i : pos_pairs) bk[(size_t)i].every = 0;   // lead rows stay; they change nothing
            } else {
                int64_t off = 0;
                for (size_t j = 0; j < pos_pairs.size(); ++j) {
                    BandKeep &k = bk[(size_t)pos_pairs[j]];
                    if (k.every <= 0) continue;
                    k.keep_r = (const Border *)ctx->keep_r.p + off;
                    rp[j].keep = (Border *)ctx->keep_r.p + off;
                    rp[j].every = k.every_r;
                    rp[j].phase = k.phase;
                    off += k.kr * k.rstride;
                }
            }
        }
        std::vector<BestCell> rev;
        if ((s = score_passes(ctx, rp, sc, st, rev, ms_rev)) != SWH_OK) return s;
        for (size_t j = 0; j < pos_pairs.size(); ++j) {
            const int64_t i = pos_pairs[j];
            if (rev[j].score != out[i].score)
                return fail(ctx, SWH_E_DEVICE, "pair " + std::to_string(i) + ": reverse pass maximum " +
                                                   std::to_string(rev[j].score) + " differs from the forward score " +
                                                   std::to_string(out[i].score));
            out[i].q_begin = out[i].q_end - (rev[j].row - rp[j].lead - 1);
            out[i].t_begin = out[i].t_end - (rev[j].col - 1);
        }
        if (mode == SWH_MODE_COORDS) {
            g0 = g1;
            continue;
        }

        // ---- band cuts of every pair of the group: one scan over all of them
        std::vector<std::vector<TbBand>> bands(pos_pairs.size());
        if (banded) {
            std::vector<CutDesc> cd;
            std::vector<int64_t> rows;
            std::vector<size_t> first(pos_pairs.size() + 1, 0);
            for (size_t j = 0; j < pos_pairs.size(); ++j) {
                const int64_t i = pos_pairs[j];
                first[j] = cd.size();
                band_cuts(bk[(size_t)i], out[i], out[i].score, ps[i].q, ps[i].t, cd, rows);
            }
            first[pos_pairs.size()] = cd.size();
            std::vector<CutOut> co;
            if ((s = resolve_cuts(ctx, sc, st, cd, co)) != SWH_OK) return s;
            for (size_t j = 0; j < pos_pairs.size(); ++j)
                if (first[j + 1] > first[j])
                    bands_from_cuts(co.data() + first[j], rows.data() + first[j], (int)(first[j + 1] - first[j]),
                                    out[pos_pairs[j]], out[pos_pairs[j]].score, bands[j]);
        }

        // ---- reconstruction: batched linear-space traceback
        size_t k = 0;
        while (k < pos_pairs.size()) {
            std::vector<TbInput> in;
            std::vector<int64_t> ids;
            int64_t cols = 0;
            while (k < pos_pairs.size()) {
                const int64_t i = pos_pairs[k];
                const int64_t p = out[i].q_end - out[i].q_begin + 1, q = out[i].t_end - out[i].t_begin + 1;
                if (!in.empty() && cols + q > kTracebackCols) break;
                in.push_back(TbInput{ps[i].q + out[i].q_begin, p, ps[i].t + out[i].t_begin, q, out[i].score});
                in.back().bands.swap(bands[k]);
                ids.push_back(i);
                cols += q;
                ++k;
            }
            std::vector<std::string> cg;
            TracebackStats t1;
            s = traceback_batch(ctx, in, sc, st, cg, t1);
            bool with_bands = false;
            for (const TbInput &x : in) with_bands = with_bands || !x.bands.empty();
            if (s != SWH_OK && t1.inconsistent && with_bands) {
                // a band did not check out: this chunk again with the plain traceback
                ++retries;
                ctx->err.clear();
                for (TbInput &x : in) x.bands.clear();
                t1 = TracebackStats{};
                s = traceback_batch(ctx, in, sc, st, cg, t1);
            }
            if (s != SWH_OK) return s;
            for (const TbInput &x : in) nbands += (int64_t)x.bands.size();
            ts.ms += t1.ms;
            ts.cells += t1.cells;
            for (size_t j = 0; j < ids.size(); ++j) cig[ids[j]].swap(cg[j]);
        }
        g0 = g1;
    }
    if (stats) {
        stats->ms_forward = ms_fwd;
        stats->ms_reverse = ms_rev;
        stats->ms_traceback = ts.ms;
        stats->cells_traceback = ts.cells;
        stats->traceback_bands = nbands;
        stats->traceback_retries = retries;
    }
    }
    if (mode != SWH_MODE_CIGAR) return SWH_OK;
    int64_t total = 0;
    for (int64_t i = 0; i < npairs; ++i) {
        cigar_off[i] = total;
        total += (int64_t)cig[i].size();
    }
    cigar_off[npairs] = total;
    if (!cigar_cat || total > cigar_cap)
        return fail(ctx, SWH_E_RANGE, "CIGARs need " + std::to_string(total) + " bytes");
    for (int64_t i = 0; i < npairs; ++i)
        if (!cig[i].empty()) std::memcpy(cigar_cat + cigar_off[i], cig[i].data(), cig[i].size());
    return SWH_OK;
}

}  // namespace swh
