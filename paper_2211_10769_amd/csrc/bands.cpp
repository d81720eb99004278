// bands.cpp -- the band traceback's first split, taken from the score passes.
//
// The divide and conquer of the reconstruction needs, for a row x of the
// aligned rectangle, where the optimal path crosses from row x into row x+1.
// Both score passes already sweep the whole rectangle (the forward pass from
// the top, the reverse pass from the end cell), so each keeps its last row
// of every few strips; for the same rows x the forward record (H(x, j),
// F(x+1, j)) and the reverse record (H'(x+2, j), F'(x+1, j)) give every edge
// of an optimal local alignment as forward + edge + reverse = S (CutDesc).
// Local values are at least the rectangle's global values and equal them on
// every optimal path that ends at the end cell (a higher prefix or suffix
// would beat S), so an edge set with one member holds the path's crossing,
// with its true forward value.  Where a kept row has one such edge (and, for
// a vertical edge, the gap cannot close on row x), the path is cut there; the
// bands between cuts are independent subproblems of the ordinary divide and
// conquer, each seeded with the single node it is entered through (rows with
// several edges join the bands on both sides).  A band's restricted DP holds
// the true value at every node the canonical walk can visit, as in the
// ordinary split, so the CIGAR is the same; the work drops from about twice
// the rectangle to about twice the bands.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "bands.h"
#include "strips.h"

namespace swh {

int64_t band_forward_layout(int R, int every, int64_t n, int64_t m, BandKeep &k)
{
    k = BandKeep{};
    const int64_t H = 64 * (int64_t)R;
    k.R = R;
    k.every = every;
    k.kf = every > 0 ? ((n + H - 1) / H) / every : 0;
    k.fstride = cols_padded(m);
    if (k.kf < 1) k.every = 0;
    return k.every ? k.kf * k.fstride : 0;
}

int64_t band_reverse_layout(int64_t q_end, int64_t t_end, BandKeep &k, int rr)
{
    if (k.every <= 0) return 0;
    // kept rows every C forward rows; the reverse strips must end on them
    const int64_t C = 64 * (int64_t)k.R * k.every;
    k.Rr = (rr > 0 && C % (64 * (int64_t)rr) == 0) ? rr : k.R;
    const int64_t H = 64 * (int64_t)k.Rr;
    k.every_r = (int)(C / H);
    k.lead = (H - q_end % H) % H;
    k.T = (q_end + k.lead) / H;
    k.phase = (int)((k.every_r - k.T % k.every_r) % k.every_r);
    const int64_t nstrips = (q_end + 1 + k.lead + H - 1) / H;
    k.kr = (nstrips + k.phase) / k.every_r;
    k.rstride = cols_padded(t_end + 1);
    return k.kr * k.rstride;
}

void band_cuts(const BandKeep &k, const swh_alignment &al, int32_t S, const uint8_t *qcodes,
               const uint8_t *tcodes, std::vector<CutDesc> &cd, std::vector<int64_t> &rows)
{
    if (k.every <= 0 || !k.keep_f || !k.keep_r) return;
    const int64_t C = 64 * (int64_t)k.R * k.every;
    const int64_t qb = al.q_begin, qe = al.q_end;
    const int64_t k_lo = std::max<int64_t>(1, (qb + 1 + C - 1) / C), k_hi = qe / C;
    for (int64_t c = k_lo; c <= k_hi; ++c) {
        const int64_t x = c * C - 1;
        const int64_t slot_r = (k.T + k.phase) / k.every_r - 1 - c;
        // the reverse strip must exist (s' + 1 = T - c every_r >= 1)
        if (x < qb || x + 1 > qe || c - 1 >= k.kf || slot_r < 0 || slot_r >= k.kr || c * k.every_r > k.T - 1)
            continue;
        cd.push_back(CutDesc{k.keep_f + (c - 1) * k.fstride, k.keep_r + slot_r * k.rstride, qcodes + x + 1, tcodes,
                             al.t_end, S, k.global ? 1 : 0});
        rows.push_back(x);
    }
}

swh_status resolve_cuts(swh_ctx *ctx, const Scoring &sc, hipStream_t st, const std::vector<CutDesc> &cd,
                        std::vector<CutOut> &co)
{
    const int nc = (int)cd.size();
    co.assign((size_t)nc, CutOut{});
    if (nc == 0) return SWH_OK;
    int64_t max_te = 0;
    for (const CutDesc &c : cd) max_te = std::max(max_te, c.te);
    swh_status s;
    if ((s = ensure(ctx, ctx->cut_desc, sizeof(CutDesc) * (size_t)nc, "cut table")) != SWH_OK ||
        (s = ensure(ctx, ctx->cut_cnt, 8 * (size_t)nc, "cut counters")) != SWH_OK ||
        (s = ensure(ctx, ctx->cut_out, sizeof(CutOut) * (size_t)nc, "cut results")) != SWH_OK)
        return s;
    int32_t *cnt = (int32_t *)ctx->cut_cnt.p, *keys = cnt + nc;
    hipError_t e;
    if ((e = hipMemcpyAsync(ctx->cut_desc.p, cd.data(), sizeof(CutDesc) * (size_t)nc, hipMemcpyHostToDevice, st)) !=
            hipSuccess ||
        (e = hipMemsetAsync(cnt, 0, 4 * (size_t)nc, st)) != hipSuccess ||
        (e = hipMemsetAsync(keys, 0x7F, 4 * (size_t)nc, st)) != hipSuccess)
        return hip_fail(ctx, e, "cut tables");
    if ((e = launch_cut_scan((const CutDesc *)ctx->cut_desc.p, nc, max_te, (const int8_t *)ctx->mat.p, sc.asize,
                             sc.o, cnt, keys, st)) != hipSuccess ||
        (e = launch_cut_resolve((const CutDesc *)ctx->cut_desc.p, nc, cnt, keys, sc.o, sc.e,
                                (CutOut *)ctx->cut_out.p, st)) != hipSuccess)
        return hip_fail(ctx, e, "cut scan launch");
    if ((e = hipMemcpyAsync(co.data(), ctx->cut_out.p, sizeof(CutOut) * (size_t)nc, hipMemcpyDeviceToHost, st)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, "cut results");
    return SWH_OK;
}

void bands_from_cuts(const CutOut *co, const int64_t *rows, int nc, const swh_alignment &al, int32_t S,
                     std::vector<TbBand> &bands)
{
    bands.clear();
    const int64_t qb = al.q_begin, qe = al.q_end, tb = al.t_begin, te = al.t_end;
    // boundaries in rectangle coordinates: the top border, the clean cuts, the end
    struct Bound {
        int64_t row, col;
        int state;
        int32_t val, seed_h, seed_f;
    };
    std::vector<Bound> bd;
    bd.push_back(Bound{0, 0, 0, 0, 0, 0});
    for (int i = 0; i < nc; ++i) {
        const CutOut &c = co[i];
        if (c.count <= 0) return;
        if (!c.clean) continue;
        const int64_t col = c.col - tb + 1, row = rows[i] - qb + 1;
        if (col < 1 || col > te - tb + 1) return;
        bd.push_back(Bound{row, col, c.state, c.val, c.seed_h, c.seed_f});
    }
    if (bd.size() < 2) return;
    bd.push_back(Bound{qe - qb + 1, te - tb + 1, 0, S, 0, 0});
    for (size_t i = 0; i + 1 < bd.size(); ++i) {
        const Bound &u = bd[i], &d = bd[i + 1];
        if (u.col > d.col || u.row >= d.row) {
            bands.clear();
            return;
        }
        bands.push_back(TbBand{u.row, d.row, u.col, d.col, i > 0, u.seed_h, u.seed_f, d.state, d.val});
    }
}

}  // namespace swh
