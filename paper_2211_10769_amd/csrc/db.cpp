// db.cpp -- exhaustive query-vs-database search: database layout, the
// inter-task kernel for sequences up to the length switch (2,048 residues by
// default, a context option otherwise), the single-pair
// strip kernel for longer ones (the length-dependent choice between
// inter-task and intra-task parallelism of SW#, paper, Background) and for
// pairs whose 16-bit scores may have saturated, then the top-k.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "context.h"
#include "db.h"
#include "db_kernels.h"
#include "strips.h"
#include "tb_kernels.h"
#include "tune.h"

namespace swh {

namespace {

constexpr int64_t kInterMax = 2048;   // longest database sequence of the inter-task kernel

void free_buf(DevBuf &b)
{
    if (b.p) hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

// Encode ASCII sequences into device codes (original order); reports the
// first bad byte of the concatenation.  cat is a host pointer (copied through
// raw first) or, with dev, a device pointer encoded in place.
swh_status encode_host(swh_ctx *ctx, const Scoring &sc, const char *cat, int64_t total, DevBuf &raw, DevBuf &codes,
                       hipStream_t st, const char *what, bool dev = false)
{
    swh_status s;
    if (!dev && (s = ensure(ctx, raw, (size_t)total + 1, what)) != SWH_OK) return s;
    if ((s = ensure(ctx, codes, (size_t)total + 1, what)) != SWH_OK) return s;
    if ((s = ensure(ctx, ctx->lut, 256, "symbol table")) != SWH_OK) return s;
    if ((s = ensure(ctx, ctx->misc, 64, "scratch words")) != SWH_OK) return s;
    hipError_t e;
    const int32_t init = INT32_MAX;
    if ((!dev && total && (e = hipMemcpyAsync(raw.p, cat, (size_t)total, hipMemcpyHostToDevice, st)) != hipSuccess) ||
        (e = hipMemcpyAsync(ctx->lut.p, sc.lut, 256, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(ctx->misc.p, &init, 4, hipMemcpyHostToDevice, st)) != hipSuccess)
        return hip_fail(ctx, e, "upload");
    const char *src = dev ? cat : (const char *)raw.p;
    if ((e = launch_encode(src, total, (uint8_t *)codes.p, total, (const uint8_t *)ctx->lut.p,
                           (uint8_t)sc.asize, (int32_t *)ctx->misc.p, st)) != hipSuccess)
        return hip_fail(ctx, e, "encode launch");
    int32_t bad = 0;
    if ((e = hipMemcpyAsync(&bad, ctx->misc.p, 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, "encode");
    if (bad != INT32_MAX)
        return fail(ctx, SWH_E_ALPHABET, std::string(what) + ": byte at position " + std::to_string(bad) +
                                             " of the concatenation is not in the alphabet");
    return SWH_OK;
}

swh_status check_offsets(swh_ctx *ctx, int64_t n, const int64_t *off, const char *what)
{
    if (n < 0 || (n > 0 && !off)) return fail(ctx, SWH_E_INVAL, std::string(what) + ": bad count or offsets");
    for (int64_t i = 0; i < n; ++i)
        if (off[i + 1] < off[i]) return fail(ctx, SWH_E_INVAL, std::string(what) + ": offsets must not decrease");
    return SWH_OK;
}

}  // namespace

swh_status gather_lite(swh_ctx *ctx, const std::vector<GatherLite> &g, uint8_t pad, hipStream_t st)
{
    if (g.empty()) return SWH_OK;
    std::vector<GatherDesc> d;
    d.reserve(g.size());
    for (const GatherLite &x : g) d.push_back(GatherDesc{x.src, x.dst, 0, x.count, x.padded, 1, 0});
    swh_status s = ensure(ctx, ctx->tb_misc, sizeof(GatherDesc) * d.size() + 16, "gather table");
    if (s != SWH_OK) return s;
    hipError_t e;
    if ((e = hipMemcpyAsync(ctx->tb_misc.p, d.data(), sizeof(GatherDesc) * d.size(), hipMemcpyHostToDevice, st)) !=
            hipSuccess ||
        (e = launch_gather((const GatherDesc *)ctx->tb_misc.p, (int32_t)d.size(), pad, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, "gather");
    return SWH_OK;
}

swh_status db_create(swh_ctx *ctx, int64_t ndb, const char *cat, const int64_t *off, const Scoring &sc,
                     swh_db **out)
{
    swh_status s;
    if ((s = check_offsets(ctx, ndb, off, "database")) != SWH_OK) return s;
    if (ndb >= INT32_MAX) return fail(ctx, SWH_E_RANGE, "database larger than 2^31 - 1 sequences");
    hipStream_t st = ctx->own_stream;
    swh_db *db = new (std::nothrow) swh_db();
    if (!db) return fail(ctx, SWH_E_NOMEM, "database handle");
    static std::atomic<uint64_t> serials{0};
    db->device = ctx->device;
    db->sc = sc;
    db->serial = ++serials;
    db->inter_max = ctx->opt.inter_max > 0 ? ctx->opt.inter_max
                    : ctx->tuned_inter_max > 0 ? ctx->tuned_inter_max
                                               : kInterMax;
    db->ndb = ndb;
    const int64_t base = ndb ? off[0] : 0, total = ndb ? off[ndb] - base : 0;
    db->h_off.resize((size_t)ndb + 1);
    for (int64_t i = 0; i <= ndb; ++i) db->h_off[i] = ndb ? off[i] - base : 0;
    DevBuf raw;
    s = encode_host(ctx, sc, cat ? cat + base : nullptr, total, raw, db->codes, st, "database");
    free_buf(raw);
    if (s != SWH_OK) {
        db_destroy(db);
        return s;
    }
    hipError_t e;
    if ((s = ensure(ctx, db->offs, sizeof(int64_t) * (size_t)(ndb + 1), "database offsets")) != SWH_OK ||
        (e = hipMemcpyAsync(db->offs.p, db->h_off.data(), sizeof(int64_t) * (size_t)(ndb + 1),
                            hipMemcpyHostToDevice, st)) != hipSuccess) {
        db_destroy(db);
        return s != SWH_OK ? s : hip_fail(ctx, e, "offsets");
    }

    // sort by length; long sequences go to the single-pair kernel
    std::vector<int32_t> order;
    order.reserve((size_t)ndb);
    for (int64_t i = 0; i < ndb; ++i) {
        const int64_t L = db->h_off[i + 1] - db->h_off[i];
        if (L > db->inter_max)
            db->long_idx.push_back((int32_t)i);
        else
            order.push_back((int32_t)i);
    }
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return db->h_off[a + 1] - db->h_off[a] < db->h_off[b + 1] - db->h_off[b];
    });
    const int64_t ngroups = ((int64_t)order.size() + 127) / 128;
    db->h_perm.assign((size_t)ngroups * 128, -1);
    std::copy(order.begin(), order.end(), db->h_perm.begin());
    db->h_groups.resize((size_t)ngroups);
    int64_t res_bytes = 0;
    for (int64_t g = 0; g < ngroups; ++g) {
        int32_t maxlen = 0;
        for (int s2 = 0; s2 < 128; ++s2) {
            const int32_t idx = db->h_perm[g * 128 + s2];
            if (idx >= 0) maxlen = std::max<int32_t>(maxlen, (int32_t)(db->h_off[idx + 1] - db->h_off[idx]));
        }
        db->h_groups[g] = DbGroup{res_bytes, maxlen, (int32_t)(g * 128)};
        res_bytes += (int64_t)maxlen * 128;
    }
    if ((s = ensure(ctx, db->res, (size_t)res_bytes + 256, "database layout")) != SWH_OK ||
        (s = ensure(ctx, db->groups, sizeof(DbGroup) * (size_t)ngroups + 16, "database groups")) != SWH_OK ||
        (s = ensure(ctx, db->perm, sizeof(int32_t) * (size_t)ngroups * 128 + 16, "database order")) != SWH_OK) {
        db_destroy(db);
        return s;
    }
    if ((ngroups && ((e = hipMemcpyAsync(db->groups.p, db->h_groups.data(), sizeof(DbGroup) * ngroups,
                                         hipMemcpyHostToDevice, st)) != hipSuccess ||
                     (e = hipMemcpyAsync(db->perm.p, db->h_perm.data(), sizeof(int32_t) * ngroups * 128,
                                         hipMemcpyHostToDevice, st)) != hipSuccess)) ||
        (e = launch_db_pack((const uint8_t *)db->codes.p, (const int64_t *)db->offs.p, (const int32_t *)db->perm.p,
                            (const DbGroup *)db->groups.p, (int32_t)ngroups, (uint8_t)sc.asize,
                            (uint8_t *)db->res.p, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess) {
        db_destroy(db);
        return hip_fail(ctx, e, "database layout");
    }
    db->total_residues = total;
    *out = db;
    return SWH_OK;
}

void db_destroy(swh_db *db)
{
    if (!db) return;
    hipSetDevice(db->device);
    hipDeviceSynchronize();
    free_buf(db->codes);
    free_buf(db->offs);
    free_buf(db->res);
    free_buf(db->groups);
    free_buf(db->perm);
    free_buf(db->pf_F);
    free_buf(db->pf_row_len);
    free_buf(db->pf_row_db);
    delete db;
}

swh_status prepare_queries(swh_ctx *ctx, const Scoring &sc, int32_t nq, const char *q_cat, const int64_t *q_off,
                           QuerySet &qs, bool dev)
{
    swh_status s;
    if ((s = check_offsets(ctx, nq, q_off, "queries")) != SWH_OK) return s;
    hipStream_t st = ctx->own_stream;
    const int64_t qbase = nq ? q_off[0] : 0, qtotal = nq ? q_off[nq] - qbase : 0;
    qs.nq = nq;
    qs.qo.assign((size_t)nq + 1, 0);
    qs.maxq = 1;
    for (int32_t i = 0; i <= nq; ++i) qs.qo[i] = nq ? q_off[i] - qbase : 0;
    for (int32_t i = 0; i < nq; ++i) qs.maxq = std::max(qs.maxq, qs.qo[i + 1] - qs.qo[i]);
    if (qs.maxq * std::max(sc.smax, 1) >= ((int64_t)1 << 26))
        return fail(ctx, SWH_E_RANGE, "query length * max|s| must stay below 2^26");
    if ((s = encode_host(ctx, sc, q_cat ? q_cat + qbase : nullptr, qtotal, ctx->qraw, ctx->qc, st, "queries", dev)) !=
        SWH_OK)
        return s;
    hipError_t e;
    if ((s = ensure(ctx, ctx->qoff, sizeof(int64_t) * (qs.qo.size() + 1), "query offsets")) != SWH_OK) return s;
    if ((s = ensure(ctx, ctx->mat, 32 * 32, "matrix")) != SWH_OK) return s;
    if ((e = hipMemcpyAsync(ctx->qoff.p, qs.qo.data(), sizeof(int64_t) * qs.qo.size(), hipMemcpyHostToDevice, st)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(ctx->mat.p, sc.mat, (size_t)sc.asize * sc.asize, hipMemcpyHostToDevice, st)) !=
            hipSuccess)
        return hip_fail(ctx, e, "query upload");
    return SWH_OK;
}

void plan_search(const swh_ctx *ctx, const swh_db *db, const std::vector<int64_t> &qo, int32_t nq,
                 std::vector<DbWork> &work, std::vector<std::pair<int32_t, int32_t>> &pairs, double &cells)
{
    const int64_t ngroups = (int64_t)db->h_groups.size();
    double colsum = 0.0;   // sum over groups of 128 x maxlen
    for (const DbGroup &g : db->h_groups) colsum += 128.0 * g.maxlen;
    double inter = 0.0;
    for (int32_t q = 0; q < nq; ++q) inter += (double)(qo[q + 1] - qo[q]) * colsum;
    const double share = inter / std::max(1, ctx->num_cu);
    const int route = ctx->opt.db_route;
    const double limit = route < 0 ? 1e300 : share * (route == 0 ? 100 : route) / 100.0;
    work.reserve(work.size() + (size_t)nq * (size_t)ngroups);
    for (int32_t q = 0; q < nq; ++q) {
        const int64_t n = qo[q + 1] - qo[q];
        if (n == 0) continue;
        for (int64_t g = 0; g < ngroups; ++g) {
            // (members are sorted by length: the first is the shortest; an empty
            // sequence is no single-pair problem, so its group is never moved)
            const int32_t first = db->h_perm[g * 128];
            const bool movable = first >= 0 && db->h_off[first + 1] > db->h_off[first];
            if (movable && (double)n * 128.0 * db->h_groups[g].maxlen > limit) {
                for (int s = 0; s < 128; ++s) {
                    const int32_t idx = db->h_perm[g * 128 + s];
                    if (idx >= 0) pairs.push_back({q, idx});
                }
            } else {
                work.push_back(DbWork{q, (int32_t)g});
            }
        }
        for (int32_t d : db->long_idx) pairs.push_back({q, d});
        cells += (double)n * (double)db->total_residues;
    }
}

DbLaunch db_launch_shape(const swh_ctx *ctx, size_t units, int32_t max_len, double mean_chunks)
{
    DbLaunch L;
    L.waves = ctx->opt.db_waves;
    if (L.waves == 0) {
        // one wave per unit while the units outnumber the resident waves sixteen to
        // one (the pipelined form pays some hand-over work per column, about 7%);
        // with fewer, the last units of the one-wave form leave SIMDs idle (a search
        // of 20 queries over a rescoring subset of 15,600 units: 238 ms with one wave
        // per unit, 135 ms with four), so the unit's chunks are spread over four waves
        L.waves = units >= (size_t)16 * db_search_grid_limit(ctx->device, 1) ? 1 : 4;
        // at most about one unit per SIMD: one work-group of eight waves per CU, or of
        // twelve for long queries (64 chunks or more per unit), so that each CU
        // list-schedules its units (one query against 100,000 proteins: eight waves
        // best up to 1,000 residues, 2.3-9.0 ms against 2.7-11.8 ms with four; twelve
        // at 5,000, 38.8 ms against 41.9 with eight and 61.3 with four)
        if (L.waves == 4 && units <= (size_t)4 * std::max(1, ctx->num_cu)) L.waves = mean_chunks >= 64.0 ? 12 : 8;
    }
    int limit = db_search_grid_limit(ctx->device, L.waves);
    if (ctx->opt.grid > 0) limit = std::min(limit, (int)ctx->opt.grid);
    L.grid = std::max(1, std::min<int>(limit, (int)std::max<size_t>(1, units)));
    L.wrap_cap = max_len + 64;
    L.border_bytes = L.waves == 1 ? (size_t)L.grid * max_len * 64 * 8 + 64
                                  : (size_t)L.grid * L.wrap_cap * 64 * 16 + 64;
    return L;
}

namespace {

// (query, sequence) pairs on the single-pair kernel, in 32 bits, enqueued on
// stream st with no host wait after the gather: padded copies of each query
// and each sequence once, the strip launch (timed by ctx->ev[0..1]), and the
// scatter of the scores into scores_dev.  The strip kernel's abort flag is
// ctx->sync[1] afterwards.
swh_status enqueue_pairs(swh_ctx *ctx, const swh_db *db, const QuerySet &qs,
                         const std::vector<std::pair<int32_t, int32_t>> &pairs, int32_t *scores_dev, hipStream_t st)
{
    swh_status s;
    hipError_t e;
    const Scoring &sc = db->sc;
    const std::vector<int64_t> &qo = qs.qo;
    const int32_t nq = qs.nq;
    const StripShape shape = tuned_shape(ctx, qs.maxq);
    const int R = shape.R;
    std::vector<int64_t> qpad_off((size_t)nq + 1, 0);
    for (int32_t q = 0; q < nq; ++q) qpad_off[q + 1] = qpad_off[q] + rows_padded(qo[q + 1] - qo[q], R);
    std::vector<int32_t> dids;
    for (auto &pq : pairs) dids.push_back(pq.second);
    std::sort(dids.begin(), dids.end());
    dids.erase(std::unique(dids.begin(), dids.end()), dids.end());
    std::vector<int64_t> dpad_off(dids.size() + 1, 0);
    for (size_t i = 0; i < dids.size(); ++i)
        dpad_off[i + 1] = dpad_off[i] + cols_padded(db->h_off[dids[i] + 1] - db->h_off[dids[i]]);
    int64_t border_entries = 0;
    for (auto &pq : pairs) border_entries += cols_padded(db->h_off[pq.second + 1] - db->h_off[pq.second]);
    const size_t code_bytes = (size_t)(qpad_off[nq] + dpad_off.back()) + 256;
    if ((s = ensure(ctx, ctx->tb_codes_q, code_bytes, "intra-task codes")) != SWH_OK ||
        (s = ensure(ctx, ctx->tb_bwd, sizeof(Border) * (size_t)border_entries + 256, "intra-task borders")) != SWH_OK ||
        (s = ensure(ctx, ctx->db_scatter, sizeof(int64_t) * pairs.size() + 64, "scatter")) != SWH_OK)
        return s;
    std::vector<GatherLite> gl;
    uint8_t *qbuf = (uint8_t *)ctx->tb_codes_q.p, *dbuf = qbuf + qpad_off[nq];
    for (int32_t q = 0; q < nq; ++q)
        gl.push_back(GatherLite{(const uint8_t *)ctx->qc.p + qo[q], qbuf + qpad_off[q], qo[q + 1] - qo[q],
                                qpad_off[q + 1] - qpad_off[q]});
    for (size_t i = 0; i < dids.size(); ++i)
        gl.push_back(GatherLite{(const uint8_t *)db->codes.p + db->h_off[dids[i]], dbuf + dpad_off[i],
                                db->h_off[dids[i] + 1] - db->h_off[dids[i]], dpad_off[i + 1] - dpad_off[i]});
    if ((s = gather_lite(ctx, gl, (uint8_t)sc.asize, st)) != SWH_OK) return s;
    if ((e = launch_fill_i32((int32_t *)ctx->tb_bwd.p, 2 * border_entries, 0, st)) != hipSuccess)
        return hip_fail(ctx, e, "intra-task borders");
    std::vector<StripProblem> probs;
    Border *bp = (Border *)ctx->tb_bwd.p;
    std::vector<int64_t> &pos = ctx->pair_pos;   // lives until the next call: the upload reads it
    pos.resize(pairs.size());
    for (size_t i = 0; i < pairs.size(); ++i) {
        const auto &pq = pairs[i];
        const size_t di = (size_t)(std::lower_bound(dids.begin(), dids.end(), pq.second) - dids.begin());
        const int64_t L = db->h_off[pq.second + 1] - db->h_off[pq.second];
        probs.push_back(StripProblem{qbuf + qpad_off[pq.first], qo[pq.first + 1] - qo[pq.first],
                                     dbuf + dpad_off[di], L, bp});
        bp += cols_padded(L);
        pos[i] = (int64_t)pq.first * db->ndb + pq.second;
    }
    PreparedStrips &ps = ctx->strips;
    if ((s = prepare_strips(ctx, probs, sc, R, true, shape.waves, false, ps)) != SWH_OK) return s;
    if ((e = enqueue_strips(ctx, ps, sc, ps.tab.data(), ps.strip_prob.data(), st, true)) != hipSuccess ||
        (e = hipMemcpyAsync(ctx->db_scatter.p, pos.data(), sizeof(int64_t) * pos.size(), hipMemcpyHostToDevice,
                            st)) != hipSuccess ||
        (e = launch_scatter_best((const int64_t *)ctx->db_scatter.p, (const int32_t *)ctx->prob_best.p,
                                 (int64_t)pos.size(), (int32_t)(sizeof(BestCell) / sizeof(int32_t)), scores_dev,
                                 st)) != hipSuccess)
        return hip_fail(ctx, e, "single-pair launch");
    return SWH_OK;
}

// Wait for an enqueue_pairs on st; adds its kernel time to stats.
swh_status finish_pairs(swh_ctx *ctx, hipStream_t st, DbStats &stats, size_t npairs)
{
    hipError_t e;
    int32_t flags[2] = {0, 0};
    if ((e = hipMemcpyAsync(flags, ctx->sync.p, sizeof(flags), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, "single-pair pass");
    if (cancelled(ctx)) return cancel_status(ctx);
    if (flags[1]) return fail(ctx, SWH_E_TIMEOUT, "strip wavefront wait expired");
    float ms = 0.f;
    hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]);
    stats.ms_intra += ms;
    stats.intra_pairs += (int64_t)npairs;
    return SWH_OK;
}

}  // namespace

swh_status score_units(swh_ctx *ctx, const swh_db *db, const QuerySet &qs, const GroupSet &gs,
                       std::vector<DbWork> work, const std::vector<std::pair<int32_t, int32_t>> &long_pairs,
                       int32_t *scores_dev, DbStats &stats)
{
    swh_status s;
    hipError_t e;
    hipStream_t st = ctx->own_stream, aux = ctx->aux_stream;
    const Scoring &sc = db->sc;
    const std::vector<int64_t> &qo = qs.qo;

    // ---- the single-pair problems known now (sequences beyond the length
    //      switch, members of oversize units) run on the auxiliary stream, beside
    //      the inter-task kernel: its last units leave most of the GPU idle
    const bool side = !long_pairs.empty();
    if (side) {
        if ((e = hipEventRecord(ctx->ev_fork, st)) != hipSuccess ||
            (e = hipStreamWaitEvent(aux, ctx->ev_fork, 0)) != hipSuccess)
            return hip_fail(ctx, e, "stream fork");
        if ((s = enqueue_pairs(ctx, db, qs, long_pairs, scores_dev, aux)) != SWH_OK) {
            hipStreamSynchronize(aux);
            return s;
        }
    }
    auto join = [&]() {
        if (side && hipEventRecord(ctx->ev_join, aux) == hipSuccess) hipStreamWaitEvent(st, ctx->ev_join, 0);
        hipStreamSynchronize(aux);
    };

    // ---- inter-task: every (query, group) unit, most expensive first
    int32_t max_len = 1;
    for (const DbWork &w : work) max_len = std::max(max_len, (*gs.h_groups)[w.g].maxlen);
    std::stable_sort(work.begin(), work.end(), [&](const DbWork &a, const DbWork &b) {
        return (qo[a.q + 1] - qo[a.q]) * (int64_t)(*gs.h_groups)[a.g].maxlen >
               (qo[b.q + 1] - qo[b.q]) * (int64_t)(*gs.h_groups)[b.g].maxlen;
    });
    double chunks = 0.0;
    for (const DbWork &w : work) chunks += (double)((qo[w.q + 1] - qo[w.q] + 31) / 32);
    const DbLaunch shape = db_launch_shape(ctx, work.size(), max_len, work.empty() ? 0.0 : chunks / work.size());
    const int redo_cap = 1 << 20;
    if ((s = ensure(ctx, ctx->db_work, sizeof(DbWork) * work.size() + 16, "work list")) != SWH_OK ||
        (s = ensure(ctx, ctx->db_border, shape.border_bytes, "inter-task borders")) != SWH_OK ||
        (s = ensure(ctx, ctx->db_redo, sizeof(int32_t) * 2 * (size_t)redo_cap + 64, "redo list")) != SWH_OK ||
        (s = ensure(ctx, ctx->db_sync, 64, "ticket")) != SWH_OK) {
        join();
        return s;
    }
    if ((!work.empty() && (e = hipMemcpyAsync(ctx->db_work.p, work.data(), sizeof(DbWork) * work.size(),
                                              hipMemcpyHostToDevice, st)) != hipSuccess) ||
        (e = launch_fill_i32((int32_t *)ctx->db_sync.p, 16, 0, st)) != hipSuccess) {
        join();
        return hip_fail(ctx, e, "work upload");
    }
    DbSearchArgs a;
    a.res = gs.res;
    a.groups = gs.groups;
    a.perm = gs.perm;
    a.qcodes = (const uint8_t *)ctx->qc.p;
    a.qoff = (const int64_t *)ctx->qoff.p;
    a.work = (const DbWork *)ctx->db_work.p;
    a.nwork = (int32_t)work.size();
    a.asize = sc.asize;
    a.mat = (const int8_t *)ctx->mat.p;
    a.o = sc.o;
    a.e = sc.e;
    a.ndb = db->ndb;
    a.scores = scores_dev;
    a.redo = (int32_t *)ctx->db_redo.p;
    a.nredo = (int32_t *)ctx->db_sync.p + 8;
    a.redo_cap = redo_cap;
    a.ticket = (int32_t *)ctx->db_sync.p;
    a.border = (uint32_t *)ctx->db_border.p;
    a.max_len = max_len;
    a.wrap_cap = shape.wrap_cap;
    a.cancel = ctx->cancel_dev;
    a.abort_flag = (int32_t *)ctx->db_sync.p + 2;
    a.wait_ticks = wait_ticks(ctx->device);
    hipEventRecord(ctx->ev[2], st);
    if (!work.empty() && (e = launch_db_search(a, shape.waves, shape.grid, st)) != hipSuccess) {
        join();
        return hip_fail(ctx, e, "search launch");
    }
    hipEventRecord(ctx->ev[3], st);
    int32_t words[16] = {0};
    e = hipMemcpyAsync(words, ctx->db_sync.p, sizeof(words), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        join();
        return hip_fail(ctx, e, "search");
    }
    if (side && (s = finish_pairs(ctx, aux, stats, long_pairs.size())) != SWH_OK) return s;
    const int32_t nredo = words[8];
    if (cancelled(ctx)) return cancel_status(ctx);
    if (words[2]) return fail(ctx, SWH_E_TIMEOUT, "database search: a hand-over wait expired");
    float ms = 0.f;
    hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]);
    stats.ms_inter += ms;
    if (nredo > redo_cap) return fail(ctx, SWH_E_RANGE, "more than 2^20 saturated pairs in one search");
    if (nredo == 0) return SWH_OK;

    // ---- 16-bit saturation: those pairs again in 32 bits on the single-pair kernel
    std::vector<int32_t> redo((size_t)2 * nredo);
    if ((e = hipMemcpyAsync(redo.data(), a.redo, sizeof(int32_t) * 2 * nredo, hipMemcpyDeviceToHost, st)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, "redo list");
    stats.redo += nredo;
    std::vector<std::pair<int32_t, int32_t>> pairs;
    for (int32_t i = 0; i < nredo; ++i) pairs.push_back({redo[2 * i], redo[2 * i + 1]});
    if ((s = enqueue_pairs(ctx, db, qs, pairs, scores_dev, st)) != SWH_OK) {
        hipStreamSynchronize(st);
        return s;
    }
    return finish_pairs(ctx, st, stats, pairs.size());
}

swh_status db_scores_device(swh_ctx *ctx, const swh_db *db, int32_t nq, const char *q_cat, const int64_t *q_off,
                            int32_t *scores_dev, DbStats &stats, bool dev)
{
    QuerySet qs;
    swh_status s = prepare_queries(ctx, db->sc, nq, q_cat, q_off, qs, dev);
    if (s != SWH_OK) return s;
    std::vector<DbWork> work;
    std::vector<std::pair<int32_t, int32_t>> long_pairs;
    for (int32_t q = 0; q < nq; ++q) {
        if (qs.qo[q + 1] == qs.qo[q]) {
            // an empty query aligns with nothing: every score is 0
            hipError_t e = launch_fill_i32(scores_dev + (int64_t)q * db->ndb, db->ndb, 0, ctx->own_stream);
            if (e != hipSuccess) return hip_fail(ctx, e, "score fill");
        }
    }
    plan_search(ctx, db, qs.qo, nq, work, long_pairs, stats.cells);
    GroupSet gs{(const uint8_t *)db->res.p, (const DbGroup *)db->groups.p, (const int32_t *)db->perm.p,
                &db->h_groups};
    return score_units(ctx, db, qs, gs, std::move(work), long_pairs, scores_dev, stats);
}

swh_status db_search(swh_ctx *ctx, const swh_db *db, int32_t nq, const char *q_cat, const int64_t *q_off, int32_t k,
                     swh_hit *hits, int32_t *scores_host, DbStats &stats, bool dev)
{
    swh_status s;
    hipError_t e;
    hipStream_t st = ctx->own_stream;
    if (hits && !scores_host && !dev && ctx->opt.graph == 2 && nq > 0 && db->ndb > 0 && k > 0) {
        bool done = false;
        if ((s = search_graph(ctx, db, nq, q_cat, q_off, k, hits, stats, done)) != SWH_OK || done) return s;
        stats = DbStats{};
    }
    if ((s = ensure(ctx, ctx->db_scores, sizeof(int32_t) * (size_t)std::max<int64_t>(1, (int64_t)nq * db->ndb) + 64,
                    "score matrix")) != SWH_OK)
        return s;
    int32_t *scores = (int32_t *)ctx->db_scores.p;
    if ((s = db_scores_device(ctx, db, nq, q_cat, q_off, scores, stats, dev)) != SWH_OK) return s;
    if (scores_host && nq && db->ndb &&
        ((e = hipMemcpyAsync(scores_host, scores, sizeof(int32_t) * (size_t)nq * db->ndb, hipMemcpyDeviceToHost,
                             st)) != hipSuccess ||
         (e = hipStreamSynchronize(st)) != hipSuccess))
        return hip_fail(ctx, e, "scores download");
    if (hits && k > 0 && nq > 0) {
        const size_t cand = topk_scratch_entries(nq, db->ndb, k);
        if ((s = ensure(ctx, ctx->db_topk, cand * 8 + (size_t)nq * k * 12 + 256, "top-k scratch")) != SWH_OK)
            return s;
        int32_t *cidx = (int32_t *)ctx->db_topk.p;
        int32_t *cscore = cidx + cand;
        int64_t *oidx = (int64_t *)(((uintptr_t)(cscore + cand) + 15) & ~(uintptr_t)15);
        int32_t *oscore = (int32_t *)(oidx + (size_t)nq * k);
        hipEventRecord(ctx->ev[2], st);
        if ((e = launch_topk(scores, nq, db->ndb, k, cidx, cscore, oidx, oscore, st)) != hipSuccess)
            return hip_fail(ctx, e, "top-k launch");
        hipEventRecord(ctx->ev[3], st);
        std::vector<int64_t> hi((size_t)nq * k);
        std::vector<int32_t> hs((size_t)nq * k);
        if ((e = hipMemcpyAsync(hi.data(), oidx, sizeof(int64_t) * hi.size(), hipMemcpyDeviceToHost, st)) !=
                hipSuccess ||
            (e = hipMemcpyAsync(hs.data(), oscore, sizeof(int32_t) * hs.size(), hipMemcpyDeviceToHost, st)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess)
            return hip_fail(ctx, e, "top-k");
        float ms = 0.f;
        hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]);
        stats.ms_topk = ms;
        for (size_t i = 0; i < hi.size(); ++i) {
            hits[i].db_index = hi[i];
            hits[i].score = hi[i] >= 0 ? hs[i] : -1;
            hits[i].reserved = 0;
        }
    }
    return SWH_OK;
}

}  // namespace swh
