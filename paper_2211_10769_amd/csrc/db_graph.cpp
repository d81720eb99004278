// db_graph.cpp -- the exhaustive top-k search replayed as a captured HIP
// graph (the batching growth of the method: the whole launch sequence of a
// search is recorded once and replayed, with no host decision between its
// launches).
//
// A plan is keyed by the database handle, k and the query lengths.  Building
// it sizes every context buffer the search needs, lays out everything the
// host would compute between launches (the work list of (query, group) units
// ordered by cost, the single-pair problems of the long database sequences,
// their gather descriptors and result positions) in pinned host memory, and
// captures on the context's stream:
//   query bytes (pinned staging) -> device; scoring tables; encode;
//   work list; counters cleared by a fill kernel; the inter-task kernel;
//   for long sequences: gather of their codes, border rows cleared, the
//   strip kernel and its per-problem reduction, results scattered into the
//   score matrix; the two top-k kernels; hits, the encoder's bad-byte word,
//   the saturated-pair count and the abort flag -> pinned host memory.
// A replay copies the new queries into the staging buffer, launches the
// graph and reads the results.  The graph refers to context buffers by
// address, so any reallocation of one of them (the context's generation
// counter) invalidates the plan; its kernels rewrite every buffer they read
// on each replay.  A search whose inter-task pass saturated 16 bits for some
// pair needs the host's recomputation list and is run eagerly instead.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <string>
#include <vector>

#include "context.h"
#include "db.h"
#include "db_kernels.h"
#include "strips.h"
#include "tb_kernels.h"
#include "tune.h"

namespace swh {

struct SearchPlan {
    // key
    const swh_db *db = nullptr;
    uint64_t serial = 0, gen = 0;
    int32_t nq = 0, k = 0;
    std::vector<int64_t> qlens;
    // graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // pinned host memory: inputs copied in by the graph, outputs copied out
    void *pinned = nullptr;
    char *q_stage = nullptr;
    int64_t *out_idx = nullptr;
    int32_t *out_score = nullptr;
    int32_t *out_words = nullptr;   // [0] first bad byte (INT32_MAX: none), [1] saturated pairs,
                                    // [2] strip abort flag, [3] database-kernel abort flag
    int64_t qtotal = 0;
    double cells = 0.0;
    int64_t long_pairs = 0;
};

namespace {

void free_plan(SearchPlan *p)
{
    if (!p) return;
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    if (p->pinned) hipHostFree(p->pinned);
    delete p;
}

// Pinned block carved into aligned regions.
struct PinnedLayout {
    size_t at = 0;
    size_t take(size_t bytes)
    {
        const size_t r = at;
        at += (bytes + 255) & ~(size_t)255;
        return r;
    }
};

bool same_key(const SearchPlan *p, const swh_db *db, int32_t nq, int32_t k, const std::vector<int64_t> &lens,
              uint64_t gen)
{
    return p && p->db == db && p->serial == db->serial && p->gen == gen && p->nq == nq && p->k == k &&
           p->qlens == lens;
}

}  // namespace

void destroy_search_plan(swh_ctx *ctx)
{
    free_plan(ctx->splan);
    ctx->splan = nullptr;
}

namespace {

// Build and capture the plan for this key; nullptr (with ctx->err clear) when
// the search must run eagerly.
swh_status build_plan(swh_ctx *ctx, const swh_db *db, int32_t nq, int32_t k, const std::vector<int64_t> &qo,
                      SearchPlan *&out)
{
    out = nullptr;
    hipStream_t st = ctx->own_stream;
    const Scoring &sc = db->sc;
    const int64_t ndb = db->ndb, ngroups = (int64_t)db->h_groups.size();
    const int64_t qtotal = qo[nq];
    int64_t maxq = 1;
    for (int32_t q = 0; q < nq; ++q) maxq = std::max(maxq, qo[q + 1] - qo[q]);
    if (maxq * std::max(sc.smax, 1) >= ((int64_t)1 << 26))
        return fail(ctx, SWH_E_RANGE, "query length * max|s| must stay below 2^26");

    // empty queries (their rows must read 0) are left to the eager path
    for (int32_t q = 0; q < nq; ++q)
        if (qo[q + 1] == qo[q]) return SWH_OK;

    // ---- what the host decides between launches, decided once
    std::vector<DbWork> work;
    std::vector<std::pair<int32_t, int32_t>> lp;
    double cells = 0.0;
    plan_search(ctx, db, qo, nq, work, lp, cells);
    int32_t max_len = 1;
    for (const DbWork &w : work) max_len = std::max(max_len, db->h_groups[w.g].maxlen);
    std::stable_sort(work.begin(), work.end(), [&](const DbWork &a, const DbWork &b) {
        return (qo[a.q + 1] - qo[a.q]) * (int64_t)db->h_groups[a.g].maxlen >
               (qo[b.q + 1] - qo[b.q]) * (int64_t)db->h_groups[b.g].maxlen;
    });
    double chunks = 0.0;
    for (const DbWork &w : work) chunks += (double)((qo[w.q + 1] - qo[w.q] + 31) / 32);
    const DbLaunch dbl = db_launch_shape(ctx, work.size(), max_len, work.empty() ? 0.0 : chunks / work.size());
    const int redo_cap = 1 << 20;
    const size_t cand = topk_scratch_entries(nq, ndb, k);

    swh_status s;
    if ((s = ensure(ctx, ctx->qraw, (size_t)qtotal + 1, "queries")) != SWH_OK ||
        (s = ensure(ctx, ctx->qc, (size_t)qtotal + 1, "queries")) != SWH_OK ||
        (s = ensure(ctx, ctx->lut, 256, "symbol table")) != SWH_OK ||
        (s = ensure(ctx, ctx->misc, 64, "scratch words")) != SWH_OK ||
        (s = ensure(ctx, ctx->qoff, sizeof(int64_t) * (size_t)(nq + 2), "query offsets")) != SWH_OK ||
        (s = ensure(ctx, ctx->mat, 32 * 32, "matrix")) != SWH_OK ||
        (s = ensure(ctx, ctx->db_scores, sizeof(int32_t) * (size_t)std::max<int64_t>(1, (int64_t)nq * ndb) + 64,
                    "score matrix")) != SWH_OK ||
        (s = ensure(ctx, ctx->db_work, sizeof(DbWork) * work.size() + 16, "work list")) != SWH_OK ||
        (s = ensure(ctx, ctx->db_border, dbl.border_bytes, "inter-task borders")) != SWH_OK ||
        (s = ensure(ctx, ctx->db_redo, sizeof(int32_t) * 2 * (size_t)redo_cap + 64, "redo list")) != SWH_OK ||
        (s = ensure(ctx, ctx->sync, 64, "ticket")) != SWH_OK ||
        (s = ensure(ctx, ctx->db_sync, 64, "ticket")) != SWH_OK ||
        (s = ensure(ctx, ctx->db_topk, cand * 8 + (size_t)nq * k * 12 + 256, "top-k scratch")) != SWH_OK)
        return s;

    // long database sequences: one single-pair problem per (query, sequence)
    const StripShape shape = tuned_shape(ctx, maxq);
    const int R = shape.R;
    std::vector<GatherDesc> gd;
    std::vector<StripProblem> probs;
    std::vector<int64_t> pos;
    if (!lp.empty()) {
        std::vector<int64_t> qpad_off((size_t)nq + 1, 0);
        for (int32_t q = 0; q < nq; ++q) qpad_off[q + 1] = qpad_off[q] + rows_padded(qo[q + 1] - qo[q], R);
        std::vector<int32_t> dids;   // each database sequence of a pair once, by index
        for (auto &pq : lp) dids.push_back(pq.second);
        std::sort(dids.begin(), dids.end());
        dids.erase(std::unique(dids.begin(), dids.end()), dids.end());
        std::vector<int64_t> dpad_off(dids.size() + 1, 0);
        for (size_t i = 0; i < dids.size(); ++i)
            dpad_off[i + 1] = dpad_off[i] + cols_padded(db->h_off[dids[i] + 1] - db->h_off[dids[i]]);
        int64_t border_entries = 0;
        for (auto &pq : lp) border_entries += cols_padded(db->h_off[pq.second + 1] - db->h_off[pq.second]);
        if ((s = ensure(ctx, ctx->tb_codes_q, (size_t)(qpad_off[nq] + dpad_off.back()) + 256, "intra-task codes")) !=
                SWH_OK ||
            (s = ensure(ctx, ctx->tb_bwd, sizeof(Border) * (size_t)border_entries + 256, "intra-task borders")) !=
                SWH_OK ||
            (s = ensure(ctx, ctx->db_scatter, sizeof(int64_t) * lp.size() + 64, "scatter")) != SWH_OK ||
            (s = ensure(ctx, ctx->tb_misc, sizeof(GatherDesc) * ((size_t)nq + dids.size()) + 16, "gather table")) !=
                SWH_OK)
            return s;
        uint8_t *qbuf = (uint8_t *)ctx->tb_codes_q.p, *dbuf = qbuf + qpad_off[nq];
        for (int32_t q = 0; q < nq; ++q)
            gd.push_back(GatherDesc{(const uint8_t *)ctx->qc.p + qo[q], qbuf + qpad_off[q], 0, qo[q + 1] - qo[q],
                                    qpad_off[q + 1] - qpad_off[q], 1, 0});
        for (size_t i = 0; i < dids.size(); ++i)
            gd.push_back(GatherDesc{(const uint8_t *)db->codes.p + db->h_off[dids[i]], dbuf + dpad_off[i], 0,
                                    db->h_off[dids[i] + 1] - db->h_off[dids[i]], dpad_off[i + 1] - dpad_off[i], 1,
                                    0});
        Border *bp = (Border *)ctx->tb_bwd.p;
        for (auto &pq : lp) {
            const size_t di = (size_t)(std::lower_bound(dids.begin(), dids.end(), pq.second) - dids.begin());
            const int64_t L = db->h_off[pq.second + 1] - db->h_off[pq.second];
            probs.push_back(StripProblem{qbuf + qpad_off[pq.first], qo[pq.first + 1] - qo[pq.first],
                                         dbuf + dpad_off[di], L, bp});
            bp += cols_padded(L);
            pos.push_back((int64_t)pq.first * ndb + pq.second);
        }
    }
    PreparedStrips prep;
    if (!probs.empty() && (s = prepare_strips(ctx, probs, sc, R, true, shape.waves, false, prep)) != SWH_OK) return s;
    prep.strip_order.clear();   // tickets in global strip order: the plan holds no order table
    int64_t border_entries = 0;
    for (const StripProblem &p : probs) border_entries += cols_padded(p.m);

    // ---- pinned host memory
    SearchPlan *p = new (std::nothrow) SearchPlan();
    if (!p) return fail(ctx, SWH_E_NOMEM, "search plan");
    PinnedLayout L;
    const size_t o_q = L.take((size_t)qtotal + 1), o_qoff = L.take(sizeof(int64_t) * (size_t)(nq + 1)),
                 o_lut = L.take(256), o_mat = L.take(32 * 32), o_init = L.take(16),
                 o_work = L.take(sizeof(DbWork) * std::max<size_t>(1, work.size())),
                 o_gd = L.take(sizeof(GatherDesc) * std::max<size_t>(1, gd.size())),
                 o_tab = L.take(sizeof(Problem) * std::max<size_t>(1, prep.tab.size())),
                 o_sp = L.take(sizeof(int32_t) * std::max<size_t>(1, prep.strip_prob.size())),
                 o_pos = L.take(sizeof(int64_t) * std::max<size_t>(1, pos.size())),
                 o_idx = L.take(sizeof(int64_t) * (size_t)nq * k), o_sco = L.take(sizeof(int32_t) * (size_t)nq * k),
                 o_words = L.take(16);
    if (hipHostMalloc(&p->pinned, L.at, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        delete p;
        return fail(ctx, SWH_E_NOMEM, "pinned memory of the search plan");
    }
    char *base = (char *)p->pinned;
    p->q_stage = base + o_q;
    p->out_idx = (int64_t *)(base + o_idx);
    p->out_score = (int32_t *)(base + o_sco);
    p->out_words = (int32_t *)(base + o_words);
    std::memcpy(base + o_qoff, qo.data(), sizeof(int64_t) * (size_t)(nq + 1));
    std::memcpy(base + o_lut, sc.lut, 256);
    std::memcpy(base + o_mat, sc.mat, (size_t)sc.asize * sc.asize);
    const int32_t init[2] = {INT32_MAX, INT32_MAX};
    std::memcpy(base + o_init, init, sizeof(init));
    if (!work.empty()) std::memcpy(base + o_work, work.data(), sizeof(DbWork) * work.size());
    if (!gd.empty()) std::memcpy(base + o_gd, gd.data(), sizeof(GatherDesc) * gd.size());
    if (!prep.tab.empty()) std::memcpy(base + o_tab, prep.tab.data(), sizeof(Problem) * prep.tab.size());
    if (!prep.strip_prob.empty())
        std::memcpy(base + o_sp, prep.strip_prob.data(), sizeof(int32_t) * prep.strip_prob.size());
    if (!pos.empty()) std::memcpy(base + o_pos, pos.data(), sizeof(int64_t) * pos.size());

    // ---- capture
    DbSearchArgs a;
    a.res = (const uint8_t *)db->res.p;
    a.groups = (const DbGroup *)db->groups.p;
    a.perm = (const int32_t *)db->perm.p;
    a.qcodes = (const uint8_t *)ctx->qc.p;
    a.qoff = (const int64_t *)ctx->qoff.p;
    a.work = (const DbWork *)ctx->db_work.p;
    a.nwork = (int32_t)work.size();
    a.asize = sc.asize;
    a.mat = (const int8_t *)ctx->mat.p;
    a.o = sc.o;
    a.e = sc.e;
    a.ndb = ndb;
    a.scores = (int32_t *)ctx->db_scores.p;
    a.redo = (int32_t *)ctx->db_redo.p;
    a.nredo = (int32_t *)ctx->db_sync.p + 8;
    a.redo_cap = redo_cap;
    a.ticket = (int32_t *)ctx->db_sync.p;
    a.border = (uint32_t *)ctx->db_border.p;
    a.max_len = max_len;
    a.wrap_cap = dbl.wrap_cap;
    a.cancel = ctx->cancel_dev;
    a.abort_flag = (int32_t *)ctx->db_sync.p + 2;
    a.wait_ticks = wait_ticks(ctx->device);
    int32_t *cidx = (int32_t *)ctx->db_topk.p;
    int32_t *cscore = cidx + cand;
    int64_t *oidx = (int64_t *)(((uintptr_t)(cscore + cand) + 15) & ~(uintptr_t)15);
    int32_t *oscore = (int32_t *)(oidx + (size_t)nq * k);

    if (hipStreamSynchronize(st) != hipSuccess || hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        free_plan(p);
        return SWH_OK;
    }
    hipError_t e = hipSuccess;
    auto step = [&](hipError_t r) {
        if (e == hipSuccess) e = r;
    };
    const hipMemcpyKind H2D = hipMemcpyHostToDevice;
    step(hipMemcpyAsync(ctx->qraw.p, p->q_stage, (size_t)qtotal, H2D, st));
    step(hipMemcpyAsync(ctx->qoff.p, base + o_qoff, sizeof(int64_t) * (size_t)(nq + 1), H2D, st));
    step(hipMemcpyAsync(ctx->lut.p, base + o_lut, 256, H2D, st));
    step(hipMemcpyAsync(ctx->mat.p, base + o_mat, (size_t)sc.asize * sc.asize, H2D, st));
    step(hipMemcpyAsync(ctx->misc.p, base + o_init, sizeof(init), H2D, st));
    step(launch_encode((const char *)ctx->qraw.p, qtotal, (uint8_t *)ctx->qc.p, qtotal, (const uint8_t *)ctx->lut.p,
                       (uint8_t)sc.asize, (int32_t *)ctx->misc.p, st));
    if (!work.empty()) step(hipMemcpyAsync(ctx->db_work.p, base + o_work, sizeof(DbWork) * work.size(), H2D, st));
    step(launch_fill_i32((int32_t *)ctx->db_sync.p, 16, 0, st));
    if (!probs.empty()) {
        // the single-pair problems on the auxiliary stream, beside the inter-task kernel
        hipStream_t aux = ctx->aux_stream;
        step(hipEventRecord(ctx->ev_fork, st));
        step(hipStreamWaitEvent(aux, ctx->ev_fork, 0));
        step(hipMemcpyAsync(ctx->tb_misc.p, base + o_gd, sizeof(GatherDesc) * gd.size(), H2D, aux));
        step(launch_gather((const GatherDesc *)ctx->tb_misc.p, (int32_t)gd.size(), (uint8_t)sc.asize, aux));
        step(launch_fill_i32((int32_t *)ctx->tb_bwd.p, 2 * border_entries, 0, aux));
        step(enqueue_strips(ctx, prep, sc, (const Problem *)(base + o_tab), (const int32_t *)(base + o_sp), aux,
                            false));
        step(hipMemcpyAsync(ctx->db_scatter.p, base + o_pos, sizeof(int64_t) * pos.size(), H2D, aux));
        step(launch_scatter_best((const int64_t *)ctx->db_scatter.p, (const int32_t *)ctx->prob_best.p,
                                 (int64_t)pos.size(), (int32_t)(sizeof(BestCell) / sizeof(int32_t)),
                                 (int32_t *)ctx->db_scores.p, aux));
    }
    if (!work.empty()) step(launch_db_search(a, dbl.waves, dbl.grid, st));
    if (!probs.empty()) {
        step(hipEventRecord(ctx->ev_join, ctx->aux_stream));
        step(hipStreamWaitEvent(st, ctx->ev_join, 0));
    }
    step(launch_topk((const int32_t *)ctx->db_scores.p, nq, ndb, k, cidx, cscore, oidx, oscore, st));
    step(hipMemcpyAsync(p->out_idx, oidx, sizeof(int64_t) * (size_t)nq * k, hipMemcpyDeviceToHost, st));
    step(hipMemcpyAsync(p->out_score, oscore, sizeof(int32_t) * (size_t)nq * k, hipMemcpyDeviceToHost, st));
    step(hipMemcpyAsync(p->out_words, ctx->misc.p, 4, hipMemcpyDeviceToHost, st));
    step(hipMemcpyAsync(p->out_words + 1, (int32_t *)ctx->db_sync.p + 8, 4, hipMemcpyDeviceToHost, st));
    step(hipMemcpyAsync(p->out_words + 2, (int32_t *)ctx->sync.p + 1, 4, hipMemcpyDeviceToHost, st));
    step(hipMemcpyAsync(p->out_words + 3, (int32_t *)ctx->db_sync.p + 2, 4, hipMemcpyDeviceToHost, st));
    const hipError_t ee = hipStreamEndCapture(st, &p->graph);
    if (e != hipSuccess || ee != hipSuccess || !p->graph ||
        hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        free_plan(p);
        return SWH_OK;
    }
    p->db = db;
    p->serial = db->serial;
    p->gen = ctx->gen;
    p->nq = nq;
    p->k = k;
    p->qlens.resize(nq);
    for (int32_t q = 0; q < nq; ++q) p->qlens[q] = qo[q + 1] - qo[q];
    p->qtotal = qtotal;
    p->cells = cells;
    p->long_pairs = (int64_t)lp.size();
    out = p;
    return SWH_OK;
}

}  // namespace

swh_status search_graph(swh_ctx *ctx, const swh_db *db, int32_t nq, const char *q_cat, const int64_t *q_off,
                        int32_t k, swh_hit *hits, DbStats &stats, bool &done)
{
    done = false;
    for (int32_t i = 0; i < nq; ++i)
        if (q_off[i + 1] < q_off[i]) return fail(ctx, SWH_E_INVAL, "queries: offsets must not decrease");
    const int64_t qbase = q_off[0];
    std::vector<int64_t> qo((size_t)nq + 1), lens((size_t)nq);
    for (int32_t i = 0; i <= nq; ++i) qo[i] = q_off[i] - qbase;
    for (int32_t i = 0; i < nq; ++i) lens[i] = qo[i + 1] - qo[i];
    if (!same_key(ctx->splan, db, nq, k, lens, ctx->gen)) {
        destroy_search_plan(ctx);
        SearchPlan *p = nullptr;
        swh_status s = build_plan(ctx, db, nq, k, qo, p);
        if (s != SWH_OK) return s;
        if (!p) return SWH_OK;   // eager path
        ctx->splan = p;
    }
    SearchPlan *p = ctx->splan;
    hipStream_t st = ctx->own_stream;
    if (p->qtotal) std::memcpy(p->q_stage, q_cat + qbase, (size_t)p->qtotal);
    hipError_t e;
    hipEventRecord(ctx->ev[2], st);
    if ((e = hipGraphLaunch(p->exec, st)) != hipSuccess) return hip_fail(ctx, e, "search graph launch");
    hipEventRecord(ctx->ev[3], st);
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(ctx, e, "search graph");
    if (p->out_words[0] != INT32_MAX)
        return fail(ctx, SWH_E_ALPHABET, "queries: byte at position " + std::to_string(p->out_words[0]) +
                                             " of the concatenation is not in the alphabet");
    if (cancelled(ctx)) return cancel_status(ctx);
    if (p->out_words[2]) return fail(ctx, SWH_E_TIMEOUT, "strip wavefront wait expired");
    if (p->out_words[3]) return fail(ctx, SWH_E_TIMEOUT, "database search: a hand-over wait expired");
    if (p->out_words[1] > 0) return SWH_OK;   // 16-bit saturation: the eager path recomputes those pairs
    float ms = 0.f;
    hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]);
    stats.cells = p->cells;
    stats.ms_inter = ms;
    stats.intra_pairs = p->long_pairs;
    stats.graph = true;
    const size_t nh = (size_t)nq * k;
    for (size_t i = 0; i < nh; ++i) {
        hits[i].db_index = p->out_idx[i];
        hits[i].score = p->out_idx[i] >= 0 ? p->out_score[i] : -1;
        hits[i].reserved = 0;
    }
    done = true;
    return SWH_OK;
}

}  // namespace swh
