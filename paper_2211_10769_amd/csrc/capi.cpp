// capi.cpp -- the extern "C" entry points of libswh.so (declared in
// include/swh.h): argument validation, context lifetime, error text.
//
// Every entry point runs its body inside guarded(): nothing thrown inside the
// library (std::bad_alloc from a host container, anything else) crosses the
// C ABI.  A failed host allocation becomes SWH_E_NOMEM, any other exception
// SWH_E_DEVICE; device work already queued is drained first, so no queued
// copy can still write into a host buffer of the aborted call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <exception>
#include <new>
#include <string>

#include "context.h"
#include "batch.h"
#include "db.h"
#include "prefilter.h"
#include "tune.h"

namespace swh {

swh_status fail(swh_ctx *ctx, swh_status st, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return st;
}

swh_status hip_fail(swh_ctx *ctx, hipError_t e, const char *what)
{
    return fail(ctx, SWH_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

swh_status ensure(swh_ctx *ctx, DevBuf &buf, size_t bytes, const char *what)
{
    if (buf.cap >= bytes && buf.p) return SWH_OK;
    // buffers that are members of the context count towards its memory cap
    const bool own = (const char *)&buf >= (const char *)ctx && (const char *)&buf < (const char *)(ctx + 1);
    if (buf.p) {
        hipDeviceSynchronize();
        hipFree(buf.p);
        if (own) ctx->held -= buf.cap;
        buf.p = nullptr;
        buf.cap = 0;
    }
    size_t want = bytes < 4096 ? 4096 : bytes + bytes / 8;
    if (own && ctx->opt.mem_cap > 0) {
        const size_t cap = (size_t)ctx->opt.mem_cap;
        if (ctx->held + want > cap) want = std::max<size_t>(bytes, 1);
        if (ctx->held + want > cap)
            return fail(ctx, SWH_E_NOMEM, std::string(what) + " needs " + std::to_string(want) +
                                              " bytes beyond the context's memory cap of " + std::to_string(cap) +
                                              " (" + std::to_string(ctx->held) + " held)");
    }
    hipError_t e = hipMalloc(&buf.p, want);
    if (e != hipSuccess) {
        buf.p = nullptr;
        (void)hipGetLastError();
        return fail(ctx, SWH_E_NOMEM, std::string("cannot allocate ") + std::to_string(want) + " bytes for " + what);
    }
    buf.cap = want;
    if (own) {
        ctx->held += want;
        ++ctx->gen;
    }
    return SWH_OK;
}

size_t cap_room(const swh_ctx *ctx)
{
    if (ctx->opt.mem_cap <= 0) return SIZE_MAX;
    const size_t cap = (size_t)ctx->opt.mem_cap;
    return ctx->held >= cap ? 0 : cap - ctx->held;
}

swh_status cancel_status(swh_ctx *ctx) { return fail(ctx, SWH_E_CANCELLED, "cancelled by swh_cancel"); }

swh_status make_scoring(swh_ctx *ctx, const swh_scoring *in, Scoring &out)
{
    if (!in) return fail(ctx, SWH_E_INVAL, "scoring is NULL");
    if (!in->alphabet || !in->matrix) return fail(ctx, SWH_E_INVAL, "scoring alphabet or matrix is NULL");
    if (in->alphabet_size < 1 || in->alphabet_size > 32)
        return fail(ctx, SWH_E_INVAL, "alphabet_size must be in 1..32");
    if (in->gap_open <= 0 || in->gap_extend <= 0 || in->gap_extend > in->gap_open || in->gap_open > 65535)
        return fail(ctx, SWH_E_INVAL, "gap penalties must satisfy 0 < gap_extend <= gap_open <= 65535");
    std::memset(out.lut, 0xFF, sizeof(out.lut));
    for (int k = 0; k < in->alphabet_size; ++k) {
        unsigned char c = (unsigned char)in->alphabet[k];
        if (c == 0) return fail(ctx, SWH_E_INVAL, "alphabet shorter than alphabet_size");
        unsigned char up = (c >= 'a' && c <= 'z') ? (unsigned char)(c - 'a' + 'A') : c;
        if (out.lut[up] != 0xFF) return fail(ctx, SWH_E_INVAL, "alphabet repeats a symbol");
        out.lut[up] = (uint8_t)k;
        if (up >= 'A' && up <= 'Z') out.lut[up - 'A' + 'a'] = (uint8_t)k;
    }
    out.asize = in->alphabet_size;
    out.smax = -128;
    out.smin = 127;
    for (int k = 0; k < out.asize * out.asize; ++k) {
        out.mat[k] = in->matrix[k];
        out.smax = out.smax > in->matrix[k] ? out.smax : in->matrix[k];
        out.smin = out.smin < in->matrix[k] ? out.smin : in->matrix[k];
    }
    out.o = in->gap_open;
    out.e = in->gap_extend;
    return SWH_OK;
}

namespace {

void set_err_noexcept(swh_ctx *ctx, const char *msg) noexcept
{
    if (!ctx) return;
    try {
        ctx->err = msg;
    } catch (...) {
        ctx->err.clear();
    }
}

// The exception barrier of every entry point (see the file comment).
template <class F>
swh_status guarded(swh_ctx *ctx, F &&body) noexcept
{
    try {
        return body();
    } catch (const std::bad_alloc &) {
        (void)hipDeviceSynchronize();
        set_err_noexcept(ctx, "host memory allocation failed inside the library (std::bad_alloc)");
        return SWH_E_NOMEM;
    } catch (const std::exception &x) {
        (void)hipDeviceSynchronize();
        if (ctx) {
            try {
                ctx->err = std::string("internal error: ") + x.what();
            } catch (...) {
                ctx->err.clear();
            }
        }
        return SWH_E_DEVICE;
    } catch (...) {
        (void)hipDeviceSynchronize();
        set_err_noexcept(ctx, "internal error (unknown exception)");
        return SWH_E_DEVICE;
    }
}

// Start of the work of an entry point, after its argument checks: the
// device, a cleared cancellation flag, and the fault-injection option.
swh_status begin_call(swh_ctx *ctx)
{
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SWH_E_DEVICE, "hipSetDevice failed");
    if (ctx->cancel_host) __atomic_store_n(ctx->cancel_host, 0, __ATOMIC_RELEASE);
    ctx->passes16 = 0;
    ctx->saturated16 = 0;
    if (ctx->opt.fault_nomem) {
        ctx->opt.fault_nomem = 0;
        throw std::bad_alloc();
    }
    return SWH_OK;
}

// Make the context's stream wait for the work queued so far on the caller's stream.
swh_status order_after(swh_ctx *ctx, void *stream)
{
    hipError_t e;
    if ((e = hipEventRecord(ctx->ev_in, (hipStream_t)stream)) != hipSuccess ||
        (e = hipStreamWaitEvent(ctx->own_stream, ctx->ev_in, 0)) != hipSuccess)
        return hip_fail(ctx, e, "stream ordering");
    return SWH_OK;
}

swh_status check_pair(swh_ctx *ctx, const void *q, int64_t qlen, const void *t, int64_t tlen, const Scoring &sc,
                      int mode, swh_alignment *out)
{
    if (!out) return fail(ctx, SWH_E_INVAL, "out is NULL");
    if (qlen < 0 || tlen < 0) return fail(ctx, SWH_E_INVAL, "negative sequence length");
    if ((qlen && !q) || (tlen && !t)) return fail(ctx, SWH_E_INVAL, "sequence pointer is NULL");
    const int forms = mode & (SWH_GLOBAL | SWH_SEMIGLOBAL | SWH_OVERLAP);
    const bool global = forms != 0;
    if (forms & (forms - 1))
        return fail(ctx, SWH_E_INVAL, "SWH_GLOBAL, SWH_SEMIGLOBAL and SWH_OVERLAP exclude each other");
    mode &= ~(SWH_GLOBAL | SWH_SEMIGLOBAL | SWH_OVERLAP);
    if (mode < SWH_MODE_SCORE || mode > SWH_MODE_CIGAR) return fail(ctx, SWH_E_INVAL, "unknown mode");
    if (qlen >= (int64_t)1 << 31 || tlen >= (int64_t)1 << 31)
        return fail(ctx, SWH_E_RANGE, "sequence longer than 2^31 - 1");
    const int64_t smax = sc.smax > 0 ? sc.smax : 1;
    const int64_t sabs = sc.smax > -sc.smin ? sc.smax : -sc.smin;
    if ((qlen < tlen ? qlen : tlen) * (sabs > 0 ? sabs : 1) >= ((int64_t)1 << 26))
        return fail(ctx, SWH_E_RANGE, "min(qlen, tlen) * max|s| must stay below 2^26");
    if (mode == SWH_MODE_CIGAR && (smax + sc.e) * (qlen + tlen) + sc.o >= ((int64_t)1 << 27))
        return fail(ctx, SWH_E_RANGE, "(max s + gap_extend) * (qlen + tlen) + gap_open must stay below 2^27");
    if (global) {
        const int64_t low = sc.e > -sc.smin ? sc.e : -sc.smin;
        if ((qlen + tlen) * (low + smax) + 2 * (int64_t)sc.o >= ((int64_t)1 << 27))
            return fail(ctx, SWH_E_RANGE,
                        "global: (qlen + tlen) * (max(gap_extend, |min s|) + max s) + 2 gap_open must stay below 2^27");
    }
    return SWH_OK;
}

}  // namespace

}  // namespace swh

using namespace swh;

namespace {

swh_status search_common(swh_ctx *ctx, const swh_db *db, int32_t nq, const char *q_cat, const int64_t *q_off,
                         int32_t k, swh_hit *hits, int32_t *scores, swh_search_stats *stats, void *dev_stream,
                         bool dev)
{
    ctx->err.clear();
    if (!db) return fail(ctx, SWH_E_INVAL, "database is NULL");
    if (db->device != ctx->device) return fail(ctx, SWH_E_INVAL, "database lives on another device");
    if (nq < 0 || (nq > 0 && (!q_off || (!q_cat && q_off[nq] > q_off[0]))))
        return fail(ctx, SWH_E_INVAL, "bad query arguments");
    if (hits && (k < 1 || k > 32)) return fail(ctx, SWH_E_INVAL, "k must be in 1..32");
    if (stats && stats->struct_size < sizeof(swh_search_stats))
        return fail(ctx, SWH_E_INVAL, "stats->struct_size too small");
    swh_status s = begin_call(ctx);
    if (s != SWH_OK) return s;
    if (dev && (s = order_after(ctx, dev_stream)) != SWH_OK) return s;
    DbStats ds;
    s = db_search(ctx, db, nq, q_cat, q_off, k, hits, scores, ds, dev);
    if (s == SWH_OK && stats) {
        stats->cells = ds.cells;
        stats->ms_inter = ds.ms_inter;
        stats->ms_intra = ds.ms_intra;
        stats->ms_topk = ds.ms_topk;
        stats->saturated = ds.redo;
        stats->intra_pairs = ds.intra_pairs;
        stats->graph = ds.graph ? 1 : 0;
        stats->reserved2 = 0;
    }
    return s;
}

swh_status model_ok(swh_ctx *ctx, const swh_model *m)
{
    if (!m) return fail(ctx, SWH_E_INVAL, "model is NULL");
    if (m->device != ctx->device) return fail(ctx, SWH_E_INVAL, "model lives on another device");
    return SWH_OK;
}

swh_status batch_common(swh_ctx *ctx, int64_t npairs, const char *q_cat, const int64_t *q_off, const char *t_cat,
                        const int64_t *t_off, const swh_scoring *scoring, int mode, swh_alignment *out,
                        char *cigar_cat, int64_t cigar_cap, int64_t *cigar_off, swh_stats *stats, void *dev_stream,
                        bool dev)
{
    ctx->err.clear();
    Scoring sc;
    swh_status s = make_scoring(ctx, scoring, sc);
    if (s != SWH_OK) return s;
    if (npairs < 0) return fail(ctx, SWH_E_INVAL, "npairs is negative");
    if (npairs > 0 && (!q_off || !t_off || !out)) return fail(ctx, SWH_E_INVAL, "offsets or out is NULL");
    const int forms = mode & (SWH_GLOBAL | SWH_SEMIGLOBAL | SWH_OVERLAP);
    if (forms & (forms - 1))
        return fail(ctx, SWH_E_INVAL, "SWH_GLOBAL, SWH_SEMIGLOBAL and SWH_OVERLAP exclude each other");
    const int base = mode & ~(SWH_GLOBAL | SWH_SEMIGLOBAL | SWH_OVERLAP);
    if (base < SWH_MODE_SCORE || base > SWH_MODE_CIGAR) return fail(ctx, SWH_E_INVAL, "unknown mode");
    if (base == SWH_MODE_CIGAR && !cigar_off) return fail(ctx, SWH_E_INVAL, "cigar_off is NULL");
    if (stats && stats->struct_size < sizeof(swh_stats)) return fail(ctx, SWH_E_INVAL, "stats->struct_size too small");
    if (npairs >= ((int64_t)1 << 31)) return fail(ctx, SWH_E_RANGE, "more than 2^31 - 1 pairs");
    for (int64_t i = 0; i < npairs; ++i) {
        const int64_t qlen = q_off[i + 1] - q_off[i], tlen = t_off[i + 1] - t_off[i];
        if (qlen < 0 || tlen < 0) return fail(ctx, SWH_E_INVAL, "offsets decrease at pair " + std::to_string(i));
        swh_alignment dummy;
        if ((s = check_pair(ctx, qlen ? q_cat : nullptr, qlen, tlen ? t_cat : nullptr, tlen, sc, mode, &dummy)) !=
            SWH_OK)
            return fail(ctx, s, "pair " + std::to_string(i) + ": " + ctx->err);
    }
    if ((s = begin_call(ctx)) != SWH_OK) return s;
    if (dev && (s = order_after(ctx, dev_stream)) != SWH_OK) return s;
    s = align_batch(ctx, npairs, q_cat, q_off, t_cat, t_off, sc, mode, out, cigar_cat, cigar_cap, cigar_off, stats,
                    dev);
    if (stats) {
        stats->passes_int16 = ctx->passes16;
        stats->saturated_int16 = ctx->saturated16;
    }
    return s;
}

}  // namespace

extern "C" {

swh_status swh_create(int device, swh_ctx **out)
{
    return guarded(nullptr, [&]() -> swh_status {
        if (!out) return SWH_E_INVAL;
        *out = nullptr;
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
            (void)hipGetLastError();
            return SWH_E_DEVICE;
        }
        if (device < 0 || device >= count) return SWH_E_INVAL;
        swh_ctx *ctx = new (std::nothrow) swh_ctx();
        if (!ctx) return SWH_E_NOMEM;
        ctx->device = device;
        if (hipSetDevice(device) != hipSuccess ||
            hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return SWH_E_DEVICE;
        }
        bool ok = hipStreamCreateWithFlags(&ctx->aux_stream, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming) == hipSuccess;
        for (auto &ev : ctx->ev) ok = ok && hipEventCreate(&ev) == hipSuccess;
        // the cancellation flag: pinned, coherent host memory the kernels read uncached
        void *hp = nullptr, *dp = nullptr;
        ok = ok && hipHostMalloc(&hp, 64, hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess;
        if (hp) {
            ctx->cancel_host = (int32_t *)hp;
            *ctx->cancel_host = 0;
            ok = ok && hipHostGetDevicePointer(&dp, hp, 0) == hipSuccess;
            ctx->cancel_dev = (int32_t *)dp;
        }
        if (!ok) {
            (void)hipGetLastError();
            swh_destroy(ctx);
            return SWH_E_DEVICE;
        }
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, device) == hipSuccess) {
            ctx->num_cu = p.multiProcessorCount;
            ctx->device_name = std::string(p.name) + " " + p.gcnArchName + " " +
                               std::to_string(p.multiProcessorCount) + "cu";
        }
        *out = ctx;
        return SWH_OK;
    });
}

void swh_destroy(swh_ctx *ctx)
{
    if (!ctx) return;
    try {
        hipSetDevice(ctx->device);
        if (ctx->own_stream) hipStreamSynchronize(ctx->own_stream);
        if (ctx->aux_stream) hipStreamSynchronize(ctx->aux_stream);
        for (DevBuf *b : ctx->all())
            if (b->p) hipFree(b->p);
        ctx->tb_arena.free_all(ctx->held);
        destroy_search_plan(ctx);
        for (auto &ev : ctx->ev)
            if (ev) hipEventDestroy(ev);
        if (ctx->ev_in) hipEventDestroy(ctx->ev_in);
        if (ctx->ev_fork) hipEventDestroy(ctx->ev_fork);
        if (ctx->ev_join) hipEventDestroy(ctx->ev_join);
        if (ctx->cancel_host) hipHostFree(ctx->cancel_host);
        if (ctx->tb_ops_host) hipHostFree(ctx->tb_ops_host);
        if (ctx->own_stream) hipStreamDestroy(ctx->own_stream);
        if (ctx->aux_stream) hipStreamDestroy(ctx->aux_stream);
        delete ctx;
    } catch (...) {
    }
}

const char *swh_last_error(const swh_ctx *ctx)
{
    if (!ctx) return "no context";
    return ctx->err.c_str();
}

swh_status swh_cancel(swh_ctx *ctx)
{
    // may run on another thread than the call it stops: touches only the flag
    if (!ctx || !ctx->cancel_host) return SWH_E_INVAL;
    __atomic_store_n(ctx->cancel_host, 1, __ATOMIC_RELEASE);
    return SWH_OK;
}

swh_status swh_set_option(swh_ctx *ctx, int32_t option, int64_t value)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        ctx->err.clear();
        Options &o = ctx->opt;
        auto bad = [&](const char *what) { return fail(ctx, SWH_E_INVAL, std::string("option value: ") + what); };
        switch (option) {
        case SWH_OPT_ROWS_PER_LANE:
            if (value != 0 && value != 4 && value != 8 && value != 16 && value != 20 && value != 24 && value != 32)
                return bad("rows per lane must be 0, 4, 8, 16, 20, 24 or 32");
            o.rows = (int32_t)value;
            return SWH_OK;
        case SWH_OPT_GRID:
            if (value < 0 || value > (1 << 20)) return bad("grid must be in 0 .. 2^20");
            o.grid = (int32_t)value;
            ++ctx->gen;   // a captured search keeps its launch shape
            return SWH_OK;
        case SWH_OPT_BAND_ROWS:
            if (value < -1 || value > (1 << 30)) return bad("band rows must be -1, 0 or a positive row count");
            o.band_rows = (int32_t)value;
            return SWH_OK;
        case SWH_OPT_TB_LEAF:
            if (value < 0 || value > 524288) return bad("leaf cells must be in 0 .. 524288");
            o.tb_leaf = value;
            return SWH_OK;
        case SWH_OPT_GRAPH:
            if (value < 0 || value > 2) return bad("graph must be 0, 1 or 2");
            o.graph = (int32_t)value;
            return SWH_OK;
        case SWH_OPT_PRUNE:
            if (value != 0 && value != 1) return bad("prune must be 0 or 1");
            o.prune = (int32_t)value;
            return SWH_OK;
        case SWH_OPT_MEM_CAP:
            if (value < 0) return bad("memory cap must be >= 0");
            o.mem_cap = value;
            return SWH_OK;
        case SWH_OPT_INT16:
            if (value < 0 || value > 2) return bad("int16 must be 0, 1 or 2");
            o.int16 = (int32_t)value;
            return SWH_OK;
        case SWH_OPT_INTER_MAX:
            if (value != 0 && (value < 32 || value > 8192)) return bad("inter-task maximum must be 0 or 32 .. 8192");
            o.inter_max = (int32_t)value;
            return SWH_OK;
        case SWH_OPT_PF_RANK:
            if (value < 0 || value > 2) return bad("prefilter ranking must be 0, 1 or 2");
            o.pf_rank = (int32_t)value;
            return SWH_OK;
        case SWH_OPT_DB_WAVES:
            if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8 && value != 12 && value != 16)
                return bad("database waves must be 0, 1, 2, 4, 8, 12 or 16");
            o.db_waves = (int32_t)value;
            ++ctx->gen;   // a captured search keeps its launch shape
            return SWH_OK;
        case SWH_OPT_DB_ROUTE:
            if (value < -1 || value > 100000) return bad("database routing must be -1, 0 or a percentage");
            o.db_route = (int32_t)value;
            ++ctx->gen;
            return SWH_OK;
        case SWH_OPT_FAULT_NOMEM:
            if (value != 0 && value != 1) return bad("fault injection must be 0 or 1");
            o.fault_nomem = (int32_t)value;
            return SWH_OK;
        default:
            return fail(ctx, SWH_E_INVAL, "unknown option " + std::to_string(option));
        }
    });
}

swh_status swh_get_option(const swh_ctx *ctx, int32_t option, int64_t *value)
{
    if (!ctx || !value) return SWH_E_INVAL;
    const Options &o = ctx->opt;
    switch (option) {
    case SWH_OPT_ROWS_PER_LANE: *value = o.rows; return SWH_OK;
    case SWH_OPT_GRID: *value = o.grid; return SWH_OK;
    case SWH_OPT_BAND_ROWS: *value = o.band_rows; return SWH_OK;
    case SWH_OPT_TB_LEAF: *value = o.tb_leaf; return SWH_OK;
    case SWH_OPT_GRAPH: *value = o.graph; return SWH_OK;
    case SWH_OPT_PRUNE: *value = o.prune; return SWH_OK;
    case SWH_OPT_MEM_CAP: *value = o.mem_cap; return SWH_OK;
    case SWH_OPT_INT16: *value = o.int16; return SWH_OK;
    case SWH_OPT_INTER_MAX: *value = o.inter_max; return SWH_OK;
    case SWH_OPT_PF_RANK: *value = o.pf_rank; return SWH_OK;
    case SWH_OPT_DB_WAVES: *value = o.db_waves; return SWH_OK;
    case SWH_OPT_DB_ROUTE: *value = o.db_route; return SWH_OK;
    case SWH_OPT_FAULT_NOMEM: *value = o.fault_nomem; return SWH_OK;
    default: return SWH_E_INVAL;
    }
}

swh_status swh_align(swh_ctx *ctx, const char *q, int64_t qlen, const char *t, int64_t tlen,
                     const swh_scoring *scoring, int mode, swh_alignment *out, char *cigar, int64_t cigar_cap,
                     int64_t *cigar_len, swh_stats *stats)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        ctx->err.clear();
        Scoring sc;
        swh_status s = make_scoring(ctx, scoring, sc);
        if (s != SWH_OK) return s;
        if ((s = check_pair(ctx, q, qlen, t, tlen, sc, mode, out)) != SWH_OK) return s;
        if (stats && stats->struct_size < sizeof(swh_stats))
            return fail(ctx, SWH_E_INVAL, "stats->struct_size too small");
        if ((s = begin_call(ctx)) != SWH_OK) return s;
        hipStream_t st = ctx->own_stream;
        if ((s = ensure(ctx, ctx->qraw, (size_t)qlen + 1, "query copy")) != SWH_OK) return s;
        if ((s = ensure(ctx, ctx->traw, (size_t)tlen + 1, "target copy")) != SWH_OK) return s;
        hipError_t e;
        if (qlen && (e = hipMemcpyAsync(ctx->qraw.p, q, (size_t)qlen, hipMemcpyHostToDevice, st)) != hipSuccess)
            return hip_fail(ctx, e, "hipMemcpyAsync(query)");
        if (tlen && (e = hipMemcpyAsync(ctx->traw.p, t, (size_t)tlen, hipMemcpyHostToDevice, st)) != hipSuccess)
            return hip_fail(ctx, e, "hipMemcpyAsync(target)");
        s = align_device(ctx, (const char *)ctx->qraw.p, qlen, (const char *)ctx->traw.p, tlen, sc, mode, st, out,
                         cigar, cigar_cap, cigar_len, stats);
        if (stats) {
            stats->passes_int16 = ctx->passes16;
            stats->saturated_int16 = ctx->saturated16;
        }
        return s;
    });
}

swh_status swh_align_dev(swh_ctx *ctx, const char *q_dev, int64_t qlen, const char *t_dev, int64_t tlen,
                         const swh_scoring *scoring, int mode, void *stream, swh_alignment *out, char *cigar,
                         int64_t cigar_cap, int64_t *cigar_len, swh_stats *stats)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        ctx->err.clear();
        Scoring sc;
        swh_status s = make_scoring(ctx, scoring, sc);
        if (s != SWH_OK) return s;
        if ((s = check_pair(ctx, q_dev, qlen, t_dev, tlen, sc, mode, out)) != SWH_OK) return s;
        if (stats && stats->struct_size < sizeof(swh_stats))
            return fail(ctx, SWH_E_INVAL, "stats->struct_size too small");
        if ((s = begin_call(ctx)) != SWH_OK) return s;
        s = align_device(ctx, q_dev, qlen, t_dev, tlen, sc, mode, (hipStream_t)stream, out, cigar, cigar_cap,
                         cigar_len, stats);
        if (stats) {
            stats->passes_int16 = ctx->passes16;
            stats->saturated_int16 = ctx->saturated16;
        }
        return s;
    });
}

swh_status swh_align_batch(swh_ctx *ctx, int64_t npairs, const char *q_cat, const int64_t *q_off, const char *t_cat,
                           const int64_t *t_off, const swh_scoring *scoring, int mode, swh_alignment *out,
                           char *cigar_cat, int64_t cigar_cap, int64_t *cigar_off, swh_stats *stats)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        return batch_common(ctx, npairs, q_cat, q_off, t_cat, t_off, scoring, mode, out, cigar_cat, cigar_cap,
                            cigar_off, stats, nullptr, false);
    });
}

swh_status swh_align_batch_dev(swh_ctx *ctx, int64_t npairs, const char *q_cat_dev, const int64_t *q_off,
                               const char *t_cat_dev, const int64_t *t_off, const swh_scoring *scoring, int mode,
                               void *stream, swh_alignment *out, char *cigar_cat, int64_t cigar_cap,
                               int64_t *cigar_off, swh_stats *stats)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        return batch_common(ctx, npairs, q_cat_dev, q_off, t_cat_dev, t_off, scoring, mode, out, cigar_cat,
                            cigar_cap, cigar_off, stats, stream, true);
    });
}

swh_status swh_autotune(swh_ctx *ctx, const swh_scoring *scoring, int64_t max_rows, double cells_per_trial)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        ctx->err.clear();
        Scoring sc;
        swh_status s = make_scoring(ctx, scoring, sc);
        if (s != SWH_OK) return s;
        if (max_rows < 1 || max_rows >= ((int64_t)1 << 31)) return fail(ctx, SWH_E_INVAL, "max_rows out of range");
        if (!(cells_per_trial > 0.0) || cells_per_trial > 1e13)
            return fail(ctx, SWH_E_INVAL, "cells_per_trial must be in (0, 1e13]");
        if ((s = begin_call(ctx)) != SWH_OK) return s;
        return autotune(ctx, sc, max_rows, cells_per_trial);
    });
}

swh_status swh_autotune_db(swh_ctx *ctx, const swh_scoring *scoring, int32_t *inter_max)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        ctx->err.clear();
        Scoring sc;
        swh_status s = make_scoring(ctx, scoring, sc);
        if (s != SWH_OK) return s;
        if ((s = begin_call(ctx)) != SWH_OK) return s;
        int32_t v = 0;
        if ((s = autotune_db(ctx, sc, scoring, v)) != SWH_OK) return s;
        if (inter_max) *inter_max = v;
        return SWH_OK;
    });
}

swh_status swh_tune_save(const swh_ctx *ctx, const char *path)
{
    if (!ctx || !path) return SWH_E_INVAL;
    try {
        return tune_save(ctx, path);
    } catch (...) {
        return SWH_E_NOMEM;
    }
}

swh_status swh_tune_load(swh_ctx *ctx, const char *path)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        ctx->err.clear();
        if (!path) return fail(ctx, SWH_E_INVAL, "path is NULL");
        return tune_load(ctx, path);
    });
}

swh_status swh_tune_get(const swh_ctx *ctx, swh_tune_entry *out, int32_t cap, int32_t *count)
{
    if (!ctx || !count || cap < 0 || (cap > 0 && !out)) return SWH_E_INVAL;
    *count = (int32_t)ctx->tune.size();
    for (int32_t i = 0; i < cap && i < *count; ++i) out[i] = ctx->tune[i];
    return SWH_OK;
}

swh_status swh_tune_set(swh_ctx *ctx, const swh_tune_entry *entries, int32_t count)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        ctx->err.clear();
        if (count < 0 || count > 64 || (count > 0 && !entries)) return fail(ctx, SWH_E_INVAL, "bad table size");
        for (int32_t i = 0; i < count; ++i) {
            const swh_tune_entry &t = entries[i];
            const int R = t.rows_per_lane;
            if (R != 4 && R != 8 && R != 16 && R != 20 && R != 24 && R != 32)
                return fail(ctx, SWH_E_INVAL, "rows_per_lane must be 4, 8, 16, 20, 24 or 32");
            if (t.waves_per_simd < 0 || t.waves_per_simd > 8)
                return fail(ctx, SWH_E_INVAL, "waves_per_simd must be in 0..8");
            if (t.max_rows < 1 || (i > 0 && t.max_rows <= entries[i - 1].max_rows))
                return fail(ctx, SWH_E_INVAL, "max_rows must be positive and increasing");
        }
        ctx->tune.assign(entries, entries + count);
        return SWH_OK;
    });
}

swh_status swh_db_create(swh_ctx *ctx, int64_t ndb, const char *db_cat, const int64_t *db_off,
                         const swh_scoring *scoring, swh_db **out)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        ctx->err.clear();
        if (!out) return fail(ctx, SWH_E_INVAL, "out is NULL");
        *out = nullptr;
        if (ndb > 0 && (!db_cat || !db_off)) return fail(ctx, SWH_E_INVAL, "database pointers are NULL");
        Scoring sc;
        swh_status s = make_scoring(ctx, scoring, sc);
        if (s != SWH_OK) return s;
        if ((s = begin_call(ctx)) != SWH_OK) return s;
        return db_create(ctx, ndb, db_cat, db_off, sc, out);
    });
}

void swh_db_destroy(swh_db *db)
{
    try {
        db_destroy(db);
    } catch (...) {
    }
}

swh_status swh_db_search(swh_ctx *ctx, const swh_db *db, int32_t nq, const char *q_cat, const int64_t *q_off,
                         int32_t k, swh_hit *hits, swh_search_stats *stats)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        if (!hits) return fail(ctx, SWH_E_INVAL, "hits is NULL");
        return search_common(ctx, db, nq, q_cat, q_off, k, hits, nullptr, stats, nullptr, false);
    });
}

swh_status swh_db_search_dev(swh_ctx *ctx, const swh_db *db, int32_t nq, const char *q_cat_dev, const int64_t *q_off,
                             int32_t k, void *stream, swh_hit *hits, swh_search_stats *stats)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        if (!hits) return fail(ctx, SWH_E_INVAL, "hits is NULL");
        return search_common(ctx, db, nq, q_cat_dev, q_off, k, hits, nullptr, stats, stream, true);
    });
}

swh_status swh_db_scores(swh_ctx *ctx, const swh_db *db, int32_t nq, const char *q_cat, const int64_t *q_off,
                         int32_t *scores, swh_search_stats *stats)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        if (!scores) return fail(ctx, SWH_E_INVAL, "scores is NULL");
        return search_common(ctx, db, nq, q_cat, q_off, 0, nullptr, scores, stats, nullptr, false);
    });
}

swh_status swh_model_create(swh_ctx *ctx, const swh_scoring *scoring, const float *theta, const float *mu,
                            const float *sd, uint64_t seed, swh_model **out)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        ctx->err.clear();
        if (!out) return fail(ctx, SWH_E_INVAL, "out is NULL");
        *out = nullptr;
        Scoring sc;
        swh_status s = make_scoring(ctx, scoring, sc);
        if (s != SWH_OK) return s;
        if ((s = begin_call(ctx)) != SWH_OK) return s;
        return model_create(ctx, sc, theta, mu, sd, seed, out);
    });
}

void swh_model_destroy(swh_model *model)
{
    try {
        model_destroy(model);
    } catch (...) {
    }
}

swh_status swh_model_get(swh_ctx *ctx, const swh_model *model, float *theta, float *mu, float *sd)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        ctx->err.clear();
        swh_status s = model_ok(ctx, model);
        if (s == SWH_OK) s = begin_call(ctx);
        return s != SWH_OK ? s : model_get(ctx, model, theta, mu, sd);
    });
}

swh_status swh_model_set(swh_ctx *ctx, swh_model *model, const float *theta, const float *mu, const float *sd)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        ctx->err.clear();
        swh_status s = model_ok(ctx, model);
        if (s == SWH_OK) s = begin_call(ctx);
        return s != SWH_OK ? s : model_set(ctx, model, theta, mu, sd);
    });
}

swh_status swh_model_save(swh_ctx *ctx, const swh_model *model, const char *path)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        ctx->err.clear();
        swh_status s = model_ok(ctx, model);
        if (s == SWH_OK && !path) s = fail(ctx, SWH_E_INVAL, "path is NULL");
        if (s == SWH_OK) s = begin_call(ctx);
        return s != SWH_OK ? s : model_save(ctx, model, path);
    });
}

swh_status swh_model_load(swh_ctx *ctx, const char *path, swh_model **out)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        ctx->err.clear();
        if (!path || !out) return fail(ctx, SWH_E_INVAL, "path or out is NULL");
        *out = nullptr;
        swh_status s = begin_call(ctx);
        return s != SWH_OK ? s : model_load(ctx, path, out);
    });
}

swh_status swh_prefilter_train(swh_ctx *ctx, swh_model *model, const swh_scoring *scoring, int64_t nseq,
                               const char *seq_cat, const int64_t *seq_off, int64_t npairs, const int32_t *pair_row,
                               const int32_t *pair_col, const int32_t *scores, const swh_train_cfg *cfg,
                               int32_t *labels_out, swh_train_stats *stats)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        ctx->err.clear();
        swh_status s = model_ok(ctx, model);
        if (s != SWH_OK) return s;
        Scoring sc;
        if ((s = make_scoring(ctx, scoring, sc)) != SWH_OK) return s;
        if (sc.asize != model->asize) return fail(ctx, SWH_E_INVAL, "scoring alphabet differs from the model's");
        if (!cfg || cfg->struct_size < sizeof(swh_train_cfg))
            return fail(ctx, SWH_E_INVAL, "cfg missing or too small");
        if (cfg->epochs < 1 || cfg->batch < 64 || cfg->batch % 64 != 0 || !(cfg->lr > 0.0))
            return fail(ctx, SWH_E_INVAL, "cfg: epochs >= 1, batch a positive multiple of 64, lr > 0");
        if (nseq < 0 || npairs < cfg->batch || (nseq > 0 && !seq_off) || !pair_row || !pair_col)
            return fail(ctx, SWH_E_INVAL, "need a sequence pool and at least one batch of pairs");
        if (stats && stats->struct_size < sizeof(swh_train_stats)) return fail(ctx, SWH_E_INVAL, "stats too small");
        if (npairs >= ((int64_t)1 << 31)) return fail(ctx, SWH_E_RANGE, "more than 2^31 - 1 pairs");
        if ((s = begin_call(ctx)) != SWH_OK) return s;
        TrainStats ts;
        s = prefilter_train(ctx, sc, nseq, seq_cat, seq_off, npairs, pair_row, pair_col, scores, cfg->epochs,
                            cfg->batch, cfg->lr, cfg->seed, model, labels_out, ts);
        if (s == SWH_OK && stats) {
            stats->first_epoch_loss = ts.first_loss;
            stats->final_epoch_loss = ts.final_loss;
            stats->ms_label = ts.ms_label;
            stats->ms_features = ts.ms_features;
            stats->ms_train = ts.ms_train;
            stats->cells_label = ts.cells_label;
            stats->steps = ts.steps;
            stats->graph = ts.graph ? 1 : 0;
        }
        return s;
    });
}

swh_status swh_prefilter_search(swh_ctx *ctx, const swh_model *model, swh_db *db, int32_t nq, const char *q_cat,
                                const int64_t *q_off, int32_t k, double rescore_frac, double audit_frac,
                                uint64_t audit_seed, swh_hit *hits, swh_prefilter_stats *stats)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        ctx->err.clear();
        swh_status s = model_ok(ctx, model);
        if (s != SWH_OK) return s;
        if (!db || db->device != ctx->device) return fail(ctx, SWH_E_INVAL, "database missing or on another device");
        if (db->sc.asize != model->asize) return fail(ctx, SWH_E_INVAL, "database alphabet differs from the model's");
        if (nq < 0 || (nq > 0 && (!q_off || !hits))) return fail(ctx, SWH_E_INVAL, "bad query arguments");
        if (k < 1 || k > 32) return fail(ctx, SWH_E_INVAL, "k must be in 1..32");
        if (!(rescore_frac > 0.0 && rescore_frac <= 1.0) || !(audit_frac >= 0.0 && audit_frac <= 1.0))
            return fail(ctx, SWH_E_INVAL, "rescore_frac must be in (0, 1], audit_frac in [0, 1]");
        if (stats && stats->struct_size < sizeof(swh_prefilter_stats))
            return fail(ctx, SWH_E_INVAL, "stats too small");
        if ((s = begin_call(ctx)) != SWH_OK) return s;
        PrefilterStats ps;
        s = prefilter_search(ctx, model, db, nq, q_cat, q_off, k, rescore_frac, audit_frac, audit_seed, hits, ps);
        if (s == SWH_OK && stats) {
            stats->candidates = ps.candidates;
            stats->audited = ps.audited;
            stats->fallbacks = ps.fallbacks;
            stats->cells_rescored = ps.cells_rescored;
            stats->cells_exhaustive = ps.cells_exhaustive;
            stats->ms_features = ps.ms_features;
            stats->ms_predict = ps.ms_predict;
            stats->ms_select = ps.ms_select;
            stats->ms_rescore = ps.ms_rescore;
            stats->ms_topk = ps.ms_topk;
            stats->ms_fallback = ps.ms_fallback;
        }
        return s;
    });
}

swh_status swh_prefilter_predict(swh_ctx *ctx, const swh_model *model, swh_db *db, int32_t nq, const char *q_cat,
                                 const int64_t *q_off, float *pred)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        ctx->err.clear();
        swh_status s = model_ok(ctx, model);
        if (s != SWH_OK) return s;
        if (!db || db->device != ctx->device) return fail(ctx, SWH_E_INVAL, "database missing or on another device");
        if (db->sc.asize != model->asize) return fail(ctx, SWH_E_INVAL, "database alphabet differs from the model's");
        if (nq < 0 || (nq > 0 && (!q_off || !pred))) return fail(ctx, SWH_E_INVAL, "bad query arguments");
        if ((s = begin_call(ctx)) != SWH_OK) return s;
        return prefilter_predict(ctx, model, db, nq, q_cat, q_off, pred);
    });
}

swh_status swh_dipeptide_counts(swh_ctx *ctx, const swh_scoring *scoring, int64_t nseq, const char *seq_cat,
                                const int64_t *seq_off, int32_t *counts)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        ctx->err.clear();
        Scoring sc;
        swh_status s = make_scoring(ctx, scoring, sc);
        if (s != SWH_OK) return s;
        if (nseq < 0 || (nseq > 0 && (!seq_off || !counts))) return fail(ctx, SWH_E_INVAL, "bad sequence arguments");
        if ((s = begin_call(ctx)) != SWH_OK) return s;
        return dipeptide_counts(ctx, sc, nseq, seq_cat, seq_off, counts);
    });
}

swh_status swh_mlp_grad(swh_ctx *ctx, swh_model *model, int32_t B, const float *z, const float *y, double *loss,
                        float *grad)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        ctx->err.clear();
        swh_status s = model_ok(ctx, model);
        if (s != SWH_OK) return s;
        if (B < 64 || B % 64 != 0 || !z || !y || !grad) return fail(ctx, SWH_E_INVAL, "B a positive multiple of 64");
        if ((s = begin_call(ctx)) != SWH_OK) return s;
        return mlp_grad(ctx, model, B, z, y, loss, grad);
    });
}

swh_status swh_mlp_train_steps(swh_ctx *ctx, swh_model *model, int32_t B, const float *z, const float *y,
                               int32_t steps, double lr)
{
    if (!ctx) return SWH_E_INVAL;
    return guarded(ctx, [&]() -> swh_status {
        ctx->err.clear();
        swh_status s = model_ok(ctx, model);
        if (s != SWH_OK) return s;
        if (B < 64 || B % 64 != 0 || !z || !y || steps < 0 || !(lr > 0.0))
            return fail(ctx, SWH_E_INVAL, "B a positive multiple of 64, steps >= 0, lr > 0");
        if ((s = begin_call(ctx)) != SWH_OK) return s;
        return mlp_train_steps(ctx, model, B, z, y, steps, lr);
    });
}

}  // extern "C"
