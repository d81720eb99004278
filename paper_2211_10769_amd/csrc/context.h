// context.h -- the opaque swh_ctx and its grow-only device buffers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/swh.h"
#include "engine.h"

namespace swh {

struct SearchPlan;   // a captured database search (db_graph.cpp)

// A device allocation that only grows; freed with the context.
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

// Validated scoring with the symbol lookup table and the device copy of the matrix.
struct Scoring {
    uint8_t lut[256];          // byte -> code, 0xFF = not in the alphabet
    int asize = 0;
    int8_t mat[32 * 32];
    int o = 0, e = 0;
    int smax = 0, smin = 0;    // extreme matrix entries
};

// Context options (swh_set_option): speed, memory and diagnostics only.
struct Options {
    int32_t rows = 0;        // forced rows per lane (0: tuned table or rule)
    int32_t grid = 0;        // > 0: single-wave workgroups of this count
    int32_t band_rows = 0;   // rows between kept rows (0: rule, -1: no band traceback)
    int64_t tb_leaf = 0;     // largest traceback leaf in cells (0: built-in)
    int32_t graph = 1;       // prefilter training step as a HIP graph
    int32_t prune = 1;       // block pruning of reverse passes
    int64_t mem_cap = 0;     // bytes the context's own buffers may hold (0: no cap)
    int32_t int16 = 1;       // packed 16-bit local passes: 0 off, 1 batches and GPU-filling passes, 2 always
    int32_t inter_max = 0;   // database length switch (0: built-in / tuned)
    int32_t pf_rank = 1;     // prefilter ranking: 1 excess over same-length mean, 2 its z-score, 0 raw
    int32_t db_waves = 0;    // waves per database unit: 0 auto, 1, 2 or 4
    int32_t db_route = 0;    // units above this % of a CU's share go to the single-pair kernel (0: 100, -1: never)
    int32_t fault_nomem = 0; // the next entry point throws std::bad_alloc
};

// Device memory handed out in pieces that never move during one use (the
// traceback keeps pointers across levels); chunks are kept for the next use,
// so a call allocates only when it needs more than any call before it.
// held / cap: the owning context's byte count of device memory and its cap
// (0: none); chunks count towards it.
struct Arena {
    static constexpr size_t kChunk = (size_t)256 << 20;
    std::vector<void *> chunks;
    std::vector<size_t> caps;
    size_t cur = 0, used = 0;
    void reset()
    {
        cur = 0;
        used = 0;
    }
    void *get(size_t bytes, size_t &held, int64_t cap)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        while (cur < chunks.size() && used + bytes > caps[cur]) {
            ++cur;
            used = 0;
        }
        if (cur == chunks.size()) {
            size_t want = bytes > kChunk ? bytes : kChunk;
            if (cap > 0 && held + want > (size_t)cap) want = bytes;
            if (cap > 0 && held + want > (size_t)cap) return nullptr;
            void *p = nullptr;
            if (hipMalloc(&p, want) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
            chunks.push_back(p);
            caps.push_back(want);
            held += want;
            used = 0;
        }
        void *r = (char *)chunks[cur] + used;
        used += bytes;
        return r;
    }
    void free_all(size_t &held)
    {
        for (size_t k = 0; k < chunks.size(); ++k) {
            hipFree(chunks[k]);
            held -= caps[k];
        }
        chunks.clear();
        caps.clear();
        reset();
    }
};

}  // namespace swh

struct swh_ctx {
    int device = 0;
    hipStream_t own_stream = nullptr;
    hipStream_t aux_stream = nullptr;   // second stream of the context (default priority)
    int num_cu = 0;
    std::string err;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t ev_in = nullptr;   // orders the context's stream after a caller's stream
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;   // own_stream <-> aux_stream ordering
    swh::Options opt;
    // cancellation flag in pinned host memory (host view and device view)
    int32_t *cancel_host = nullptr;
    int32_t *cancel_dev = nullptr;
    // device bytes held by the context's own buffers (the memory cap counts these)
    size_t held = 0;
    // bumped whenever one of the context's buffers is (re)allocated: a captured
    // graph that uses them is valid only while it is unchanged
    uint64_t gen = 0;
    swh::SearchPlan *splan = nullptr;
    // local passes of the current call run in packed 16 bits, and those redone
    // in 32 bits after a possible saturation
    int64_t passes16 = 0, saturated16 = 0;

    // pairwise buffers
    swh::DevBuf qraw, traw;        // ASCII copies of host inputs
    swh::DevBuf qc, tc;            // codes
    swh::DevBuf qr, tr;            // reversed codes
    swh::DevBuf border, flags, misc, strip_best, mat, lut;
    // strip-kernel problem tables
    swh::DevBuf probs, strip_prob, strip_order, prob_best, sync;
    swh::PreparedStrips strips;   // host tables of the last strip launch
    // database search buffers
    swh::DevBuf qoff, db_work, db_border, db_redo, db_scatter, db_scores, db_topk;
    swh::DevBuf db_sync;                 // the inter-task kernel's ticket, abort flag and redo count
    std::vector<int64_t> pair_pos;       // score positions of the last single-pair launch (upload source)
    // batched pairs: padded per-pair copies and border rows of one launch
    swh::DevBuf bq, bt, bborder;
    // strip shapes measured by the autotuner (empty: built-in rule)
    std::vector<swh_tune_entry> tune;
    int32_t tuned_inter_max = 0;   // database length switch measured by the autotuner (0: built-in)
    std::string device_name;
    // prefilter: query features, folded queries, predictions, selection, candidate layout
    swh::DevBuf pf_fq, pf_qlen, pf_Aq, pf_pred, pf_hist, pf_prefix, pf_marks, pf_chunk, pf_cand, pf_res, pf_groups,
        pf_perm;
    float pf_infer_ms = 0.f;
    // traceback buffers
    swh::Arena tb_arena;
    // pinned host copy of the traceback leaves' ops, kept across calls (grown by
    // doubling): copies land without staging or page faults
    char *tb_ops_host = nullptr;
    size_t tb_ops_host_cap = 0;
    swh::DevBuf tb_fwd, tb_bwd, tb_front, tb_codes_q, tb_flags, tb_leaf, tb_misc;
    // band traceback: rows kept by the forward and reverse score passes, cut tables
    swh::DevBuf keep_f, keep_r, cut_desc, cut_cnt, cut_out;
    // global alignments: the end values G(n, m) of a launch's problems
    swh::DevBuf gscores;
    std::vector<swh::DevBuf *> all() {
        return {&qraw, &traw, &qc, &tc, &qr, &tr, &border, &flags, &misc, &strip_best, &mat, &lut,
                &probs, &strip_prob, &strip_order, &prob_best, &sync,
                &qoff, &db_work, &db_border, &db_redo, &db_scatter, &db_scores, &db_topk, &db_sync,
                &bq, &bt, &bborder,
                &pf_fq, &pf_qlen, &pf_Aq, &pf_pred, &pf_hist, &pf_prefix, &pf_marks, &pf_chunk, &pf_cand,
                &pf_res, &pf_groups, &pf_perm,
                &tb_fwd, &tb_bwd, &tb_front, &tb_codes_q, &tb_flags, &tb_leaf, &tb_misc,
                &keep_f, &keep_r, &cut_desc, &cut_cnt, &cut_out, &gscores};
    }
};

namespace swh {

// Status helpers: set ctx->err and return the status.
swh_status fail(swh_ctx *ctx, swh_status st, const std::string &msg);
swh_status hip_fail(swh_ctx *ctx, hipError_t e, const char *what);
// Make sure buf holds at least bytes; on failure sets the error and returns
// SWH_E_NOMEM.  Buffers that are members of ctx count towards its memory cap.
swh_status ensure(swh_ctx *ctx, DevBuf &buf, size_t bytes, const char *what);
// Device bytes the context may still take under its memory cap (SIZE_MAX: no cap).
size_t cap_room(const swh_ctx *ctx);
// True once swh_cancel has been called during the current entry point.
inline bool cancelled(const swh_ctx *ctx)
{
    return ctx->cancel_host && __atomic_load_n(ctx->cancel_host, __ATOMIC_ACQUIRE) != 0;
}
// SWH_E_CANCELLED with its message
swh_status cancel_status(swh_ctx *ctx);
swh_status make_scoring(swh_ctx *ctx, const swh_scoring *in, Scoring &out);

// Pairwise alignment on device-resident ASCII inputs (engine.cpp).
swh_status align_device(swh_ctx *ctx, const char *q_dev, int64_t qlen, const char *t_dev, int64_t tlen,
                        const Scoring &sc, int mode, hipStream_t st, swh_alignment *out, char *cigar,
                        int64_t cigar_cap, int64_t *cigar_len, swh_stats *stats);

}  // namespace swh
