// context.h -- the opaque swh_ctx and its grow-only device buffers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/swh.h"
#include "engine.h"

namespace swh {

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

// Device memory handed out in pieces that never move during one use (the
// traceback keeps pointers across levels); chunks are kept for the next use,
// so a call allocates only when it needs more than any call before it.
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
    void *get(size_t bytes)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        while (cur < chunks.size() && used + bytes > caps[cur]) {
            ++cur;
            used = 0;
        }
        if (cur == chunks.size()) {
            const size_t cap = bytes > kChunk ? bytes : kChunk;
            void *p = nullptr;
            if (hipMalloc(&p, cap) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
            chunks.push_back(p);
            caps.push_back(cap);
            used = 0;
        }
        void *r = (char *)chunks[cur] + used;
        used += bytes;
        return r;
    }
    void free_all()
    {
        for (void *p : chunks) hipFree(p);
        chunks.clear();
        caps.clear();
        reset();
    }
};

}  // namespace swh

struct swh_ctx {
    int device = 0;
    hipStream_t own_stream = nullptr;
    int num_cu = 0;
    std::string err;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};

    // pairwise buffers
    swh::DevBuf qraw, traw;        // ASCII copies of host inputs
    swh::DevBuf qc, tc;            // codes
    swh::DevBuf qr, tr;            // reversed codes
    swh::DevBuf border, flags, misc, strip_best, mat, lut;
    // strip-kernel problem tables
    swh::DevBuf probs, strip_prob, prob_best, sync;
    std::vector<swh::Problem> h_probs;
    std::vector<int32_t> h_strip_prob;
    // database search buffers
    swh::DevBuf qoff, db_work, db_border, db_redo, db_scatter, db_scores, db_topk;
    // batched pairs: padded per-pair copies and border rows of one launch
    swh::DevBuf bq, bt, bborder;
    // strip shapes measured by the autotuner (empty: built-in rule)
    std::vector<swh_tune_entry> tune;
    // prefilter: query features, folded queries, predictions, selection, candidate layout
    swh::DevBuf pf_fq, pf_qlen, pf_Aq, pf_pred, pf_hist, pf_prefix, pf_marks, pf_chunk, pf_cand, pf_res, pf_groups,
        pf_perm;
    float pf_infer_ms = 0.f;
    // traceback buffers
    swh::Arena tb_arena;
    swh::DevBuf tb_fwd, tb_bwd, tb_front, tb_codes_q, tb_flags, tb_leaf, tb_misc;
    // band traceback: rows kept by the forward and reverse score passes, cut tables
    swh::DevBuf keep_f, keep_r, cut_desc, cut_cnt, cut_out;
    // global alignments: the end values G(n, m) of a launch's problems
    swh::DevBuf gscores;
    std::vector<swh::DevBuf *> all() {
        return {&qraw, &traw, &qc, &tc, &qr, &tr, &border, &flags, &misc, &strip_best, &mat, &lut,
                &probs, &strip_prob, &prob_best, &sync,
                &qoff, &db_work, &db_border, &db_redo, &db_scatter, &db_scores, &db_topk,
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
// Make sure buf holds at least bytes; on failure sets the error and returns SWH_E_NOMEM.
swh_status ensure(swh_ctx *ctx, DevBuf &buf, size_t bytes, const char *what);
swh_status make_scoring(swh_ctx *ctx, const swh_scoring *in, Scoring &out);

// Pairwise alignment on device-resident ASCII inputs (engine.cpp).
swh_status align_device(swh_ctx *ctx, const char *q_dev, int64_t qlen, const char *t_dev, int64_t tlen,
                        const Scoring &sc, int mode, hipStream_t st, swh_alignment *out, char *cigar,
                        int64_t cigar_cap, int64_t *cigar_len, swh_stats *stats);

}  // namespace swh
