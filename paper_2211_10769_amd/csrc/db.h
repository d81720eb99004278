// db.h -- the opaque database handle and the search entry points.
#pragma once

#include <stdint.h>

#include <utility>
#include <vector>

#include "context.h"
#include "db_kernels.h"

struct swh_db {
    int device = 0;
    swh::Scoring sc;
    int64_t ndb = 0;
    int64_t total_residues = 0;
    int32_t inter_max = 0;                 // longest sequence of the inter-task kernel
    uint64_t serial = 0;                   // unique per handle (keys captured search graphs)
    std::vector<int64_t> h_off;            // per database index, rebased to 0
    std::vector<swh::DbGroup> h_groups;
    std::vector<int32_t> h_perm;           // sorted position -> database index, -1 padding
    std::vector<int32_t> long_idx;         // sequences handled by the single-pair kernel
    swh::DevBuf codes, offs, res, groups, perm;
    // prefilter feature rows (built on first use): inter-task slots, then long sequences
    bool pf_ready = false;
    int64_t pf_nrows = 0, pf_nslots = 0;
    std::vector<int32_t> h_row_db, h_row_len;
    swh::DevBuf pf_F, pf_row_len, pf_row_db;
};

namespace swh {

struct DbStats {
    double cells = 0.0;
    double ms_inter = 0.0, ms_intra = 0.0, ms_topk = 0.0;
    int64_t redo = 0;
    int64_t intra_pairs = 0;
    bool graph = false;   // the search ran as a graph replay (ms_inter then times the whole graph)
};

// dst[i] = src[i] for i < count, pad code up to padded
struct GatherLite {
    const uint8_t *src;
    uint8_t *dst;
    int64_t count;
    int64_t padded;
};
swh_status gather_lite(swh_ctx *ctx, const std::vector<GatherLite> &g, uint8_t pad, hipStream_t st);

// Encoded queries in ctx->qc with host offsets (rebased to 0) in qo and
// device offsets in ctx->qoff; the matrix in ctx->mat.
struct QuerySet {
    int32_t nq = 0;
    std::vector<int64_t> qo;
    int64_t maxq = 1;
};
// dev: q_cat is a device pointer (encoded in place), else a host pointer.
swh_status prepare_queries(swh_ctx *ctx, const Scoring &sc, int32_t nq, const char *q_cat, const int64_t *q_off,
                           QuerySet &qs, bool dev = false);

// A set of interleaved 128-sequence groups (device) with the host copy of the
// group table.
struct GroupSet {
    const uint8_t *res;
    const DbGroup *groups;
    const int32_t *perm;
    const std::vector<DbGroup> *h_groups;
};
// Scores of the given (query, group) units and (query, database index) pairs
// into scores_dev[q * ndb + index]; 16-bit saturation is redone in 32 bits.
swh_status score_units(swh_ctx *ctx, const swh_db *db, const QuerySet &qs, const GroupSet &gs,
                       std::vector<DbWork> work, const std::vector<std::pair<int32_t, int32_t>> &long_pairs,
                       int32_t *scores_dev, DbStats &stats);

// The units of a search: (query, group) units for the inter-task kernel and
// (query, sequence) pairs for the single-pair kernel -- sequences beyond the
// length switch, and the members of a group whose unit alone would exceed
// SWH_OPT_DB_ROUTE percent of one compute unit's share of the inter-task
// cells.  Empty queries get neither; cells += their DP cells.
void plan_search(const swh_ctx *ctx, const swh_db *db, const std::vector<int64_t> &qo, int32_t nq,
                 std::vector<DbWork> &work, std::vector<std::pair<int32_t, int32_t>> &pairs, double &cells);

// Launch shape of the inter-task kernel for `units` units of groups up to
// max_len columns: waves per unit, persistent work-groups, border bytes.
struct DbLaunch {
    int waves = 1;
    int grid = 1;
    int32_t wrap_cap = 0;
    size_t border_bytes = 0;
};
DbLaunch db_launch_shape(const swh_ctx *ctx, size_t units, int32_t max_len, double mean_chunks);

swh_status db_create(swh_ctx *ctx, int64_t ndb, const char *cat, const int64_t *off, const Scoring &sc,
                     swh_db **out);
void db_destroy(swh_db *db);
swh_status db_scores_device(swh_ctx *ctx, const swh_db *db, int32_t nq, const char *q_cat, const int64_t *q_off,
                            int32_t *scores_dev, DbStats &stats, bool dev = false);
swh_status db_search(swh_ctx *ctx, const swh_db *db, int32_t nq, const char *q_cat, const int64_t *q_off, int32_t k,
                     swh_hit *hits, int32_t *scores_host, DbStats &stats, bool dev = false);

// The top-k search as the replay of a captured HIP graph (db_graph.cpp): the
// context keeps one plan, keyed by the database, k and the query lengths, and
// captures a new one when they (or any context buffer) change.  done = false
// when the search must run eagerly instead (capture unavailable, or a 16-bit
// saturation that needs the eager recomputation).
swh_status search_graph(swh_ctx *ctx, const swh_db *db, int32_t nq, const char *q_cat, const int64_t *q_off,
                        int32_t k, swh_hit *hits, DbStats &stats, bool &done);
void destroy_search_plan(swh_ctx *ctx);

}  // namespace swh
