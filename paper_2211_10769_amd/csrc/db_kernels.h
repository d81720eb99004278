// db_kernels.h -- descriptors of the database-search kernels (db_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swh {

// 128 database sequences (64 lanes x 2 packed halves), sorted by length and
// stored column-major: residue j of slot s at res[offset + j*128 + s].
struct DbGroup {
    int64_t offset;
    int32_t maxlen;
    int32_t first;     // first sorted position of the group
};

// One unit of inter-task work: query q against group g.
struct DbWork {
    int32_t q;
    int32_t g;
};

struct DbSearchArgs {
    const uint8_t *res;        // group-major interleaved residues (pad code beyond a length)
    const DbGroup *groups;
    const int32_t *perm;       // sorted position -> database index (-1 for empty slots)
    const uint8_t *qcodes;     // all queries, concatenated codes
    const int64_t *qoff;       // nq + 1 offsets
    const DbWork *work;        // in order of decreasing cost
    int32_t nwork;
    int32_t asize;             // pad code = asize
    const int8_t *mat;
    int32_t o, e;
    int64_t ndb;
    int32_t *scores;           // nq x ndb; saturated pairs get -1
    int32_t *redo;             // (q, db index) pairs that saturated
    int32_t *nredo;
    int32_t redo_cap;
    int32_t *ticket;
    uint32_t *border;          // one wave per unit: per persistent wave, max_len * 64 lanes * 2 words;
                               // pipelined: per work-group, wrap_cap * 64 lanes * 4 words
    int32_t max_len;           // longest group handled here
    int32_t wrap_cap;          // pipelined: columns of the global ring (>= max_len + 64)
    const int32_t *cancel;     // pinned host flag: nonzero = take no further unit (NULL: none)
    int32_t *abort_flag;       // pipelined: set when a bounded wait expires
    uint64_t wait_ticks;       // wall-clock ticks one wait may last
};

hipError_t launch_db_pack(const uint8_t *codes, const int64_t *offs, const int32_t *perm, const DbGroup *groups,
                          int32_t ngroups, uint8_t pad, uint8_t *res, hipStream_t st);
// waves = 1: one wave per (query, group) unit; 2, 4, 8 or 16: the pipelined form,
// a work-group of that many waves shares each unit, its 32-row chunks on
// neighbouring waves.  grid = work-groups (persistent).
hipError_t launch_db_search(const DbSearchArgs &a, int waves, int grid, hipStream_t st);
int db_search_grid_limit(int device, int waves);
// Top-k per row of an nq x ndb score matrix: score desc, index asc; -1 padding.
hipError_t launch_topk(const int32_t *scores, int32_t nq, int64_t ndb, int32_t k, int32_t *cand_idx,
                       int32_t *cand_score, int64_t *out_idx, int32_t *out_score, hipStream_t st);
size_t topk_scratch_entries(int32_t nq, int64_t ndb, int32_t k);
// dst[i] = v for i < n (a kernel, so that it may sit inside a captured graph)
hipError_t launch_fill_i32(int32_t *dst, int64_t n, int32_t v, hipStream_t st);
// dst[pos[i]] = best[i * stride] (the scores of a strip launch's BestCell results, stride in int32)
hipError_t launch_scatter_best(const int64_t *pos, const int32_t *best, int64_t n, int32_t stride, int32_t *dst,
                               hipStream_t st);
// dst[pos[i]] = val[i]
hipError_t launch_scatter(const int64_t *pos, const int32_t *val, int64_t n, int32_t *dst, hipStream_t st);

}  // namespace swh
