/*
 * swh.h -- C ABI of the MI355X Smith-Waterman engine (libswh.so).
 *
 * The library computes optimal local alignments with affine gaps
 * (Smith-Waterman with Gotoh's three-state recurrences), the method whose
 * "resolution" phase (find the maximum score) and "reconstruction" phase
 * (find the optimal path with space-efficient methods) the paper describes in
 * its Background section, "SW# suite".  Scoring follows the same paragraph:
 * a substitution matrix plus gap open / gap extension penalties.
 *
 * Conventions shared by every entry point
 *  - Sequences are ASCII; a symbol is looked up case-insensitively in the
 *    scoring alphabet.  Any other byte fails with SWH_E_ALPHABET and the last
 *    error names the sequence and the position.
 *  - A gap of length k costs gap_open + (k-1) * gap_extend.
 *  - Coordinates are 0-based and inclusive.  The query indexes rows, the
 *    target columns.
 *  - The end of an alignment is the first cell in row-major order (smallest
 *    query position, then smallest target position) that holds the optimal
 *    score; the start is the largest start (query first, then target) of an
 *    optimal alignment with that end.  A score of 0 means "no alignment":
 *    all coordinates are -1 and the CIGAR is empty.
 *  - CIGAR: run-length M (aligned pair), I (query residue against a gap),
 *    D (target residue against a gap).  Among co-optimal paths the one
 *    returned is the greedy backward walk of the global DP over the aligned
 *    rectangle that prefers, at an H cell, the diagonal, then I, then D, and
 *    inside a gap prefers closing it over extending it.
 *  - The caller owns every buffer.  Nothing keeps a caller pointer after the
 *    call returns.  Host-pointer calls are synchronous.
 *  - Every call returns a status; on failure swh_last_error() describes it.
 *    No entry point aborts, exits or throws: a failed host allocation inside
 *    the library returns SWH_E_NOMEM, any other internal exception
 *    SWH_E_DEVICE.
 *  - A context belongs to one host thread at a time.
 */
#ifndef SWH_H
#define SWH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SWH_OK = 0,
    SWH_E_INVAL = -1,      /* bad argument (null pointer, bad size, bad scoring) */
    SWH_E_ALPHABET = -2,   /* a sequence byte is not in the alphabet */
    SWH_E_NOMEM = -3,      /* device or host allocation failed */
    SWH_E_RANGE = -4,      /* output buffer too small, or input beyond a documented limit */
    SWH_E_DEVICE = -5,     /* HIP runtime error */
    SWH_E_TIMEOUT = -6,    /* a kernel's bounded wait expired (internal error) */
    SWH_E_CANCELLED = -7
} swh_status;

typedef struct swh_ctx swh_ctx;

/* Scoring scheme.  matrix is alphabet_size x alphabet_size int8, row-major,
 * matrix[q * alphabet_size + t] = s(query symbol q, target symbol t).
 * Limits: 1 <= alphabet_size <= 32, 0 < gap_extend <= gap_open <= 65535. */
typedef struct {
    const char   *alphabet;
    int32_t       alphabet_size;
    const int8_t *matrix;
    int32_t       gap_open;
    int32_t       gap_extend;
} swh_scoring;

typedef struct {
    int32_t  score;
    uint32_t flags;            /* SWH_F_* */
    int64_t  q_begin, q_end;   /* -1 when score == 0 */
    int64_t  t_begin, t_end;
} swh_alignment;

#define SWH_F_NONE 0u

enum { SWH_MODE_SCORE = 0,   /* score and end coordinates (forward pass only) */
       SWH_MODE_COORDS = 1,  /* + start coordinates (reverse pass) */
       SWH_MODE_CIGAR = 2 }; /* + CIGAR (linear-space traceback) */

/*
 * OR'd into mode (swh_align, swh_align_dev, swh_align_batch): the optimal
 * GLOBAL alignment of the whole query against the whole target instead of
 * the local one -- Needleman-Wunsch with the same affine gaps (paper,
 * Background, "Needleman-Wunsch algorithm"; SW# offers it beside SW).  score
 * = G(n, m) of the global DP (may be negative); the coordinates are always
 * 0 .. n-1 and 0 .. m-1 (-1 for an empty sequence); the CIGAR is the greedy
 * backward walk of the global DP from (n, m) to (0, 0) with the preferences
 * of the local CIGAR (at H: diagonal, then I, then D; in a gap: close it), so
 * it may begin or end with I or D runs.  An empty sequence against one of
 * length k scores -(gap_open + (k-1) gap_extend).  Extra limit:
 * (qlen + tlen) * (max(gap_extend, |min s|) + max s) + 2 gap_open < 2^27.
 */
#define SWH_GLOBAL 0x100

/*
 * OR'd into mode (swh_align, swh_align_dev, swh_align_batch): the optimal
 * SEMI-GLOBAL alignment -- the whole query against a part of the target, the
 * target residues before and after that part unpenalised, gaps at the ends
 * of the query penalised (paper, Background, "Semi-global algorithm (HW)").
 * score = max_j G(n, j) of the DP with G(0, j) = 0, G(i, 0) = -(o + (i-1) e);
 * t_end = the smallest such j (minus one); t_begin = the largest start of an
 * optimal alignment ending there (found by the same DP on the reversed
 * sequences); q_begin = 0, q_end = n-1; the CIGAR is the greedy walk of the
 * global DP over query x target[t_begin .. t_end].  No target residue
 * aligned: t_begin = t_end = -1, CIGAR "nI"; an empty query: score 0, all
 * coordinates -1.  Limits as for SWH_GLOBAL.
 */
#define SWH_SEMIGLOBAL 0x200

/*
 * OR'd into mode (swh_align, swh_align_dev, swh_align_batch): the optimal
 * OVERLAP alignment -- gaps before the first and after the last aligned
 * residue of either sequence cost nothing (paper, Background, "Overlap
 * algorithm (OV)").  DP with G(0, j) = G(i, 0) = 0; score = the maximum over
 * the last row G(n, j) and the last column G(i, m); the end is the first of
 * those cells in row-major order holding it (the last column above row n,
 * then the last row from the left); the start is the largest one, on the top
 * row or the left column, of an alignment of that score ending there; the
 * CIGAR is the greedy walk of the global DP between the two.  Score 0 (only
 * the empty overlap) reports no alignment: coordinates -1, empty CIGAR.
 * Costs two score passes (the last column comes from the same DP with the
 * sequences swapped) and two more for the start.  Limits as for SWH_GLOBAL;
 * exactly one of SWH_GLOBAL, SWH_SEMIGLOBAL, SWH_OVERLAP may be set.
 */
#define SWH_OVERLAP 0x400

/* Per-call statistics; set struct_size = sizeof(swh_stats) before the call. */
typedef struct {
    uint32_t struct_size;
    uint32_t reserved;
    double   cells_forward;     /* n * m of the forward pass */
    double   ms_forward;        /* device time of the forward pass */
    double   ms_reverse;        /* device time of the reverse pass */
    double   ms_traceback;      /* wall time of the traceback */
    double   cells_traceback;   /* DP cells evaluated by the traceback */
    int64_t  traceback_bands;   /* bands the traceback was cut into at rows kept by the
                                   score passes (0: one divide and conquer over the rectangle) */
    int64_t  traceback_retries; /* band traceback abandoned for the plain one (expected 0) */
    int64_t  passes_int16;      /* local score passes run in packed 16-bit arithmetic */
    int64_t  saturated_int16;   /* of those, passes whose maximum reached 32767 - max s and that were
                                   recomputed in 32 bits (every reported value is exact) */
} swh_stats;

/* Context on HIP device `device` (ordinal).  Allocates nothing large; device
 * buffers grow on demand and are kept until swh_destroy. */
swh_status  swh_create(int device, swh_ctx **out);
void        swh_destroy(swh_ctx *ctx);
/* Text of the last failure on ctx; valid until the next call on ctx. */
const char *swh_last_error(const swh_ctx *ctx);

/*
 * Cancellation (the paper's migration notes single out error handling as the
 * part of the port that needed most attention, Migration process; a caller
 * that can stop a long call is part of that contract).  swh_cancel may be
 * called from any host thread while another thread runs a call on ctx: the
 * running call stops at its next unit of work (a strip of rows, a
 * (query, database group) unit, a traceback level, a training step) and
 * returns SWH_E_CANCELLED; its outputs are then undefined.  Kernels see the
 * request through a flag in pinned host memory and drain normally.  Every
 * entry point clears the flag when it starts, so a request made while no
 * call runs is dropped.  The context stays usable after a cancelled call.
 */
swh_status  swh_cancel(swh_ctx *ctx);

/*
 * Context options.  Every option changes speed, memory or diagnostics only,
 * never a result.  Values:
 *   SWH_OPT_ROWS_PER_LANE  strip height of every pass: 4, 8, 16, 20, 24 or 32
 *                          rows per lane; 0 (default) = the tuned table or the
 *                          built-in rule
 *   SWH_OPT_GRID           > 0: run the strip kernel as this many single-wave
 *                          workgroups instead of the balanced placement, and the
 *                          database kernel with at most this many persistent
 *                          work-groups; 0 default
 *   SWH_OPT_BAND_ROWS      rows between the rows the score passes keep for the
 *                          band traceback: 0 (default) = built-in, -1 = no band
 *                          traceback, > 0 = that many (rounded up to strips)
 *   SWH_OPT_TB_LEAF        largest leaf of the linear-space traceback, in DP
 *                          cells (1 .. 524288); 0 (default) = the largest
 *   SWH_OPT_GRAPH          1 (default): the prefilter's training step runs as
 *                          the replay of a captured HIP graph; 2: repeated
 *                          database searches as well (swh_db_search with the
 *                          same database, k and query lengths: one replay per
 *                          search, no host work between its launches; a replay
 *                          runs the single-pair branch after the inter-task
 *                          kernel rather than beside it, so searches that have
 *                          such problems are faster as plain launches); 0: plain
 *                          launches everywhere
 *   SWH_OPT_PRUNE          1 (default): block pruning of reverse passes; 0: off
 *   SWH_OPT_MEM_CAP        bytes of device memory the context's own working
 *                          buffers may hold (database and model handles are
 *                          not counted); 0 (default) = no cap.  A call that
 *                          would need more fails with SWH_E_NOMEM; optional
 *                          buffers (rows kept for the band traceback) shrink
 *                          to fit instead.
 *   SWH_OPT_INT16          local score passes in packed 16-bit arithmetic
 *                          (two cells per lane operation), exact: a pass whose
 *                          maximum reaches 32767 - max s is recomputed in 32
 *                          bits.  1 (default): batches, and single passes large
 *                          enough to fill the GPU; 2: also every single pass
 *                          that cannot reach the limit; 0: 32-bit only
 *   SWH_OPT_INTER_MAX      database sequences up to this length go to the
 *                          inter-task kernel, longer ones to the single-pair
 *                          kernel (applies to databases created afterwards);
 *                          0 (default) = the built-in or autotuned threshold
 *   SWH_OPT_PF_RANK        how swh_prefilter_search ranks the database for a
 *                          query: 1 (default) by the predicted score's excess
 *                          over the mean prediction of database sequences of
 *                          similar length (the length-sorted groups of 128 the
 *                          database is stored in), so that long sequences do not
 *                          take the rescoring budget by length alone; 2 by that
 *                          excess divided by the group's deviation (fewer
 *                          rescored cells, but noise in groups of near-equal
 *                          predictions is amplified); 0 by the predicted score
 *                          itself.  Reported scores are exact either way.
 *   SWH_OPT_DB_WAVES       waves that share one (query, group) unit of the
 *                          database kernel: 1 (one wave per unit), 2, 4, 8, 12 or 16 (the
 *                          unit's 32-row query chunks run on neighbouring waves
 *                          and hand their bottom rows on through LDS, so that a
 *                          few queries still fill the GPU); 0 (default): chosen
 *                          from the number of units
 *   SWH_OPT_DB_ROUTE       a (query, group) unit whose cells exceed this percentage
 *                          of one compute unit's share of the search runs on the
 *                          single-pair kernel instead (one work-group would
 *                          otherwise finish long after the rest: a unit cannot
 *                          leave its compute unit, a single-pair problem can);
 *                          0 (default) = 100, -1 = never
 *   SWH_OPT_FAULT_NOMEM    1: the next entry point on ctx fails as if a host
 *                          allocation had thrown std::bad_alloc (after its
 *                          argument checks), then the option resets; a test
 *                          of the error path
 * swh_set_option: SWH_E_INVAL for an unknown option or a value out of range.
 */
enum {
    SWH_OPT_ROWS_PER_LANE = 1,
    SWH_OPT_GRID = 2,
    SWH_OPT_BAND_ROWS = 3,
    SWH_OPT_TB_LEAF = 4,
    SWH_OPT_GRAPH = 5,
    SWH_OPT_PRUNE = 6,
    SWH_OPT_MEM_CAP = 7,
    SWH_OPT_INT16 = 8,
    SWH_OPT_INTER_MAX = 9,
    SWH_OPT_FAULT_NOMEM = 10,
    SWH_OPT_PF_RANK = 11,
    SWH_OPT_DB_WAVES = 12,
    SWH_OPT_DB_ROUTE = 13
};
swh_status  swh_set_option(swh_ctx *ctx, int32_t option, int64_t value);
swh_status  swh_get_option(const swh_ctx *ctx, int32_t option, int64_t *value);

/*
 * One local alignment of query q (qlen bytes) against target t (tlen bytes),
 * host pointers.  Resolution: forward score pass (score, end).  mode >=
 * COORDS adds the reverse pass over the reversed prefixes ending at the end
 * cell, which gives the start.  mode == CIGAR adds the reconstruction.
 *
 * cigar: caller buffer of cigar_cap bytes, NUL-terminated on success; may be
 * NULL when mode < CIGAR.  *cigar_len (may be NULL) receives the CIGAR
 * length without the NUL; when cigar_cap is too small the call fails with
 * SWH_E_RANGE and *cigar_len holds the required length.
 * Limits: qlen, tlen < 2^31; min(qlen, tlen) * max|s| < 2^26;
 * for mode CIGAR also (max s + gap_extend) * (qlen + tlen) + gap_open < 2^27.
 * stats may be NULL.
 */
swh_status swh_align(swh_ctx *ctx, const char *q, int64_t qlen, const char *t, int64_t tlen,
                     const swh_scoring *scoring, int mode, swh_alignment *out,
                     char *cigar, int64_t cigar_cap, int64_t *cigar_len, swh_stats *stats);

/*
 * Same as swh_align with q and t in device memory (for example torch tensor
 * data pointers).  stream is a hipStream_t (NULL = the default stream); the
 * call orders its work after prior work on that stream and returns when the
 * result is on the host.  Inputs must stay valid until the call returns.
 */
swh_status swh_align_dev(swh_ctx *ctx, const char *q_dev, int64_t qlen, const char *t_dev,
                         int64_t tlen, const swh_scoring *scoring, int mode, void *stream,
                         swh_alignment *out, char *cigar, int64_t cigar_cap,
                         int64_t *cigar_len, swh_stats *stats);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the score
 * pass, and with SWH_MODE_COORDS the start pass, of swh_align_dev, with no
 * allocation of any kind -- no hipMalloc or hipFree, no host heap, no
 * context.  Every buffer the passes need beyond the inputs and `out` comes
 * from one static device array of 64 MiB per GPU, held from the library's
 * load on that GPU until the process ends.  q_dev, t_dev: device pointers;
 * stream: a hipStream_t (NULL = default stream); the call orders its work
 * after prior work on it and returns when *out is on the host.  mode:
 * SWH_MODE_SCORE or SWH_MODE_COORDS only (no CIGAR, no global forms).
 * Results equal swh_align_dev's in the same mode.  Size limit: about
 * 2 qlen + 10 tlen bytes of the array (a 5 Mbp query against a 5.1 Mbp
 * target fits); beyond it SWH_E_RANGE.  Other errors: SWH_E_INVAL (bad
 * device, NULL pointers, bad scoring or mode), SWH_E_ALPHABET,
 * SWH_E_DEVICE, SWH_E_TIMEOUT; there is no context and so no error text.
 * Calls on one GPU share the array: the library serialises them with a host
 * mutex per device, so concurrent calls from several threads of a process
 * wait for each other (the array keeps the last call's contents; everything
 * that must start at zero is cleared on each call).
 */
swh_status swh_align_dev_noalloc(int device, const char *q_dev, int64_t qlen, const char *t_dev,
                                 int64_t tlen, const swh_scoring *scoring, int mode, void *stream,
                                 swh_alignment *out);

/*
 * Many independent local alignments in one call (paper, Background: SW# and
 * CUDASW++ both run many independent matrices; the library batches them).
 * Pair i is query q_cat[q_off[i] .. q_off[i+1]) against target
 * t_cat[t_off[i] .. t_off[i+1]) (host pointers, offsets non-decreasing; the
 * first offset need not be 0).  Every pair gets exactly the result swh_align
 * gives it; all pairs share the launches of each phase (forward pass,
 * reverse pass, traceback levels), most expensive pairs first.
 *
 * out: npairs results (caller-owned).  mode CIGAR: cigar_off (npairs + 1
 * entries, caller-owned) receives offsets into cigar_cat, CIGAR i being the
 * bytes cigar_cat[cigar_off[i] .. cigar_off[i+1]) without terminator; when
 * cigar_cat is NULL or cigar_off[npairs] > cigar_cap the call returns
 * SWH_E_RANGE with out and cigar_off filled (cigar_off[npairs] = bytes
 * needed).  cigar arguments are ignored in the other modes.  Each pair must
 * satisfy the limits of swh_align.  Errors: SWH_E_INVAL (NULL pointers,
 * decreasing offsets, bad mode), SWH_E_ALPHABET (names the pair and the
 * byte), SWH_E_RANGE, SWH_E_NOMEM, SWH_E_DEVICE, SWH_E_TIMEOUT.  stats
 * (optional) sums the phases over all pairs.
 */
swh_status swh_align_batch(swh_ctx *ctx, int64_t npairs, const char *q_cat, const int64_t *q_off,
                           const char *t_cat, const int64_t *t_off, const swh_scoring *scoring,
                           int mode, swh_alignment *out, char *cigar_cat, int64_t cigar_cap,
                           int64_t *cigar_off, swh_stats *stats);

/*
 * Same as swh_align_batch with the concatenated sequences q_cat and t_cat in
 * device memory (for example torch tensor data pointers); the offsets and
 * every output stay in host memory.  stream is a hipStream_t (NULL = the
 * default stream): the call's work is ordered after prior work on that
 * stream, runs on the context's own stream, and the call returns when the
 * results are on the host.  Inputs must stay valid until the call returns.
 */
swh_status swh_align_batch_dev(swh_ctx *ctx, int64_t npairs, const char *q_cat_dev, const int64_t *q_off,
                               const char *t_cat_dev, const int64_t *t_off, const swh_scoring *scoring,
                               int mode, void *stream, swh_alignment *out, char *cigar_cat,
                               int64_t cigar_cap, int64_t *cigar_off, swh_stats *stats);

/*
 * Strip shape of the intra-task kernel, per bucket of query rows: problems
 * with n <= max_rows rows (first matching entry) use strips of
 * 64 * rows_per_lane rows and a persistent grid of waves_per_simd waves per
 * SIMD (0: the built-in choice for that height).  Shapes change speed only,
 * never results.
 */
typedef struct {
    int64_t max_rows;
    int32_t rows_per_lane;      /* 4, 8, 16, 20, 24 or 32 */
    int32_t waves_per_simd;     /* 0..8 */
} swh_tune_entry;

/* Measure every shape on synthetic problems for row buckets 1 Ki, 4 Ki, ...
 * up to max_rows (about cells_per_trial DP cells per timed launch, scored
 * with the given scoring) and install the fastest per bucket in ctx. */
swh_status swh_autotune(swh_ctx *ctx, const swh_scoring *scoring, int64_t max_rows,
                        double cells_per_trial);
/* Copy ctx's table (at most cap entries) to out; *count = its length
 * (0: built-in rule).  A caller may store it and install it with
 * swh_tune_set in a later context. */
swh_status swh_tune_get(const swh_ctx *ctx, swh_tune_entry *out, int32_t cap, int32_t *count);
/* Install a table (count = 0 restores the built-in rule).  SWH_E_INVAL for
 * an entry with an unsupported shape or max_rows not increasing. */
swh_status swh_tune_set(swh_ctx *ctx, const swh_tune_entry *entries, int32_t count);

/*
 * Measure the database length switch (paper, Background: SW# picks
 * inter-task parallelism for short and intra-task parallelism for long
 * sequences): for lengths 512 .. 8192, time a search of synthetic sequences
 * of that length range (scored with `scoring`) on the inter-task kernel and
 * on the single-pair kernel, and keep the largest length at which the
 * inter-task kernel is still the faster.  The value goes into ctx (used by
 * databases created afterwards while SWH_OPT_INTER_MAX is 0) and *inter_max
 * (may be NULL).  Results never depend on it.
 */
swh_status swh_autotune_db(swh_ctx *ctx, const swh_scoring *scoring, int32_t *inter_max);

/*
 * The context's tuning -- strip-shape table and database length switch -- as
 * a small text file tagged with the device's name, so that a later process
 * can skip the measurements.  swh_tune_load fails with SWH_E_INVAL when the
 * file was written on a device of another name or is not such a file.
 */
swh_status swh_tune_save(const swh_ctx *ctx, const char *path);
swh_status swh_tune_load(swh_ctx *ctx, const char *path);

/* ------------------------------------------------------------------------
 * Database search (paper, Background: database similarity search, many
 * independent matrices; Experimental Work: 20 protein queries against
 * Swiss-Prot / Env. NR with BLOSUM62, gap open 10, extend 2).
 * ------------------------------------------------------------------------ */

typedef struct swh_db swh_db;   /* encoded, length-sorted database in device memory */

typedef struct {
    int64_t db_index;   /* -1 when fewer than k sequences exist */
    int32_t score;      /* -1 for an empty slot */
    int32_t reserved;
} swh_hit;

typedef struct {
    uint32_t struct_size;        /* sizeof(swh_search_stats) */
    uint32_t reserved;
    double   cells;              /* sum over queries of query length x database residues */
    double   ms_inter;           /* device time of the 16-bit inter-task kernel */
    double   ms_intra;           /* device time of the 32-bit single-pair kernel (long / saturated) */
    double   ms_topk;            /* device time of the top-k selection */
    int64_t  saturated;          /* pairs recomputed in 32 bits after a 16-bit saturation */
    int64_t  intra_pairs;        /* pairs scored by the single-pair kernel */
    int32_t  graph;              /* 1: the search ran as the replay of a captured HIP graph (ms_inter then
                                    times the whole graph; ms_intra and ms_topk are 0) */
    int32_t  reserved2;
} swh_search_stats;

/*
 * Encode and lay out a database of ndb sequences (ASCII, concatenated in
 * db_cat, sequence i = db_cat[db_off[i] .. db_off[i+1]), db_off has ndb+1
 * non-decreasing entries).  The scoring is fixed for the handle.  The handle
 * owns its device memory until swh_db_destroy.  Sequences longer than 2,048
 * residues are scored by the single-pair kernel at search time.
 */
swh_status swh_db_create(swh_ctx *ctx, int64_t ndb, const char *db_cat, const int64_t *db_off,
                         const swh_scoring *scoring, swh_db **out);
void       swh_db_destroy(swh_db *db);

/*
 * Exhaustive local-alignment scores of nq queries (q_cat / q_off as for the
 * database) against every database sequence, then the k best hits per query
 * (score descending, database index ascending), hits[q * k + r].  Scores
 * are exact 32-bit optima: pairs whose packed 16-bit values may have
 * saturated are recomputed.  1 <= k <= 32.  stats may be NULL.
 * With SWH_OPT_GRAPH on (the default) the whole launch sequence of a search
 * is captured once as a HIP graph per (database, k, query lengths) and
 * replayed by later searches with the same lengths (new query contents); a
 * replay that meets a 16-bit saturation, an empty query, or any change of the
 * context's buffers runs the search eagerly instead.  Results are identical.
 */
swh_status swh_db_search(swh_ctx *ctx, const swh_db *db, int32_t nq, const char *q_cat,
                         const int64_t *q_off, int32_t k, swh_hit *hits, swh_search_stats *stats);

/*
 * Same as swh_db_search with the concatenated queries q_cat_dev in device
 * memory (q_off, hits and stats in host memory); ordered after prior work on
 * stream (a hipStream_t, NULL = the default stream), returns when the hits
 * are on the host.
 */
swh_status swh_db_search_dev(swh_ctx *ctx, const swh_db *db, int32_t nq, const char *q_cat_dev,
                             const int64_t *q_off, int32_t k, void *stream, swh_hit *hits,
                             swh_search_stats *stats);

/* All scores, scores[q * ndb + i] (host buffer of nq * ndb int32). */
swh_status swh_db_scores(swh_ctx *ctx, const swh_db *db, int32_t nq, const char *q_cat,
                         const int64_t *q_off, int32_t *scores, swh_search_stats *stats);

/* ------------------------------------------------------------------------
 * Learned prefilter for the database search.  The paper runs the search
 * exhaustively (Background: database similarity search); this growth ranks
 * the database for each query with a small network that predicts the
 * Smith-Waterman score, rescores the best-ranked fraction exactly with the
 * search kernels above, and keeps the exhaustive search as its fallback, so
 * every reported score is an exact one.
 *
 * Features of a (query, database sequence) pair: the 400 products
 * f_q[k] f_t[k] of their dipeptide frequencies (over the first 20 alphabet
 * symbols, the standard residues; f = counts / (L - 1)) and ln(min(L_q, L_t)),
 * normalised with the training set's mean and standard deviation.  Network:
 * 401 -> 256 (ReLU) -> 256 (ReLU) -> 1, predicting ln(1 + S); bfloat16
 * products with float32 accumulation on the GPU, float32 master weights.
 * Parameters are one float array of SWH_MODEL_PARAMS entries: W1 [256][401],
 * b1 [256], W2 [256][256], b2 [256], w3 [256], b3.
 * ------------------------------------------------------------------------ */

#define SWH_MODEL_PARAMS 168961
#define SWH_MODEL_INPUTS 401

typedef struct swh_model swh_model;   /* weights (device), normalisation, Adam state */

typedef struct {
    uint32_t struct_size;
    uint32_t reserved;
    int32_t  epochs;       /* passes over the pairs (>= 1) */
    int32_t  batch;        /* pairs per Adam step, a multiple of 64 (the last partial batch of an epoch is dropped) */
    double   lr;           /* Adam step size (betas 0.9, 0.999, eps 1e-8) */
    uint64_t seed;         /* batch order */
} swh_train_cfg;

typedef struct {
    uint32_t struct_size;
    uint32_t reserved;
    double   first_epoch_loss;   /* mean squared error over the first epoch */
    double   final_epoch_loss;
    double   ms_label, ms_features, ms_train;
    double   cells_label;        /* DP cells of the engine's labelling pass */
    int64_t  steps;
    int32_t  graph;              /* 1: each step ran as a replay of one captured HIP graph */
    int32_t  reserved2;
} swh_train_stats;

typedef struct {
    uint32_t struct_size;
    uint32_t reserved;
    int64_t  candidates;         /* pairs kept by the ranking, all queries */
    int64_t  audited;            /* pairs rescored as audit sample */
    int64_t  fallbacks;          /* queries that fell back to the exhaustive search */
    double   cells_rescored;     /* DP cells of the exact rescoring (candidates + audit) */
    double   cells_exhaustive;   /* DP cells an exhaustive search would take */
    double   ms_features, ms_predict, ms_select, ms_rescore, ms_topk, ms_fallback;
} swh_prefilter_stats;

/* A model for `scoring` (alphabet of >= 20 symbols).  theta (SWH_MODEL_PARAMS
 * floats), mu and sd (SWH_MODEL_INPUTS floats each) may be NULL: He-normal
 * weights drawn from seed, zero biases, mu = 0, sd = 1.  Host pointers,
 * copied. */
swh_status swh_model_create(swh_ctx *ctx, const swh_scoring *scoring, const float *theta, const float *mu,
                            const float *sd, uint64_t seed, swh_model **out);
void       swh_model_destroy(swh_model *model);
/* Copy out (NULL entries skipped) / replace (NULL: keep) the parameters and the
 * normalisation; replacing resets the Adam state. */
swh_status swh_model_get(swh_ctx *ctx, const swh_model *model, float *theta, float *mu, float *sd);
swh_status swh_model_set(swh_ctx *ctx, swh_model *model, const float *theta, const float *mu, const float *sd);
/* Binary model file: magic "SWHMLP01", alphabet size, parameter count,
 * parameters, mu, sd (little-endian float32).  SWH_E_INVAL on I/O errors or a
 * file of another kind. */
swh_status swh_model_save(swh_ctx *ctx, const swh_model *model, const char *path);
swh_status swh_model_load(swh_ctx *ctx, const char *path, swh_model **out);

/*
 * Train `model` on labelled pairs.  Sequences: a pool seq_cat[seq_off[i] ..
 * seq_off[i+1]) of nseq entries; pair p is (pool[pair_row[p]],
 * pool[pair_col[p]]).  Labels: scores (npairs exact local scores) or, when
 * NULL, the engine's own score pass over every pair (the scoring of
 * `scoring`); labels_out (optional, npairs) receives the labels used.  The
 * feature normalisation is recomputed from these pairs, then cfg->epochs
 * passes of Adam over shuffled batches run on the GPU.  Errors:
 * SWH_E_INVAL (bad indices, cfg, alphabet), SWH_E_ALPHABET, SWH_E_RANGE,
 * SWH_E_NOMEM, SWH_E_DEVICE.
 */
swh_status swh_prefilter_train(swh_ctx *ctx, swh_model *model, const swh_scoring *scoring, int64_t nseq,
                               const char *seq_cat, const int64_t *seq_off, int64_t npairs,
                               const int32_t *pair_row, const int32_t *pair_col, const int32_t *scores,
                               const swh_train_cfg *cfg, int32_t *labels_out, swh_train_stats *stats);

/*
 * Top-k search through the prefilter: per query, the database sequences whose
 * prediction is at or above the ceil(rescore_frac * ndb)-th largest (ties
 * kept, at least k) are rescored exactly, plus an audit sample of the rest
 * (pair (q, i) is audited when the high 32 bits of splitmix64(audit_seed +
 * 0x9E3779B97F4A7C15 (q 2^32 + i + 1)) are below audit_frac 2^32).  A query
 * whose top-k would contain an audited pair, or that has fewer than k
 * candidates, is searched exhaustively instead.  hits as swh_db_search.
 * 0 < rescore_frac <= 1, 0 <= audit_frac <= 1, 1 <= k <= 32; the database
 * and the model must use alphabets of the same size.
 */
swh_status swh_prefilter_search(swh_ctx *ctx, const swh_model *model, swh_db *db, int32_t nq,
                                const char *q_cat, const int64_t *q_off, int32_t k, double rescore_frac,
                                double audit_frac, uint64_t audit_seed, swh_hit *hits,
                                swh_prefilter_stats *stats);

/* Predicted ln(1 + S) for every (query, database sequence): pred[q * ndb + i]. */
swh_status swh_prefilter_predict(swh_ctx *ctx, const swh_model *model, swh_db *db, int32_t nq,
                                 const char *q_cat, const int64_t *q_off, float *pred);

/* Dipeptide counts of nseq sequences: counts[i * 400 + 20 a + b] (first 20
 * alphabet symbols; pairs with any other symbol are not counted). */
swh_status swh_dipeptide_counts(swh_ctx *ctx, const swh_scoring *scoring, int64_t nseq, const char *seq_cat,
                                const int64_t *seq_off, int32_t *counts);

/* One forward and backward pass of the model on B normalised inputs
 * z [B][SWH_MODEL_INPUTS] with targets y [B]: *loss = mean squared error,
 * grad = its gradient (SWH_MODEL_PARAMS floats).  B a multiple of 64. */
swh_status swh_mlp_grad(swh_ctx *ctx, swh_model *model, int32_t B, const float *z, const float *y,
                        double *loss, float *grad);
/* `steps` Adam steps of size lr on one fixed batch (as swh_mlp_grad). */
swh_status swh_mlp_train_steps(swh_ctx *ctx, swh_model *model, int32_t B, const float *z, const float *y,
                               int32_t steps, double lr);

#ifdef __cplusplus
}
#endif

#endif /* SWH_H */
