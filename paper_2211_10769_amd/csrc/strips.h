// strips.h -- run the strip-wavefront kernel over a table of DP problems.
#pragma once

#include <stdint.h>

#include <vector>

#include "context.h"
#include "engine.h"

namespace swh {

// One problem as the caller sees it.  qc holds rows_padded(n, R) codes and tc
// cols_padded(m) codes (pad code beyond the real ones).  border holds
// cols_padded(m) entries: the caller fills the top row (zeros for a local
// pass) and finds the last row there afterwards.
struct StripProblem {
    const uint8_t *qc;
    int64_t n;
    const uint8_t *tc;
    int64_t m;
    Border *border;
    // optional: keep the last rows of every save_every-th strip (Problem)
    Border *save = nullptr;
    int64_t save_stride = 0;
    int32_t save_every = 0;
    int32_t save_phase = 0;
    int32_t free_left = 0;   // global mode: H = 0 left of column 0 (Problem)
    int32_t prune = 0;       // local mode: known maximum, enables block pruning (Problem)
    int32_t top_pass = 0;    // global mode: pass-through rows on top (Problem)
};

inline int64_t rows_padded(int64_t n, int R) { return ((n + 64 * R - 1) / (64 * R)) * 64 * R; }
inline int64_t cols_padded(int64_t m) { return 64 * (sweep_blocks(m) + 3); }

int pick_rows_per_lane(int64_t n, int simds);
// Wall-clock ticks a kernel's bounded wait may last before it gives up.
uint64_t wait_ticks(int device);
int strip_grid(int64_t nstrips, int R, int limit, int num_cu, int waves = 0, int forced = 0);

// One launch over all problems; local mode fills best (one entry per problem).
// waves: waves per SIMD of the persistent grid, 0 = the rule for R.  int16
// (local mode, R in 4, 8, 16): the packed 16-bit kernel with strips of 128 R
// rows made of two sub-strips of 64 R rows, so that rows kept every
// save_every strips of 64 R rows land where the 32-bit kernel's would (row
// codes must then be padded to rows_padded(n, 2 R)); a problem whose best
// score reaches sat16_limit(smax) may have saturated and must be redone in 32
// bits by the caller, at the same R.
swh_status run_strips(swh_ctx *ctx, const std::vector<StripProblem> &probs, const Scoring &sc, int R, bool local,
                      hipStream_t st, std::vector<BestCell> *best, float *ms, int waves = 0, bool int16 = false);

// run_strips in two steps, so that the launches can be captured in a graph:
// prepare_strips builds the problem tables on the host (device pointers
// resolved) and sizes the context's buffers and the grid; enqueue_strips
// copies the tables from tab_src / sp_src (the prepared tables, or a pinned
// copy of them), clears the counters with kernels and launches the strip
// kernel and, in local mode, the per-problem reduction into ctx->prob_best,
// with no host synchronisation (PreparedStrips: engine.h).
swh_status prepare_strips(swh_ctx *ctx, const std::vector<StripProblem> &probs, const Scoring &sc, int R, bool local,
                          int waves, bool int16, PreparedStrips &out);
hipError_t enqueue_strips(swh_ctx *ctx, const PreparedStrips &ps, const Scoring &sc, const Problem *tab_src,
                          const int32_t *sp_src, hipStream_t st, bool timed);

// Whether the context may run a 16-bit pass of nominal height R (4, 8 or 16).
bool int16_usable(const swh_ctx *ctx, const Scoring &sc, int R);
// No cell of an n x m local pass can reach sat16_limit (S <= min(n, m) max s).
inline bool never_saturates(int64_t n, int64_t m, const Scoring &sc)
{
    const int64_t smax = sc.smax > 0 ? sc.smax : 1;
    return (n < m ? n : m) * smax < sat16_limit(sc.smax);
}

}  // namespace swh
