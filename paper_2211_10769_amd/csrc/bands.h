// bands.h -- set-up of the band traceback, shared by the single-pair and the
// batched paths (bands.cpp): which rows the two score passes keep, where the
// optimal path crosses them, and the bands between clean crossings.
#pragma once

#include <stdint.h>

#include <vector>

#include "context.h"
#include "tb_kernels.h"
#include "traceback.h"

namespace swh {

// Kept-row layout of one pair (strips of H = 64 R rows, cuts C = H every apart).
// Forward pass: strip s keeps its last row when (s + 1) % every == 0, in slot
// (s + 1) / every - 1; slot k - 1 holds the cut row x = k C - 1.  Reverse pass:
// same R with `lead` all-zero pad rows on top, so that reversed strip s' ends
// on row q_end - (s' + 1) H + 1 + lead = x + 2 exactly when s' + 1 = T - k every,
// T = (q_end + lead) / H; it keeps its last row when (s' + 1 + phase) % every
// == 0 (phase = -T mod every), in slot (T + phase) / every - 1 - k.
struct BandKeep {
    int R = 0, every = 0;               // every == 0: no kept rows
    int64_t kf = 0, fstride = 0;        // kept forward rows, records per row
    int64_t lead = 0, T = 0, kr = 0, rstride = 0;
    int phase = 0;
    int Rr = 0, every_r = 0;            // reverse strip height and strips between its kept rows
    // global passes: keep_f / keep_r point one record past the boundary
    // column's record (DP column 0), which the cut scan reads at index -1
    bool global = false;
    const Border *keep_f = nullptr, *keep_r = nullptr;
};

// Forward layout of an n x m pass; returns the records to keep (kf * fstride).
int64_t band_forward_layout(int R, int every, int64_t n, int64_t m, BandKeep &k);
// Reverse layout once the end cell is known; returns the records to keep.
// The reverse pass runs rows_per_lane rr when 64 rr divides the distance
// between kept rows (else the forward height).
int64_t band_reverse_layout(int64_t q_end, int64_t t_end, BandKeep &k, int rr = 0);

// One CutDesc per kept row strictly inside the pair's rectangle (rows x with
// q_begin <= x < q_end), with the cut row of each.  qcodes / tcodes: the
// pair's codes on the device, row 0 and column 0 first.
void band_cuts(const BandKeep &k, const swh_alignment &al, int32_t S, const uint8_t *qcodes,
               const uint8_t *tcodes, std::vector<CutDesc> &cd, std::vector<int64_t> &rows);

// Scan and resolve all cuts (one launch each); co receives one entry per cut.
swh_status resolve_cuts(swh_ctx *ctx, const Scoring &sc, hipStream_t st, const std::vector<CutDesc> &cd,
                        std::vector<CutOut> &co);

// Bands of a rectangle from its resolved cuts (in row order).  Empty when
// there is no clean cut, or when a cut has no edge at all (cannot happen for
// a true optimum; the plain traceback then takes over).
void bands_from_cuts(const CutOut *co, const int64_t *rows, int nc, const swh_alignment &al, int32_t S,
                     std::vector<TbBand> &bands);

}  // namespace swh
