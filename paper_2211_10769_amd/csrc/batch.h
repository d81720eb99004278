// batch.h -- many pairwise alignments per call (batch.cpp).
#pragma once

#include <stdint.h>

#include "context.h"

namespace swh {

swh_status align_batch(swh_ctx *ctx, int64_t npairs, const char *q_cat, const int64_t *q_off, const char *t_cat,
                       const int64_t *t_off, const Scoring &sc, int mode, swh_alignment *out, char *cigar_cat,
                       int64_t cigar_cap, int64_t *cigar_off, swh_stats *stats);

}  // namespace swh
