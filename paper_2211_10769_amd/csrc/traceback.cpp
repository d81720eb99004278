// traceback.cpp -- placeholder until the linear-space traceback lands.
#include "traceback.h"

namespace swh {

swh_status traceback(swh_ctx *ctx, const uint8_t *, int64_t, const uint8_t *, int64_t, const Scoring &, int32_t,
                     hipStream_t, std::string &, TracebackStats &)
{
    return fail(ctx, SWH_E_INVAL, "CIGAR mode is not available yet");
}

}  // namespace swh
