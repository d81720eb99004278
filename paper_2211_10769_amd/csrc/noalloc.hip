// noalloc.hip -- swh_align_dev_noalloc: the score (and start) passes of one
// local alignment on device-resident sequences without any device or host
// allocation, for callers that cannot allocate (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).
//
// Everything the passes need beyond the caller's inputs and output -- the
// encoded and reversed sequences, the border row and its chunk counters, the
// per-strip results, the problem table, the ticket and abort words and the
// scoring tables -- is carved out of one file-scope device array, `scratch`,
// of kScratchBytes.  Each GPU holds its own copy of the array (allocated when
// the library's code object is loaded on that device, kept until the process
// ends); host code never uses the array's name as an address: on the first
// call on a device it asks the runtime for that device's address of the
// array (hipGetSymbolAddress) and keeps it, and every kernel receives
// pointers derived from it.  Calls on one device share the array, so they
// are serialised by a per-device host mutex; every region that must start at
// zero is cleared by a fill kernel at the start of each pass.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/swh.h"
#include "db_kernels.h"
#include "engine.h"
#include "strips.h"

namespace swh {

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_mu[kMaxDevices];
uint8_t *g_scratch[kMaxDevices];   // device address of `scratch` per device (set once)

inline size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// The validated scoring, without the library's string-building error path.
bool make_scoring_plain(const swh_scoring *in, Scoring &out)
{
    if (!in || !in->alphabet || !in->matrix) return false;
    if (in->alphabet_size < 1 || in->alphabet_size > 32) return false;
    if (in->gap_open <= 0 || in->gap_extend <= 0 || in->gap_extend > in->gap_open || in->gap_open > 65535)
        return false;
    for (int c = 0; c < 256; ++c) out.lut[c] = 0xFF;
    for (int k = 0; k < in->alphabet_size; ++k) {
        unsigned char c = (unsigned char)in->alphabet[k];
        if (c == 0) return false;
        unsigned char up = (c >= 'a' && c <= 'z') ? (unsigned char)(c - 'a' + 'A') : c;
        if (out.lut[up] != 0xFF) return false;
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
    return true;
}

// Regions of the scratch array for one call (byte offsets, 256-aligned).
struct Layout {
    size_t mat, lut, misc, sync, prob, best, qc, tc, border, flags, strip_best, qr, tr, total;
};

Layout plan(int64_t n, int64_t m, int R, int Rr)
{
    Layout L{};
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t r = at;
        at += up256(bytes);
        return r;
    };
    L.mat = take(32 * 32);
    L.lut = take(256);
    L.misc = take(64);
    L.sync = take(64);
    L.prob = take(sizeof(Problem));
    L.best = take(sizeof(BestCell));
    L.qc = take((size_t)rows_padded(n, R));
    L.tc = take((size_t)cols_padded(m));
    L.border = take((size_t)cols_padded(m) * sizeof(Border));
    L.flags = take((size_t)(sweep_blocks(m) + 3) * 4);
    const int64_t strips = std::max((n + 64 * R - 1) / (64 * R), (n + 64 * Rr - 1) / (64 * Rr));
    L.strip_best = take((size_t)strips * sizeof(BestCell));
    L.qr = take((size_t)rows_padded(n, Rr));
    L.tr = take((size_t)cols_padded(m));
    L.total = at;
    return L;
}

// One local pass (rows qc x columns tc) over the scratch regions of L; the
// best cell into *best.  prune > 0: the pass's known maximum.
swh_status local_pass_noalloc(int device, int num_cu, uint8_t *base, const Layout &L, const uint8_t *qc, int64_t n,
                              const uint8_t *tc, int64_t m, const Scoring &sc, int R, int32_t prune,
                              hipStream_t st, BestCell *best)
{
    const int64_t tpad = cols_padded(m);
    Problem P{};
    P.qc = qc;
    P.tc = tc;
    P.border = (Border *)(base + L.border);
    P.flags = (int32_t *)(base + L.flags);
    P.n = (int32_t)n;
    P.m = (int32_t)m;
    P.nstrips = (int32_t)((n + 64 * R - 1) / (64 * R));
    P.nblocks = (int32_t)sweep_blocks(m);
    P.strip0 = 0;
    P.prune = prune;
    hipError_t e;
    // the regions that must start at zero, cleared by kernels (no memset node
    // ends up in a graph that captures this stream)
    if ((e = launch_fill_border(P.border, tpad, Border{0, 0}, st)) != hipSuccess ||
        (e = launch_fill_i32(P.flags, P.nblocks + 3, 0, st)) != hipSuccess ||
        (e = launch_fill_i32((int32_t *)(base + L.sync), 16, 0, st)) != hipSuccess ||
        (e = hipMemcpyAsync(base + L.prob, &P, sizeof(P), hipMemcpyHostToDevice, st)) != hipSuccess)
        return SWH_E_DEVICE;
    StripArgs a{};
    a.probs = (const Problem *)(base + L.prob);
    a.strip_prob = nullptr;
    a.total_strips = P.nstrips;
    a.mat = (const int8_t *)(base + L.mat);
    a.asize = sc.asize;
    a.o = sc.o;
    a.e = sc.e;
    a.smax = sc.smax;
    a.ticket = (int32_t *)(base + L.sync);
    a.abort_flag = (int32_t *)(base + L.sync) + 1;
    a.cancel = nullptr;
    a.strip_best = (BestCell *)(base + L.strip_best);
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || khz <= 0) khz = 100000;
    a.wait_ticks = (uint64_t)(30.0 * 1e3 * khz);
    int per_simd = P.nstrips >= 16 ? 1 : 4;
    while (per_simd > 1 && (int64_t)per_simd / 2 * 4 * num_cu >= P.nstrips) per_simd /= 2;
    StripLaunch grid{0, 1, strip_lds_bytes(R, sc.asize)};
    if (!strip_balanced_launch(device, R, true, sc.asize, per_simd, num_cu, grid))
        grid = StripLaunch{strip_grid(P.nstrips, R, strip_grid_limit(device, R, true, sc.asize), num_cu), 1,
                           strip_lds_bytes(R, sc.asize)};
    int32_t flags_host[2] = {0, 0};
    if ((e = launch_strip(a, R, true, grid, st, prune > 0)) != hipSuccess ||
        (e = launch_reduce_best_multi(a.strip_best, a.probs, 1, (BestCell *)(base + L.best), st)) != hipSuccess ||
        (e = hipMemcpyAsync(flags_host, a.ticket, 8, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipMemcpyAsync(best, base + L.best, sizeof(BestCell), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return SWH_E_DEVICE;
    if (flags_host[1]) return SWH_E_TIMEOUT;
    return SWH_OK;
}

swh_status align_noalloc(int device, const char *q_dev, int64_t qlen, const char *t_dev, int64_t tlen,
                         const swh_scoring *scoring, int mode, hipStream_t st, swh_alignment *out)
{
    if (!out || device < 0 || device >= kMaxDevices) return SWH_E_INVAL;
    out->score = 0;
    out->flags = SWH_F_NONE;
    out->q_begin = out->q_end = out->t_begin = out->t_end = -1;
    if (mode != SWH_MODE_SCORE && mode != SWH_MODE_COORDS) return SWH_E_INVAL;
    if (qlen < 0 || tlen < 0 || (qlen && !q_dev) || (tlen && !t_dev)) return SWH_E_INVAL;
    Scoring sc;
    if (!make_scoring_plain(scoring, sc)) return SWH_E_INVAL;
    if (qlen >= ((int64_t)1 << 31) || tlen >= ((int64_t)1 << 31)) return SWH_E_RANGE;
    const int64_t sabs = std::max(std::max(sc.smax, -sc.smin), 1);
    if (std::min(qlen, tlen) * sabs >= ((int64_t)1 << 26)) return SWH_E_RANGE;
    if (qlen == 0 || tlen == 0) return SWH_OK;

    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device >= count) {
        (void)hipGetLastError();
        return SWH_E_INVAL;
    }
    if (hipSetDevice(device) != hipSuccess) return SWH_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_mu[device]);
    if (!g_scratch[device]) {
        // set-up on this device: the device's own address of the array
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return SWH_E_DEVICE;
        }
        g_scratch[device] = (uint8_t *)p;
    }
    uint8_t *base = g_scratch[device];
    int num_cu = 0;
    if (hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || num_cu <= 0)
        return SWH_E_DEVICE;
    const int R = pick_rows_per_lane(qlen, 4 * num_cu);
    // reverse pass: block-pruned, at the shortest step (8 rows per lane) from 512 rows up
    const int Rr = qlen >= 512 ? 8 : pick_rows_per_lane(qlen, 4 * num_cu);
    const Layout L = plan(qlen, tlen, R, Rr);
    if (L.total > kScratchBytes) return SWH_E_RANGE;

    hipError_t e;
    const int32_t init[2] = {INT32_MAX, INT32_MAX};
    if ((e = hipMemcpyAsync(base + L.mat, sc.mat, (size_t)sc.asize * sc.asize, hipMemcpyHostToDevice, st)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(base + L.lut, sc.lut, 256, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(base + L.misc, init, sizeof(init), hipMemcpyHostToDevice, st)) != hipSuccess)
        return SWH_E_DEVICE;
    const uint8_t pad = (uint8_t)sc.asize;
    int32_t *misc = (int32_t *)(base + L.misc);
    uint8_t *qc = base + L.qc, *tc = base + L.tc;
    if ((e = launch_encode(q_dev, qlen, qc, rows_padded(qlen, R), base + L.lut, pad, misc, st)) != hipSuccess ||
        (e = launch_encode(t_dev, tlen, tc, cols_padded(tlen), base + L.lut, pad, misc + 1, st)) != hipSuccess)
        return SWH_E_DEVICE;
    int32_t bad[2] = {0, 0};
    if ((e = hipMemcpyAsync(bad, misc, sizeof(bad), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return SWH_E_DEVICE;
    if (bad[0] != INT32_MAX || bad[1] != INT32_MAX) return SWH_E_ALPHABET;

    BestCell fwd{0, 0, 0, 0};
    swh_status s = local_pass_noalloc(device, num_cu, base, L, qc, qlen, tc, tlen, sc, R, 0, st, &fwd);
    if (s != SWH_OK) return s;
    out->score = fwd.score;
    if (fwd.score == 0) return SWH_OK;
    out->q_end = fwd.row - 1;
    out->t_end = fwd.col - 1;
    if (mode == SWH_MODE_SCORE) return SWH_OK;

    // start: the same pass on the reversed prefixes ending at the end cell
    const int64_t rn = out->q_end + 1, rm = out->t_end + 1;
    uint8_t *qr = base + L.qr, *tr = base + L.tr;
    if ((e = launch_reverse(qc, rn, qr, rows_padded(rn, Rr), pad, st)) != hipSuccess ||
        (e = launch_reverse(tc, rm, tr, cols_padded(rm), pad, st)) != hipSuccess)
        return SWH_E_DEVICE;
    BestCell rev{0, 0, 0, 0};
    if ((s = local_pass_noalloc(device, num_cu, base, L, qr, rn, tr, rm, sc, Rr, fwd.score, st, &rev)) != SWH_OK)
        return s;
    if (rev.score != fwd.score) return SWH_E_DEVICE;
    out->q_begin = out->q_end - (rev.row - 1);
    out->t_begin = out->t_end - (rev.col - 1);
    return SWH_OK;
}

}  // namespace

}  // namespace swh

extern "C" swh_status swh_align_dev_noalloc(int device, const char *q_dev, int64_t qlen, const char *t_dev,
                                            int64_t tlen, const swh_scoring *scoring, int mode, void *stream,
                                            swh_alignment *out)
{
    try {
        return swh::align_noalloc(device, q_dev, qlen, t_dev, tlen, scoring, mode, (hipStream_t)stream, out);
    } catch (...) {
        (void)hipDeviceSynchronize();
        return SWH_E_DEVICE;
    }
}
