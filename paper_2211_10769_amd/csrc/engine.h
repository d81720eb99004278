// engine.h -- internal interface between the C ABI (capi.cpp), the host
// orchestration (engine.cpp, traceback.cpp) and the HIP kernels (*.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace swh {

// "Minus infinity" of the int32 DP.  Every reachable value of the global DP
// stays well above it (input limits in swh.h), so sums of two of them never
// overflow and no value derived from it can tie with a real one.
constexpr int32_t kNeg = -(1 << 29);

// Border record passed from one strip of rows to the next: the strip's last
// row H and the F value it hands down to the row below.
struct Border {
    int32_t h;
    int32_t f;
};

// Per strip of rows: best cell of the local DP (score, 1-based row, col).
struct BestCell {
    int32_t score, row, col, pad;
};

// One DP problem of the strip-wavefront kernel: a rows x m-columns matrix
// swept by strips of 64*R rows.  Many problems can share one launch: their
// strips share one ticket space, and strips of different problems never wait
// on each other.
struct Problem {
    const uint8_t *qc;       // row codes, padded with the pad code to nstrips*64*R rows
    const uint8_t *tc;       // column codes, 64*(nblocks+3) entries (pad code beyond m)
    Border *border;          // 64*(nblocks+3) entries: top row in, bottom row out
    int32_t *flags;          // nblocks+3 chunk counters, zero on entry
    int32_t n, m;            // real rows and columns
    int32_t nstrips;
    int32_t nblocks;         // sweep_blocks(m)
    int32_t strip0;          // global index of this problem's first strip
    int32_t save_every;      // > 0: keep the bottom rows of some strips (below)
    // Strip s with (s + 1 + save_phase) % save_every == 0 also writes its last
    // row (the same records as the border) to save + slot * save_stride, slot =
    // (s + 1 + save_phase) / save_every - 1, columns 0 .. m-1.
    Border *save;
    int64_t save_stride;
    int32_t save_phase;
    // global mode only: H = 0 left of column 0 (free leading row residues,
    // the overlap form) instead of the penalised boundary
    int32_t free_left;
    // local mode only, > 0: the pass's maximum is known to be prune (a
    // reverse pass); a block whose inputs cannot lead to that value is
    // skipped, its cells left at the floor (block pruning, see the kernel)
    int32_t prune;
    // global mode only: rows 0 .. top_pass-1 pass their input through (H and F
    // of the row above unchanged), so the pass's real rows start below them
    // with the top border as given (aligns strip boundaries, like the zero
    // lead rows of a local pass)
    int32_t top_pass;
};

// Arguments of the strip-wavefront kernel (dp_strip.hip).
struct StripArgs {
    const Problem *probs;
    const int32_t *strip_prob;   // global strip -> problem index (NULL: single problem)
    // ticket -> global strip (NULL: the identity).  Global strips number the
    // strips of problem 0, then problem 1, ...; the order keeps every problem's
    // strips in increasing tickets (a strip only waits for strips taken before it)
    const int32_t *strip_order;
    int32_t total_strips;
    const int8_t *mat;           // asize x asize substitution scores
    int32_t asize;               // the pad code equals asize
    int32_t o, e;                // gap open, gap extend (> 0)
    int32_t smax;                // largest substitution score (block pruning)
    int32_t *ticket;             // strip ticket, zero on entry
    int32_t *abort_flag;         // set when a bounded wait expires (or on cancellation)
    const int32_t *cancel;       // pinned host flag: nonzero = stop taking strips (NULL: none)
    BestCell *strip_best;        // one entry per global strip (local mode)
    uint64_t wait_ticks;         // wall-clock ticks one wait may last before it gives up
};

// Launchers (return hipSuccess or the launch error).
hipError_t launch_encode(const char *src, int64_t len, uint8_t *dst, int64_t padded_len,
                         const uint8_t *lut, uint8_t pad, int32_t *bad_pos, hipStream_t st);
// dst = lead pad codes, then src[len-1] .. src[0], then pad codes up to padded_len
hipError_t launch_reverse(const uint8_t *src, int64_t len, uint8_t *dst, int64_t padded_len,
                          uint8_t pad, hipStream_t st, int64_t lead = 0);
hipError_t launch_fill_border(Border *b, int64_t count, Border v, hipStream_t st);
// A launch of the strip kernel: nwg workgroups of `waves` waves (every wave
// runs strips on its own), lds bytes of LDS per workgroup.
struct StripLaunch {
    int nwg;
    int waves;
    size_t lds;
};
// Every SIMD gets exactly per_simd waves: one or two workgroups per CU whose
// waves the CU spreads over its four SIMDs, held to that count per CU by
// their LDS request.  False when that placement cannot be made.
bool strip_balanced_launch(int device, int R, bool local, int asize, int per_simd, int num_cu, StripLaunch &out);
// prune: some problem of a local launch has Problem::prune set (the pruning
// instantiation of the kernel runs)
hipError_t launch_strip(const StripArgs &a, int R, bool local, const StripLaunch &grid, hipStream_t st,
                        bool prune = false);
hipError_t launch_reduce_best(const BestCell *in, int32_t count, BestCell *out, hipStream_t st);
// Per problem: best cell over its strips (strip_best indexed by global strip).
hipError_t launch_reduce_best_multi(const BestCell *strip_best, const Problem *probs, int32_t nprobs,
                                    BestCell *out, hipStream_t st);

// Packed 16-bit local passes (dp_strip16.hip).  R = rows per lane of the
// kernel's strip (8, 16 or 32; each half of a register holds R / 2 of them,
// one sub-strip of 32 R rows per half); the sweep takes one block more.  Rows
// kept for the band traceback are counted in sub-strips.  Results are exact
// when the pass's maximum stays below sat16_limit.
size_t strip16_lds_bytes(int R, int asize);
bool strip16_supported(int R, int asize, int device);
bool strip16_balanced_launch(int device, int R, int asize, int per_simd, int num_cu, StripLaunch &out);
int strip16_grid_limit(int device, int R, int asize);
hipError_t launch_strip16(const StripArgs &a, int R, const StripLaunch &grid, hipStream_t st, bool prune);
inline int32_t sat16_limit(int smax) { return 32767 - (smax > 0 ? smax : 0); }

// The host side of one strip launch (strips.h: prepare_strips, enqueue_strips).
struct PreparedStrips {
    int R = 0, np = 0;
    bool local = true, int16 = false, prune = false;
    int64_t total_strips = 0, total_flags = 0;
    StripLaunch grid{0, 1, 0};
    std::vector<Problem> tab;
    std::vector<int32_t> strip_prob;
    std::vector<int32_t> strip_order;   // empty: tickets in global strip order
};

// Blocks of 64 steps that sweep m columns with the 63-step lane skew:
// ceil((m + 63) / 64).  Code and border buffers hold 64 * (blocks + 3) entries.
inline int64_t sweep_blocks(int64_t m) { return (m + 63 + 63) / 64; }

// Largest resident grid of the strip kernel for this R and alphabet (per device).
int strip_grid_limit(int device, int R, bool local, int asize);
size_t strip_lds_bytes(int R, int asize);

}  // namespace swh
