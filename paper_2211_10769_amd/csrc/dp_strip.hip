// dp_strip.hip -- the score pass of the alignment DP on CDNA4 (gfx950).
//
// One wave64 owns a strip of 64*R consecutive query rows; lane l owns rows
// [l*R, l*R + R) of the strip.  The wave sweeps the target columns with a
// skew of one column per lane: at step t lane l works on column t - l + 1,
// all R of its rows at that column, the vertical dependency inside the lane
// carried in registers.  Lane l-1's last row (H and the F it passes down)
// reaches lane l through a whole-wave DPP shift (wave_shr:1); lane 0 reads the
// previous strip's last row from a border buffer in HBM, lane 63's last row is
// collected 64 columns at a time (wave_shl:1) and written back to the same
// buffer, in place.  Strips are taken in order from an atomic ticket and
// hand over the border one 64-column chunk at a time through per-chunk
// counters, so a strip only ever waits on a strip with a smaller ticket that
// is already running: the wavefront cannot deadlock whatever the grid size.
//
// Recurrences (paper, Background: Smith-Waterman with affine open/extension
// penalties, the "resolution" phase of SW#):
//   E(i,j) = max(E(i,j-1) - e, H(i,j-1) - o)
//   F(i,j) = max(F(i-1,j) - e, H(i-1,j) - o)
//   H(i,j) = max(floor, H(i-1,j-1) + s(a_i,b_j), E(i,j), F(i,j))
// LOCAL: floor = 0 and E, F are stored clamped at 0 -- max(E,0) obeys the
// same recurrence clamped at 0, and H = max3(diag + s, E', F') then needs no
// extra operation.  GLOBAL (traceback passes): floor = kNeg, no clamp.
//
// Substitution scores come from a per-strip query profile in LDS: for each
// symbol code, the lane's R int8 scores in R/4 consecutive words,
// prof[code][lane][R/4] (above 16 rows in two planes, see prof_index).  One
// step reads them with a single ds_read_b128 (R=16), conflict-free whatever
// code each lane holds, and each byte enters
// the add through an SDWA sign-extended byte select at no extra cost.  The
// pad code scores -128: in a virtual column left of the sweep the diagonal
// is the boundary value, so the pad can never raise H there; everything to
// the right of the last column or below the last row is never read back.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "engine.h"
#include "strip_sync.h"

namespace swh {

namespace {

using namespace strip_dev;

template <int R>
struct Prof {
    static constexpr int W = R / 4;                      // profile words per (code, lane)
    static constexpr int LOGR = R > 16 ? 5 : R == 16 ? 4 : R == 8 ? 3 : 2;   // bits of a row index
};

// Word w of (code, lane): with W <= 4 words at prof[(code*64 + lane)*W + w];
// with W > 4 in two planes so that every read is a conflict-free
// lane-contiguous ds_read: words 0..3 at prof[(code*64 + lane)*4 + w], words
// 4..W-1 at prof[A1*256 + (code*64 + lane)*(W-4) + w-4].
template <int W>
__device__ __forceinline__ int prof_index(int a1, int code, int lane, int w)
{
    if constexpr (W <= 4) return (code * 64 + lane) * W + w;
    return w < 4 ? (code * 64 + lane) * 4 + w : a1 * 256 + (code * 64 + lane) * (W - 4) + (w - 4);
}

template <int W>
__device__ __forceinline__ void load_prof(const int *prof, int a1, int code, int lane, int (&w)[W])
{
    const int *p = prof + (code * 64 + lane) * (W > 4 ? 4 : W);
    if constexpr (W > 4) {
        const int4 x = reinterpret_cast<const int4 *>(p)[0];
        w[0] = x.x; w[1] = x.y; w[2] = x.z; w[3] = x.w;
        const int *q = prof + a1 * 256 + (code * 64 + lane) * (W - 4);
        if constexpr (W == 8) {
            const int4 y = reinterpret_cast<const int4 *>(q)[0];
            w[4] = y.x; w[5] = y.y; w[6] = y.z; w[7] = y.w;
        } else if constexpr (W == 6) {
            const int2 y = reinterpret_cast<const int2 *>(q)[0];
            w[4] = y.x; w[5] = y.y;
        } else {
            w[4] = q[0];
        }
    } else if constexpr (W == 4) {
        const int4 x = reinterpret_cast<const int4 *>(p)[0];
        w[0] = x.x; w[1] = x.y; w[2] = x.z; w[3] = x.w;
    } else if constexpr (W == 2) {
        const int2 x = reinterpret_cast<const int2 *>(p)[0];
        w[0] = x.x; w[1] = x.y;
    } else {
        w[0] = p[0];
    }
}

template <int W>
__device__ __forceinline__ int prof_score(const int (&w)[W], int k)
{
    return (int)(signed char)(w[k >> 2] >> (8 * (k & 3)));
}

// One DP step for the lane's R rows at one column.
//   dg   : H(row0-1, j-1)                f    : F handed down into row0 (in), out of row R-1 (out)
//   hp[] : H(row, j-1) in, H(row, j) out E[]  : E(row, j) in (already the value for this column), E(row, j+1) out
// PASS: rows with index < nlead or >= nreal copy the row above (pass-through),
// so the wave's last row reproduces the last real row (global mode, ragged
// strip) and real rows below leading pass-through rows see the top border.
template <int R, bool LOCAL, bool PASS>
__device__ __forceinline__ void dp_step(int (&hp)[R], int (&E)[R], const int (&sc)[R / 4], int dg, int hup,
                                        int &f, int o, int e, int nreal, int nlead)
{
    constexpr int B = LOCAL ? 0 : kNeg;
    int habove = hup;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        int h = max3i(dg + prof_score<R / 4>(sc, k), E[k], f);
        int hop = h - o;
        int fn = max3i(f - e, hop, B);
        E[k] = max3i(E[k] - e, hop, B);
        dg = hp[k];
        if (PASS) {
            const bool real = k >= nlead && k < nreal;
            h = real ? h : habove;
            fn = real ? fn : f;
            habove = h;
        }
        f = fn;
        hp[k] = h;
    }
}

// Waves per SIMD one workgroup may bring (its waves spread round-robin over
// the CU's four SIMDs); it bounds the registers a wave may use.
template <int R>
constexpr int kWgPerSimd = R <= 8 ? 4 : 2;

// Each wave of a workgroup runs strips on its own (no barrier anywhere); the
// workgroup only places waves evenly over the SIMDs of a CU.
// PRUNE (local passes with a known maximum: the reverse pass) is its own
// instantiation, so the forward pass carries no pruning test at all.
template <int R, bool LOCAL, bool PRUNE = false>
__global__ void __launch_bounds__(256 * kWgPerSimd<R>) strip_kernel(StripArgs a)
{
    extern __shared__ int prof_all[];
    constexpr int W = Prof<R>::W;
    constexpr int B = LOCAL ? 0 : kNeg;
    const int lane = threadIdx.x & 63;
    const int pad = a.asize;
    const int A1 = a.asize + 1;
    int *prof = prof_all + (threadIdx.x >> 6) * (A1 * 64 * W);   // this wave's profile
    const int o = a.o, e = a.e;

    for (;;) {
        // every lane takes part in the atomic (lane 0 adds 1, the others 0), so no
        // lane-dependent branch precedes the readfirstlane that broadcasts the ticket
        const int sv = __hip_atomic_fetch_add(a.ticket, lane == 0 ? 1 : 0, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
        const int sg = __builtin_amdgcn_readfirstlane(sv);
        if (sg >= a.total_strips) break;
        // cancellation (pinned host flag, read uncached): this strip is not
        // run, and the abort flag releases every wave waiting on it
        if (a.cancel &&
            __builtin_amdgcn_readfirstlane(__hip_atomic_load(a.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM))) {
            __hip_atomic_store(a.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        const int g = a.strip_order ? __builtin_amdgcn_readfirstlane((int)a.strip_order[sg]) : sg;
        const int pi = a.strip_prob ? __builtin_amdgcn_readfirstlane((int)a.strip_prob[g]) : 0;
        const Problem P = a.probs[pi];
        const int s = g - P.strip0;                                       // strip within the problem
        const int64_t row0 = (int64_t)s * 64 * R + (int64_t)lane * R;   // 0-based

        // ---- query profile for this lane's rows (written and read by this lane only)
        for (int c = 0; c < A1; ++c) {
#pragma unroll
            for (int w = 0; w < W; ++w) {
                unsigned word = 0;
#pragma unroll
                for (int b4 = 0; b4 < 4; ++b4) {
                    const int q = P.qc[row0 + 4 * w + b4];
                    const int v = (q >= a.asize || c >= a.asize) ? -128 : (int)a.mat[q * a.asize + c];
                    word |= (unsigned)(v & 0xFF) << (8 * b4);
                }
                prof[prof_index<W>(A1, c, lane, w)] = (int)word;
            }
        }
        // kept copy of this strip's last row (wave-uniform), if any
        Border *keep = nullptr;
        if (P.save_every > 0) {
            const int t = s + 1 + P.save_phase;
            if (t % P.save_every == 0) keep = P.save + (int64_t)(t / P.save_every - 1) * P.save_stride;
        }
        int nreal = (int)min<int64_t>(max<int64_t>(P.n - row0, 0), R);
        const int nlead = LOCAL ? 0 : (int)min<int64_t>(max<int64_t>((int64_t)P.top_pass - row0, 0), R);
        const bool ragged = !LOCAL && __builtin_amdgcn_readfirstlane(
                                          (int)((int64_t)(s + 1) * 64 * R > P.n || (int64_t)s * 64 * R < P.top_pass));

        // free left border (global mode): H = 0 and E = -o entering column 0;
        // a lane's steps left of column 0 are reset to the same values below
        const bool free_left = !LOCAL && P.free_left != 0;
        const int B0 = free_left ? 0 : B;
        int hp[R], E[R];
#pragma unroll
        for (int k = 0; k < R; ++k) { hp[k] = B0; E[k] = free_left ? -o : B; }
        int hup_prev = B0;         // H(row0-1, j-1): diag of the first row
        int hbot = B0, fbot = B;   // this lane's last row output of the previous step
        int oh = B, of = B;        // collected outputs of lane 63
        // best cell (local): key = (H << log2 R) | (R-1-k) orders cells of one
        // step by value, then smaller row; bkey keeps the largest key seen and
        // bstep the first step that reached it, so (value desc, row asc, column
        // asc) -- the first cell in row-major order -- falls out of a max.
        // The keys of a step are only formed when some lane holds a cell of at
        // least bthr = max(best value, 1): otherwise no key can exceed bkey
        // (cells of value 0 never decide the result), and after a lane's first
        // few hundred columns such steps are rare, so the tracker costs one
        // max tree per step instead of a key per cell.  Cells right of the last
        // column or below the last row only hold values derived from real cells
        // minus a gap penalty, so they can never reach the optimum and need no
        // mask.
        int bkey = 0, bstep = 0, bthr = 1;

        // block 0 inputs, settled before the step loop so that no load is in
        // flight into a register the loop reads (the loop then carries no wait
        // for the next block's prefetches)
        int code = lane == 0 ? (int)P.tc[0] : pad;       // current column's code
        int tfeed = P.tc[1 + lane];                       // lane 0 = code of column t+2
        int fh = B, ff = B;
        bool ok = true;
        if (ok && !wait_chunk(a, P.flags, 0, s)) ok = false;
        if (ok) load_border(P.border + lane, fh, ff);
        // chunk 1's counter, read ahead: checked at the top of block 0
        int fl_next = 64 < P.m ? peek_chunk(P.flags, 1) : s;
        code = settled(code);
        tfeed = settled(tfeed);
        fh = settled(fh);
        ff = settled(ff);

        int sc[W];
        load_prof<W>(prof, A1, code, lane, sc);

        for (int b = 0; b < P.nblocks && ok; ++b) {
            // prefetch the next block's target codes and border chunk; its
            // counter was read a block ago, so the wait is only taken when the
            // strip above had not yet published the chunk then
            const int tfeed_n = P.tc[64 * (b + 1) + 1 + lane];
            int fh_n = B, ff_n = B;
            if (64 * (b + 1) < P.m) {
                if (__builtin_amdgcn_readfirstlane(fl_next) < s && !wait_chunk(a, P.flags, b + 1, s)) {
                    ok = false;
                    break;
                }
                load_border(P.border + 64 * (b + 1) + lane, fh_n, ff_n);
                fl_next = 64 * (b + 2) < P.m ? peek_chunk(P.flags, b + 2) : s;
            }

            const int tbase = 64 * b;
            // One block of 64 steps.  The variants of global mode (ragged
            // strip: pass-through rows; free left border: the steps left of
            // column 0 reset) are separate loops, chosen once per block, so
            // that no step carries a test or a select it does not need.
            auto block_steps = [&](auto pass_c, auto fix_c) {
                constexpr bool PASS = decltype(pass_c)::value;
                constexpr bool FIX = decltype(fix_c)::value;
#pragma unroll 2
                for (int u = 0; u < 64; ++u) {
                    // next column's code (lane 0 from the feed, others from the lane above)
                    const int code_n = shr1(tfeed, code);
                    tfeed = shl1(tfeed, tfeed);
                    int sc_n[W];
                    // retire the previous profile read (issued a whole step ago) before
                    // issuing this one, so that the wait for `sc` below never has to
                    // include the read just issued
                    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0), vmcnt/expcnt untouched
                    load_prof<W>(prof, A1, code_n, lane, sc_n);
                    // keep the profile read for the next column ahead of this column's
                    // arithmetic, so its LDS latency overlaps one whole step
                    __builtin_amdgcn_sched_barrier(0);
                    // row above this lane's first row at this column
                    const int hup = shr1(fh, hbot);
                    int f = shr1(ff, fbot);
                    fh = shl1(fh, fh);
                    ff = shl1(ff, ff);

                    dp_step<R, LOCAL, PASS>(hp, E, sc, hup_prev, hup, f, o, e, nreal, nlead);
                    if (FIX && u < lane) {
#pragma unroll
                        for (int k = 0; k < R; ++k) { hp[k] = 0; E[k] = -o; }
                    }
                    hup_prev = hup;
                    hbot = hp[R - 1];
                    fbot = f;
                    oh = shl1(hbot, oh);
                    of = shl1(fbot, of);

                    if (LOCAL) {
                        constexpr int LOGR = Prof<R>::LOGR;
                        int hm = hp[0];
#pragma unroll
                        for (int k = 1; k < R; ++k) hm = max(hm, hp[k]);
                        if (__builtin_amdgcn_ballot_w64(hm >= bthr)) {   // wave-uniform
                            int mx = (hp[0] << LOGR) | (R - 1);
#pragma unroll
                            for (int k = 1; k < R; ++k) mx = max(mx, (hp[k] << LOGR) | (R - 1 - k));
                            const bool gt = mx > bkey;
                            bkey = gt ? mx : bkey;
                            bstep = gt ? tbase + u : bstep;
                            bthr = max(bkey >> LOGR, 1);
                        }
                    }
#pragma unroll
                    for (int w = 0; w < W; ++w) sc[w] = sc_n[w];
                    code = code_n;
                }
            };
            using T_ = BoolC<true>;
            using F_ = BoolC<false>;
            // Block pruning (local passes whose maximum V is known): every
            // value the block computes, and every value reachable through its
            // cells, is at most max(0, largest input) + smax * min(rows, columns
            // left from the block's first row and column).  Below V the block
            // cannot hold or lead to a cell of value V, nor lie on a path to
            // one, so it is skipped and its cells left at the floor (0): only
            // cells below V can be underestimated, and every cell on an optimal
            // path keeps its exact value.
            bool pruned = false;
            if (LOCAL && PRUNE && P.prune > 0) {
                int hin = max(max(hup_prev, hbot), max(fbot, max(fh, ff)));
#pragma unroll
                for (int k = 0; k < R; ++k) hin = max(hin, max(hp[k], E[k]));
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) hin = max(hin, __shfl_xor(hin, off));
                hin = __builtin_amdgcn_readfirstlane(hin);
                const int64_t rows_left = (int64_t)P.n - (int64_t)s * 64 * R;
                const int64_t cols_left = (int64_t)P.m - max(64 * b - 63, 0);
                const int64_t bound = (int64_t)max(hin, 0) + (int64_t)max(a.smax, 0) * min(rows_left, cols_left);
                pruned = bound < (int64_t)P.prune;
            }
            if (LOCAL && PRUNE && pruned) {
                // the block's 64 steps at the floor: last-row outputs 0, state 0;
                // lane 0's diagonal input of the next block is the chunk's last
                // record (exact: it comes from the strip above)
                const int last_h = __shfl(fh, 63);
#pragma unroll
                for (int k = 0; k < R; ++k) { hp[k] = 0; E[k] = 0; }
                hbot = 0;
                fbot = 0;
                oh = 0;
                of = 0;
                hup_prev = lane == 0 ? last_h : 0;
                code = __shfl(tfeed, 63 - lane);   // column 64 (b + 1) - lane
                load_prof<W>(prof, A1, code, lane, sc);
            } else if (LOCAL) {
                block_steps(F_{}, F_{});
            } else if (ragged) {
                if (free_left && b == 0)
                    block_steps(T_{}, T_{});
                else
                    block_steps(T_{}, F_{});
            } else {
                if (free_left && b == 0)
                    block_steps(F_{}, T_{});
                else
                    block_steps(F_{}, F_{});
            }

            // The previous block's border records (chunk b-2, columns
            // 64(b-2)+1 .. 64(b-1)) were stored a whole block ago: the drain
            // finds them (and this block's prefetches) done, and chunk b-2 is
            // published.  This block's records stay in flight across the next
            // block, so no wave ever stalls on its own stores.
            drain_stores();
            if (lane == 0 && b >= 2)
                __hip_atomic_store(P.flags + (b - 2), s + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            tfeed = settled(tfeed_n);
            fh = settled(fh_n);
            ff = settled(ff_n);
            // lane l holds lane 63's output of step 64b+l: column 64b+l-62 (1-based)
            const int idx = 64 * b + lane - 63;
            if (idx >= 0 && idx < P.m) {
                store_border(P.border + idx, oh, of);
                if (keep) keep[idx] = Border{oh, of};
            }
        }
        // publish the remaining chunks once the last records are done (also on
        // abort, so that no waiter is left behind)
        drain_stores();
        {
            const int nchunks = (P.m + 63) / 64;
            const int first = ok ? max(P.nblocks - 2, 0) : 0;
            for (int c0 = first; c0 < nchunks; c0 += 64) {
                const int c = c0 + lane;
                if (c < nchunks)
                    __hip_atomic_store(P.flags + c, s + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }

        if (LOCAL) {
            constexpr int LOGR = Prof<R>::LOGR;
            int bv = bkey >> LOGR;
            int br = bv > 0 ? (int)(row0 + (R - 1 - (bkey & ((1 << LOGR) - 1))) + 1) : 0;
            int bc = bv > 0 ? bstep - lane + 1 : 0;
            // wave reduction: score desc, row asc, col asc
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const int ov = __shfl_xor(bv, off), orr = __shfl_xor(br, off), oc = __shfl_xor(bc, off);
                const bool better = ov > bv || (ov == bv && (orr < br || (orr == br && oc < bc)));
                bv = better ? ov : bv;
                br = better ? orr : br;
                bc = better ? oc : bc;
            }
            if (lane == 0) a.strip_best[g] = BestCell{bv, br, bc, 0};
        }
    }
}

__global__ void encode_kernel(const char *src, int64_t len, uint8_t *dst, int64_t padded_len,
                              const uint8_t *lut, uint8_t pad, int32_t *bad_pos)
{
    __shared__ uint8_t tab[256];
    for (int i = threadIdx.x; i < 256; i += blockDim.x) tab[i] = lut[i];
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < padded_len; i += stride) {
        uint8_t c = pad;
        if (i < len) {
            c = tab[(uint8_t)src[i]];
            if (c == 0xFF) {
                atomicMin(bad_pos, (int32_t)min<int64_t>(i, INT32_MAX - 1));
                c = pad;
            }
        }
        dst[i] = c;
    }
}

// dst = lead pad codes, then src reversed, then pad codes up to padded_len
__global__ void reverse_kernel(const uint8_t *src, int64_t len, uint8_t *dst, int64_t padded_len, int64_t lead,
                               uint8_t pad)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < padded_len; i += stride) {
        const int64_t k = i - lead;
        dst[i] = (k >= 0 && k < len) ? src[len - 1 - k] : pad;
    }
}

__global__ void fill_border_kernel(Border *b, int64_t count, Border v)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) b[i] = v;
}

__global__ void __launch_bounds__(1024) reduce_best_kernel(const BestCell *in, int32_t count, BestCell *out)
{
    __shared__ BestCell part[1024];
    BestCell best{0, 0, 0, 0};
    for (int i = threadIdx.x; i < count; i += blockDim.x) {
        BestCell c = in[i];
        const bool better = c.score > best.score ||
                            (c.score == best.score && c.score > 0 &&
                             (best.score == 0 || c.row < best.row || (c.row == best.row && c.col < best.col)));
        if (better) best = c;
    }
    part[threadIdx.x] = best;
    __syncthreads();
    for (int w = blockDim.x / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            BestCell x = part[threadIdx.x], y = part[threadIdx.x + w];
            const bool better = y.score > x.score ||
                                (y.score == x.score && y.score > 0 &&
                                 (y.row < x.row || (y.row == x.row && y.col < x.col)));
            if (better) part[threadIdx.x] = y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = part[0];
}

// One block per problem: the problem's best cell over its strips
// (score desc, row asc, col asc).
__global__ void __launch_bounds__(256) reduce_best_multi_kernel(const BestCell *strip_best, const Problem *probs,
                                                                  int32_t nprobs, BestCell *out)
{
    __shared__ BestCell part[256];
    for (int p = blockIdx.x; p < nprobs; p += gridDim.x) {
        const int s0 = probs[p].strip0, ns = probs[p].nstrips;
        BestCell best{0, 0, 0, 0};
        for (int i = threadIdx.x; i < ns; i += blockDim.x) {
            const BestCell c = strip_best[s0 + i];
            const bool better = c.score > best.score ||
                                (c.score == best.score && c.score > 0 &&
                                 (c.row < best.row || (c.row == best.row && c.col < best.col)));
            if (better) best = c;
        }
        part[threadIdx.x] = best;
        __syncthreads();
        for (int w = blockDim.x / 2; w >= 1; w >>= 1) {
            if ((int)threadIdx.x < w) {
                const BestCell x = part[threadIdx.x], y = part[threadIdx.x + w];
                const bool better = y.score > x.score ||
                                    (y.score == x.score && y.score > 0 &&
                                     (y.row < x.row || (y.row == x.row && y.col < x.col)));
                if (better) part[threadIdx.x] = y;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) out[p] = part[0];
        __syncthreads();
    }
}

int grid_for(int64_t work, int threads)
{
    int64_t g = (work + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return (int)g;
}

template <int R, bool LOCAL>
hipError_t launch_strip_t(const StripArgs &a, const StripLaunch &l, hipStream_t st, bool prune)
{
    if (LOCAL && prune)
        hipLaunchKernelGGL((strip_kernel<R, true, true>), dim3(l.nwg), dim3(64 * l.waves), l.lds, st, a);
    else
        hipLaunchKernelGGL((strip_kernel<R, LOCAL>), dim3(l.nwg), dim3(64 * l.waves), l.lds, st, a);
    return hipGetLastError();
}

template <int R, bool LOCAL>
int blocks_per_cu_t(int threads, size_t lds)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(&strip_kernel<R, LOCAL>),
                                                     threads, lds) != hipSuccess)
        return 0;
    return n;
}

int blocks_per_cu(int R, bool local, int threads, size_t lds)
{
#define SWH_BPC(RR)                                                                                         \
    if (R == RR) return local ? blocks_per_cu_t<RR, true>(threads, lds) : blocks_per_cu_t<RR, false>(threads, lds);
    SWH_BPC(4) SWH_BPC(8) SWH_BPC(16) SWH_BPC(20) SWH_BPC(24) SWH_BPC(32)
#undef SWH_BPC
    return 0;
}

int wg_per_simd(int R) { return R <= 8 ? kWgPerSimd<4> : kWgPerSimd<16>; }

template <int R, bool LOCAL>
int grid_limit_t(int device, int asize)
{
    int per_cu = 0;
    hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void *>(&strip_kernel<R, LOCAL>), 64, strip_lds_bytes(R, asize));
    if (err != hipSuccess || per_cu < 1) per_cu = 1;
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return per_cu * 64;
    return per_cu * p.multiProcessorCount;
}

}  // namespace

size_t strip_lds_bytes(int R, int asize) { return (size_t)(asize + 1) * R * 64; }

hipError_t launch_encode(const char *src, int64_t len, uint8_t *dst, int64_t padded_len,
                         const uint8_t *lut, uint8_t pad, int32_t *bad_pos, hipStream_t st)
{
    hipLaunchKernelGGL(encode_kernel, dim3(grid_for(padded_len, 256)), dim3(256), 0, st, src, len, dst,
                       padded_len, lut, pad, bad_pos);
    return hipGetLastError();
}

hipError_t launch_reverse(const uint8_t *src, int64_t len, uint8_t *dst, int64_t padded_len, uint8_t pad,
                          hipStream_t st, int64_t lead)
{
    hipLaunchKernelGGL(reverse_kernel, dim3(grid_for(padded_len, 256)), dim3(256), 0, st, src, len, dst,
                       padded_len, lead, pad);
    return hipGetLastError();
}

hipError_t launch_fill_border(Border *b, int64_t count, Border v, hipStream_t st)
{
    hipLaunchKernelGGL(fill_border_kernel, dim3(grid_for(count, 256)), dim3(256), 0, st, b, count, v);
    return hipGetLastError();
}

hipError_t launch_reduce_best(const BestCell *in, int32_t count, BestCell *out, hipStream_t st)
{
    hipLaunchKernelGGL(reduce_best_kernel, dim3(1), dim3(1024), 0, st, in, count, out);
    return hipGetLastError();
}

hipError_t launch_reduce_best_multi(const BestCell *strip_best, const Problem *probs, int32_t nprobs,
                                    BestCell *out, hipStream_t st)
{
    const int grid = nprobs < 4096 ? (nprobs > 0 ? nprobs : 1) : 4096;
    hipLaunchKernelGGL(reduce_best_multi_kernel, dim3(grid), dim3(256), 0, st, strip_best, probs, nprobs, out);
    return hipGetLastError();
}

bool strip_balanced_launch(int device, int R, bool local, int asize, int per_simd, int num_cu, StripLaunch &out)
{
    int lds_cu = 0, lds_wg = 0;
    if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) != hipSuccess ||
        hipDeviceGetAttribute(&lds_wg, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess ||
        lds_cu <= 0 || lds_wg <= 0 || num_cu <= 0 || per_simd < 1) {
        (void)hipGetLastError();
        return false;
    }
    const size_t wave_lds = strip_lds_bytes(R, asize);
    // one workgroup per CU (needs a request above half the CU's LDS), else two
    for (int wgs = 1; wgs <= 2; ++wgs) {
        if (per_simd % wgs != 0) continue;
        const int waves = 4 * per_simd / wgs;
        if (waves > 4 * wg_per_simd(R)) continue;
        const size_t lds = std::max(wave_lds * waves, (size_t)lds_cu / (wgs + 1) + 256);
        if (lds > (size_t)lds_wg || lds * wgs > (size_t)lds_cu) continue;
        if (blocks_per_cu(R, local, 64 * waves, lds) != wgs) continue;
        out = StripLaunch{num_cu * wgs, waves, lds};
        return true;
    }
    return false;
}

hipError_t launch_strip(const StripArgs &a, int R, bool local, const StripLaunch &grid, hipStream_t st, bool prune)
{
#define SWH_LAUNCH(RR)                                                                                      \
    if (R == RR)                                                                                            \
        return local ? launch_strip_t<RR, true>(a, grid, st, prune) : launch_strip_t<RR, false>(a, grid, st, false);
    SWH_LAUNCH(32) SWH_LAUNCH(24) SWH_LAUNCH(20) SWH_LAUNCH(16) SWH_LAUNCH(8) SWH_LAUNCH(4)
#undef SWH_LAUNCH
    return hipErrorInvalidValue;
}

int strip_grid_limit(int device, int R, bool local, int asize)
{
    if (R == 32) return local ? grid_limit_t<32, true>(device, asize) : grid_limit_t<32, false>(device, asize);
    if (R == 24) return local ? grid_limit_t<24, true>(device, asize) : grid_limit_t<24, false>(device, asize);
    if (R == 20) return local ? grid_limit_t<20, true>(device, asize) : grid_limit_t<20, false>(device, asize);
    if (R == 16) return local ? grid_limit_t<16, true>(device, asize) : grid_limit_t<16, false>(device, asize);
    if (R == 8) return local ? grid_limit_t<8, true>(device, asize) : grid_limit_t<8, false>(device, asize);
    return local ? grid_limit_t<4, true>(device, asize) : grid_limit_t<4, false>(device, asize);
}

}  // namespace swh
