// dp_strip16.hip -- the local score pass in packed 16-bit arithmetic
// (gfx950): two cells per 32-bit lane operation, exact while every value stays
// below 32767 - max s; a pass that reaches that limit is recomputed in 32
// bits by the host (lower-precision integers are the direction the paper's
// conclusions name as future work for SW#).
//
// Layout.  One wave owns a strip of 128 RH rows as two sub-strips of 64 RH
// rows held in the two halves of every register: lane l's low halves are rows
// [l RH, l RH + RH) of the upper sub-strip, its high halves the same rows of
// the lower sub-strip (64 RH further down).  Within each half the 32-bit
// kernel's scheme runs unchanged: at step t the low half of lane l is at
// column t - l + 1, the vertical dependency inside the lane is a register
// chain, lane l-1 hands its last row to lane l.  The high half runs 64
// columns behind the low half, so that lane 0's high half can take the upper
// sub-strip's last row (lane 63's low half) one step after it was produced: a
// whole-wave rotate (wave_ror:1) brings lane 63's value to lane 0, and one
// v_perm per value puts it in the high half beside the border row from HBM in
// the low half.  The border row itself is exchanged in the 32-bit layout of
// the other kernel (H and the F handed down), so kept rows, the band
// traceback and every host routine read the same records; the strip's last
// row is lane 63's high half, one block later than in the 32-bit kernel.
//
// Arithmetic (local recurrences of the paper's Background section, Gotoh's
// three states with affine gaps): H, E and F are held in [0, 32767]; E and F
// clamped at zero by unsigned saturating subtraction (max(E, 0) obeys the
// same recurrence clamped at 0); diag + s by a signed saturating add, which
// may go below zero, where the signed maximum with E, F >= 0 supplies the
// local floor.  Eight packed operations per row pair of cells:
//   h = max(max(diag + s, E), F); hop = h -sat o;
//   F = max(F -sat e, hop); E = max(E -sat e, hop).
// Saturation: diag + s can only clip when diag > 32767 - max s, and such a
// diag is itself a cell of the pass; so a pass whose maximum stays below
// 32767 - max s computed every value exactly.  The host checks the maximum.
//
// Scores: per-half int16 query profiles in LDS, prof[half][plane][code][lane]
// of int16 pairs (two consecutive rows per word, RH/2 words per lane,
// planes of four words so every read is a conflict-free ds_read_b128); row
// k's packed score comes from one v_perm of the two halves' words.  The two
// halves look up different columns (64 apart): their codes travel together in
// one register as profile byte offsets (low 16 bits the low half's, high 16
// bits the high half's), and the high half's feed is the low half's feed of
// the previous block.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "engine.h"
#include "strip_sync.h"

namespace swh {

namespace {

using namespace strip_dev;

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));

constexpr int kDppWaveRor1 = 0x13C;   // lane i reads lane i-1, lane 0 reads lane 63

// every lane has a source under the rotation, so no old value is needed
__device__ __forceinline__ unsigned rot1(unsigned src)
{
    return (unsigned)__builtin_amdgcn_mov_dpp((int)src, kDppWaveRor1, 0xF, 0xF, false);
}

__device__ __forceinline__ u16x2 as16(unsigned x) { return __builtin_bit_cast(u16x2, x); }
__device__ __forceinline__ unsigned as32(u16x2 x) { return __builtin_bit_cast(unsigned, x); }
__device__ __forceinline__ unsigned subs(unsigned a, unsigned b)
{
    return as32(__builtin_elementwise_sub_sat(as16(a), as16(b)));
}
__device__ __forceinline__ unsigned umax(unsigned a, unsigned b)
{
    return as32(__builtin_elementwise_max(as16(a), as16(b)));
}
// signed halves: diag + s (may be negative) and the maximum that absorbs it
__device__ __forceinline__ unsigned sadds(unsigned a, unsigned b)
{
    return __builtin_bit_cast(unsigned, __builtin_elementwise_add_sat(__builtin_bit_cast(i16x2, a),
                                                                        __builtin_bit_cast(i16x2, b)));
}
__device__ __forceinline__ unsigned smax(unsigned a, unsigned b)
{
    return __builtin_bit_cast(unsigned, __builtin_elementwise_max(__builtin_bit_cast(i16x2, a),
                                                                   __builtin_bit_cast(i16x2, b)));
}

template <int RH>
struct Prof16 {
    static constexpr int W = RH / 2;                   // int16-pair words per (half, code, lane)
    static constexpr int P = (W + 3) / 4;              // planes of (up to) four words
    static constexpr int PW = W < 4 ? W : 4;           // words per plane
};

// word w of (half, code, lane): plane w / 4, prof[((half * P + plane) * A1 + code) * 64 * PW + lane * PW + w % 4]
template <int RH>
__device__ __forceinline__ int prof16_index(int a1, int half, int code, int lane, int w)
{
    constexpr int P = Prof16<RH>::P, PW = Prof16<RH>::PW;
    return (((half * P + w / PW) * a1 + code) * 64 + lane) * PW + (w % PW);
}

// The RH / 2 words of one (half, code, lane): base is the lane's entry of the
// half's first plane and code 0, off the code's byte offset in a plane,
// plane_b the bytes between planes.
template <int RH>
__device__ __forceinline__ void load_prof16_at(const int *base, unsigned off, int plane_b, unsigned (&w)[RH / 2])
{
    constexpr int P = Prof16<RH>::P, PW = Prof16<RH>::PW;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int *q = reinterpret_cast<const int *>(reinterpret_cast<const char *>(base) + off + p * plane_b);
        if constexpr (PW == 4) {
            const int4 x = reinterpret_cast<const int4 *>(q)[0];
            w[4 * p] = (unsigned)x.x;
            w[4 * p + 1] = (unsigned)x.y;
            w[4 * p + 2] = (unsigned)x.z;
            w[4 * p + 3] = (unsigned)x.w;
        } else if constexpr (PW == 2) {
            const int2 x = reinterpret_cast<const int2 *>(q)[0];
            w[0] = (unsigned)x.x;
            w[1] = (unsigned)x.y;
        } else {
            w[0] = (unsigned)q[0];
        }
    }
}

// Waves per SIMD one workgroup may bring (bounds the registers a wave may use).
template <int RH>
constexpr int kWg16PerSimd = RH <= 8 ? 4 : 2;

template <int RH, bool PRUNE>
__global__ void __launch_bounds__(256 * kWg16PerSimd<RH>) strip16_kernel(StripArgs a)
{
    extern __shared__ int prof_all[];
    constexpr int W = Prof16<RH>::W;
    const int lane = threadIdx.x & 63;
    const int pad = a.asize;
    const int A1 = a.asize + 1;
    int *prof = prof_all + (threadIdx.x >> 6) * (2 * A1 * 64 * W);   // this wave's profiles
    const unsigned o2 = (unsigned)a.o | ((unsigned)a.o << 16);
    const unsigned e2 = (unsigned)a.e | ((unsigned)a.e << 16);

    for (;;) {
        const int sv = __hip_atomic_fetch_add(a.ticket, lane == 0 ? 1 : 0, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
        const int sg = __builtin_amdgcn_readfirstlane(sv);
        if (sg >= a.total_strips) break;
        if (a.cancel &&
            __builtin_amdgcn_readfirstlane(__hip_atomic_load(a.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM))) {
            __hip_atomic_store(a.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        const int g = a.strip_order ? __builtin_amdgcn_readfirstlane((int)a.strip_order[sg]) : sg;
        const int pi = a.strip_prob ? __builtin_amdgcn_readfirstlane((int)a.strip_prob[g]) : 0;
        const Problem P = a.probs[pi];
        const int s = g - P.strip0;
        const int64_t rowA = (int64_t)s * 128 * RH + (int64_t)lane * RH;   // low halves (0-based rows)
        const int64_t rowB = rowA + 64 * RH;                                 // high halves

        // ---- the two halves' int16 profiles (written and read by this lane only)
        for (int c = 0; c < A1; ++c) {
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                const int64_t r0 = half ? rowB : rowA;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    unsigned word = 0;
#pragma unroll
                    for (int b2 = 0; b2 < 2; ++b2) {
                        const int q = P.qc[r0 + 2 * w + b2];
                        const int v = (q >= a.asize || c >= a.asize) ? -128 : (int)a.mat[q * a.asize + c];
                        word |= (unsigned)(v & 0xFFFF) << (16 * b2);
                    }
                    prof[prof16_index<RH>(A1, half, c, lane, w)] = (int)word;
                }
            }
        }
        // kept rows count half strips (64 RH rows): half strip 2 s ends with the
        // upper sub-strip (lane 63's low halves), 2 s + 1 with the lower one; a
        // lower sub-strip that starts below the last row is not a strip of the
        // pass and keeps nothing (its slot would lie past the kept rows)
        Border *keep_lo = nullptr, *keep_hi = nullptr;
        if (P.save_every > 0) {
            const int t0 = 2 * s + 1 + P.save_phase, t1 = 2 * s + 2 + P.save_phase;
            if (t0 % P.save_every == 0) keep_lo = P.save + (int64_t)(t0 / P.save_every - 1) * P.save_stride;
            if (t1 % P.save_every == 0 && (int64_t)(2 * s + 1) * 64 * RH < (int64_t)P.n)
                keep_hi = P.save + (int64_t)(t1 / P.save_every - 1) * P.save_stride;
        }

        unsigned hp[RH], E[RH];
#pragma unroll
        for (int k = 0; k < RH; ++k) { hp[k] = 0u; E[k] = 0u; }
        unsigned hup_prev = 0u;            // H(row0 - 1, j - 1) of both halves
        unsigned hbot = 0u, fbot = 0u;     // the lane's last row outputs of the previous step
        // lane 63's outputs of the block's steps, collected one per lane: high
        // halves (H low, F high), and low halves where the upper sub-strip's last
        // row is kept
        unsigned ohf = 0u, olf = 0u;
        // Best cell: lane keys (H << 16) | (2 RH - 1 - i), i the row over the
        // lane's 2 RH rows (low half first), so a maximum orders a step's cells
        // by value, then smaller row; bkey keeps the largest key and bstep the
        // first step that reached it.  Keys are formed only in steps where some
        // half reaches its threshold (thr2 + 1 per half): the lane's own best
        // value, and at every block end the strip's best so far over all lanes
        // (value V at row r*): a half whose rows all lie below r* needs V + 1,
        // the others V.  No cell below its threshold can be the strip's best,
        // so the strip's result is that of a tracker that forms every key.
        int bkey = 0, bstep = 0;
        unsigned thrw2 = 0u, thr2 = 0u;

        // Column codes as profile byte offsets (CS bytes per code in a plane):
        // low 16 bits the low half's column, high 16 bits the high half's.
        constexpr unsigned CS = 4u * Prof16<RH>::PW * 64u;
        const int plane_b = A1 * (int)CS;
        const int *base_lo = prof + lane * Prof16<RH>::PW;
        const int *base_hi = base_lo + Prof16<RH>::P * A1 * 64 * Prof16<RH>::PW;
        int code0 = lane == 0 ? (int)P.tc[0] : pad;
        int traw = P.tc[1 + lane];                            // the low half's feed (raw codes)
        // the high half's feed of block 0: columns <= 0 (pad), except that its
        // last entry brings column 1 to lane 0 on step 64
        int traw_h = lane == 63 ? (int)P.tc[0] : pad;
        int fh = 0, ff = 0;
        bool ok = true;
        if (!wait_chunk(a, P.flags, 0, s)) ok = false;
        if (ok) load_border(P.border + lane, fh, ff);
        int fl_next = 64 < P.m ? peek_chunk(P.flags, 1) : s;
        code0 = settled(code0);
        traw = settled(traw);
        traw_h = settled(traw_h);
        // the border chunk packed: H in the low half, F in the high half
        unsigned hf = ((unsigned)settled(fh) & 0xFFFFu) | ((unsigned)settled(ff) << 16);
        unsigned code2 = (unsigned)code0 * CS | (((unsigned)pad * CS) << 16);
        unsigned tfeed2 = (unsigned)traw * CS | (((unsigned)traw_h * CS) << 16);
        // lane 0 takes the border into the low half and lane 63's low half into
        // the high half: H from the chunk's low half, F from its high half
        const unsigned sel_h = lane == 0 ? 0x05040100u : 0x07060504u;
        const unsigned sel_f = lane == 0 ? 0x05040302u : 0x07060504u;

        unsigned sl[W], sh[W];
        load_prof16_at<RH>(base_lo, code2 & 0xFFFFu, plane_b, sl);
        load_prof16_at<RH>(base_hi, code2 >> 16, plane_b, sh);

        for (int b = 0; b < P.nblocks && ok; ++b) {
            const int traw_n = P.tc[64 * (b + 1) + 1 + lane];
            int fh_n = 0, ff_n = 0;
            if (64 * (b + 1) < P.m) {
                if (__builtin_amdgcn_readfirstlane(fl_next) < s && !wait_chunk(a, P.flags, b + 1, s)) {
                    ok = false;
                    break;
                }
                load_border(P.border + 64 * (b + 1) + lane, fh_n, ff_n);
                fl_next = 64 * (b + 2) < P.m ? peek_chunk(P.flags, b + 2) : s;
            }
            const int tbase = 64 * b;

            bool pruned = false;
            if (PRUNE && P.prune > 0) {
                unsigned hin = umax(umax(hup_prev, hbot), fbot);
#pragma unroll
                for (int k = 0; k < RH; ++k) hin = umax(hin, umax(hp[k], E[k]));
                int hmax = max((int)(hin & 0xFFFF), (int)(hin >> 16));
                hmax = max(hmax, max((int)(hf & 0xFFFFu), (int)(hf >> 16)));
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) hmax = max(hmax, __shfl_xor(hmax, off));
                hmax = __builtin_amdgcn_readfirstlane(hmax);
                // the high half is 64 columns behind: count columns from its first one
                const int64_t rows_left = (int64_t)P.n - (int64_t)s * 128 * RH;
                const int64_t cols_left = (int64_t)P.m - max(64 * b - 127, 0);
                const int64_t bound = (int64_t)max(hmax, 0) + (int64_t)max(a.smax, 0) * min(rows_left, cols_left);
                pruned = bound < (int64_t)P.prune;
            }
            if (PRUNE && pruned) {
                // the block's steps at the floor (see the 32-bit kernel); lane 0's
                // next diagonal input: the border chunk's last record (low half)
                // and lane 63's floor value (high half)
                const unsigned last_h = (unsigned)__shfl((int)hf, 63) & 0xFFFFu;
#pragma unroll
                for (int k = 0; k < RH; ++k) { hp[k] = 0u; E[k] = 0u; }
                hbot = 0u;
                fbot = 0u;
                ohf = 0u;
                olf = 0u;
                hup_prev = lane == 0 ? last_h : 0u;
                code2 = (unsigned)__shfl((int)tfeed2, 63 - lane);
                load_prof16_at<RH>(base_lo, code2 & 0xFFFFu, plane_b, sl);
                load_prof16_at<RH>(base_hi, code2 >> 16, plane_b, sh);
            } else {
                auto block_steps = [&](auto keep_c) {
                    constexpr bool KEEP = decltype(keep_c)::value;
#pragma unroll 2
                    for (int u = 0; u < 64; ++u) {
                        const unsigned code2_n = (unsigned)shr1((int)tfeed2, (int)code2);
                        tfeed2 = (unsigned)shl1((int)tfeed2, (int)tfeed2);
                        unsigned sl_n[W], sh_n[W];
                        __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): retire the previous profile reads
                        load_prof16_at<RH>(base_lo, code2_n & 0xFFFFu, plane_b, sl_n);
                        load_prof16_at<RH>(base_hi, code2_n >> 16, plane_b, sh_n);
                        __builtin_amdgcn_sched_barrier(0);
                        // the rows above each half's first row at this column
                        const unsigned hup = __builtin_amdgcn_perm(rot1(hbot), hf, sel_h);
                        unsigned f = __builtin_amdgcn_perm(rot1(fbot), hf, sel_f);
                        hf = (unsigned)shl1((int)hf, (int)hf);

                        unsigned dg = hup_prev;
#pragma unroll
                        for (int k = 0; k < RH; ++k) {
                            const unsigned sel = (k & 1) ? 0x07060302u : 0x05040100u;
                            const unsigned sk = __builtin_amdgcn_perm(sh[k >> 1], sl[k >> 1], sel);
                            const unsigned h = smax(smax(sadds(dg, sk), E[k]), f);
                            const unsigned hop = subs(h, o2);
                            f = umax(subs(f, e2), hop);
                            E[k] = umax(subs(E[k], e2), hop);
                            dg = hp[k];
                            hp[k] = h;
                        }
                        hup_prev = hup;
                        hbot = hp[RH - 1];
                        fbot = f;
                        ohf = (unsigned)shl1((int)__builtin_amdgcn_perm(fbot, hbot, 0x07060302u), (int)ohf);
                        if constexpr (KEEP)
                            olf = (unsigned)shl1((int)__builtin_amdgcn_perm(fbot, hbot, 0x05040100u), (int)olf);

                        unsigned hm = hp[0];
#pragma unroll
                        for (int k = 1; k < RH; ++k) hm = umax(hm, hp[k]);
                        if (__builtin_amdgcn_ballot_w64(subs(hm, thr2) != 0u)) {
                            int mx = (int)((hp[0] << 16) | (2u * RH - 1u));
#pragma unroll
                            for (int k = 1; k < RH; ++k) mx = max(mx, (int)((hp[k] << 16) | (unsigned)(2 * RH - 1 - k)));
#pragma unroll
                            for (int k = 0; k < RH; ++k) mx = max(mx, (int)((hp[k] & 0xFFFF0000u) | (unsigned)(RH - 1 - k)));
                            const bool gt = mx > bkey;
                            bkey = gt ? mx : bkey;
                            bstep = gt ? tbase + u : bstep;
                            const unsigned own = (unsigned)max((bkey >> 16) - 1, 0);
                            thr2 = umax(thrw2, own | (own << 16));
                        }
#pragma unroll
                        for (int w = 0; w < W; ++w) {
                            sl[w] = sl_n[w];
                            sh[w] = sh_n[w];
                        }
                        code2 = code2_n;
                    }
                };
                if (keep_lo)
                    block_steps(BoolC<true>{});
                else
                    block_steps(BoolC<false>{});
            }

            // the strip's best so far (strip-relative key: value, then smaller
            // row) sets every lane's threshold for the next block
            {
                const int bv = bkey >> 16;
                const int i = 2 * RH - 1 - (bkey & 0xFFFF);
                const int row = lane * RH + (i < RH ? i : 63 * RH + i);
                int K = bv > 0 ? (bv << 11) | (2047 - row) : 0;
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) K = max(K, __shfl_xor(K, off));
                K = __builtin_amdgcn_readfirstlane(K);
                const int V = K >> 11, brow = 2047 - (K & 2047);
                const unsigned tlo = (unsigned)max(V + (lane * RH > brow ? 1 : 0), 1) - 1u;
                const unsigned thi = (unsigned)max(V + (64 * RH + lane * RH > brow ? 1 : 0), 1) - 1u;
                thrw2 = tlo | (thi << 16);
                const unsigned own = (unsigned)max(bv - 1, 0);
                thr2 = umax(thrw2, own | (own << 16));
            }

            // border records: lane l holds lane 63's high-half output of step
            // 64 b + l, column 64 b + l - 126 (1-based); chunk b - 3 was completed
            // by the previous block's records and is published once they drained
            drain_stores();
            if (lane == 0 && b >= 3)
                __hip_atomic_store(P.flags + (b - 3), s + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            {
                const int tn = settled(traw_n);
                tfeed2 = (unsigned)tn * CS | (((unsigned)traw * CS) << 16);   // the high half takes this block's feed
                traw = tn;
            }
            hf = ((unsigned)settled(fh_n) & 0xFFFFu) | ((unsigned)settled(ff_n) << 16);
            const int idx = 64 * b + lane - 127;
            if (idx >= 0 && idx < P.m) {
                const int h32 = (int)(ohf & 0xFFFFu), f32 = (int)(ohf >> 16);
                store_border(P.border + idx, h32, f32);
                if (keep_hi) keep_hi[idx] = Border{h32, f32};
            }
            // the upper sub-strip's last row (low halves) runs 64 columns ahead
            const int idx_lo = 64 * b + lane - 63;
            if (keep_lo && idx_lo >= 0 && idx_lo < P.m)
                keep_lo[idx_lo] = Border{(int)(olf & 0xFFFFu), (int)(olf >> 16)};
        }
        drain_stores();
        {
            const int nchunks = (P.m + 63) / 64;
            const int first = ok ? max(P.nblocks - 3, 0) : 0;
            for (int c0 = first; c0 < nchunks; c0 += 64) {
                const int c = c0 + lane;
                if (c < nchunks) __hip_atomic_store(P.flags + c, s + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }

        // lane's best: row index i over the lane's 2 RH rows (0 .. RH-1 low, RH .. 2RH-1 high)
        int bv = bkey >> 16;
        const int i = 2 * RH - 1 - (bkey & 0xFFFF);
        int br = 0, bc = 0;
        if (bv > 0) {
            br = (int)((i < RH ? rowA + i : rowB + (i - RH)) + 1);
            bc = bstep - lane + 1 - (i < RH ? 0 : 64);
        }
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

template <int RH>
hipError_t launch16_t(const StripArgs &a, const StripLaunch &l, hipStream_t st, bool prune)
{
    if (prune)
        hipLaunchKernelGGL((strip16_kernel<RH, true>), dim3(l.nwg), dim3(64 * l.waves), l.lds, st, a);
    else
        hipLaunchKernelGGL((strip16_kernel<RH, false>), dim3(l.nwg), dim3(64 * l.waves), l.lds, st, a);
    return hipGetLastError();
}

template <int RH>
int blocks16_t(int threads, size_t lds)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(&strip16_kernel<RH, false>),
                                                     threads, lds) != hipSuccess)
        return 0;
    return n;
}

int blocks16(int RH, int threads, size_t lds)
{
    if (RH == 4) return blocks16_t<4>(threads, lds);
    if (RH == 8) return blocks16_t<8>(threads, lds);
    if (RH == 16) return blocks16_t<16>(threads, lds);
    return 0;
}

}  // namespace

size_t strip16_lds_bytes(int R, int asize) { return (size_t)(asize + 1) * 64 * (size_t)R * 2; }

bool strip16_supported(int R, int asize, int device)
{
    if (R != 8 && R != 16 && R != 32) return false;
    int lds_wg = 0;
    if (hipDeviceGetAttribute(&lds_wg, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return strip16_lds_bytes(R, asize) <= (size_t)lds_wg;
}

bool strip16_balanced_launch(int device, int R, int asize, int per_simd, int num_cu, StripLaunch &out)
{
    const int RH = R / 2;
    int lds_cu = 0, lds_wg = 0;
    if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) != hipSuccess ||
        hipDeviceGetAttribute(&lds_wg, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess ||
        lds_cu <= 0 || lds_wg <= 0 || num_cu <= 0 || per_simd < 1) {
        (void)hipGetLastError();
        return false;
    }
    const size_t wave_lds = strip16_lds_bytes(R, asize);
    const int cap = 4 * (RH <= 8 ? kWg16PerSimd<4> : kWg16PerSimd<16>);
    for (int wgs = 1; wgs <= 2; ++wgs) {
        if (per_simd % wgs != 0) continue;
        const int waves = 4 * per_simd / wgs;
        if (waves > cap) continue;
        const size_t lds = std::max(wave_lds * waves, (size_t)lds_cu / (wgs + 1) + 256);
        if (lds > (size_t)lds_wg || lds * wgs > (size_t)lds_cu) continue;
        if (blocks16(RH, 64 * waves, lds) != wgs) continue;
        out = StripLaunch{num_cu * wgs, waves, lds};
        return true;
    }
    return false;
}

int strip16_grid_limit(int device, int R, int asize)
{
    int per_cu = blocks16(R / 2, 64, strip16_lds_bytes(R, asize));
    if (per_cu < 1) per_cu = 1;
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return per_cu * 64;
    return per_cu * p.multiProcessorCount;
}

hipError_t launch_strip16(const StripArgs &a, int R, const StripLaunch &grid, hipStream_t st, bool prune)
{
    if (R == 8) return launch16_t<4>(a, grid, st, prune);
    if (R == 16) return launch16_t<8>(a, grid, st, prune);
    if (R == 32) return launch16_t<16>(a, grid, st, prune);
    return hipErrorInvalidValue;
}

}  // namespace swh
