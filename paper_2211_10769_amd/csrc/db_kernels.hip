// db_kernels.hip -- exhaustive query-vs-database scoring with inter-task
// parallelism: every (query, database sequence) matrix is independent of the
// others, so each is computed whole by one lane (paper, Background: database
// similarity search).
//
// Each lane aligns one query against two database sequences at once: the
// two DP values live in the two halves of a 32-bit register and every
// recurrence step is one packed 16-bit instruction.  H, E and F are kept in
// [0, 32767]: E and F clamped at zero by unsigned saturating subtraction (as
// in the single-pair kernel), and the diagonal term diag + s by a signed
// saturating add that may go below zero, where the signed max with E, F >= 0
// supplies the zero of the local recurrence.  A lane result of 32767 - 127
// or more may have saturated; such pairs are recomputed in 32-bit (flagged
// -1 here, redone by the host on the strip kernel).
//
// The query is processed 32 rows at a time (rows in registers); the row
// between two chunks (H and the F handed down, both packed) is kept per lane
// in a per-wave border area laid out column-major over the 64 lanes so every
// access is one coalesced 512-byte transaction.  The query profile of a
// chunk (32 int16 scores per symbol) sits in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "db_kernels.h"

namespace swh {

namespace {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u16x2 as16(unsigned x) { return __builtin_bit_cast(u16x2, x); }
__device__ __forceinline__ unsigned as32(u16x2 x) { return __builtin_bit_cast(unsigned, x); }
__device__ __forceinline__ u16x2 subs(u16x2 a, u16x2 b) { return __builtin_elementwise_sub_sat(a, b); }
__device__ __forceinline__ u16x2 vmax(u16x2 a, u16x2 b) { return __builtin_elementwise_max(a, b); }
// signed halves: diag + s (may be negative) and the max that absorbs it
__device__ __forceinline__ i16x2 sadds(u16x2 a, i16x2 b)
{
    return __builtin_elementwise_add_sat(__builtin_bit_cast(i16x2, a), b);
}
__device__ __forceinline__ u16x2 smax3(i16x2 t, u16x2 e, u16x2 f)
{
    return __builtin_bit_cast(u16x2, __builtin_elementwise_max(__builtin_elementwise_max(t, __builtin_bit_cast(i16x2, e)),
                                                                __builtin_bit_cast(i16x2, f)));
}

constexpr int kChunk = 32;                 // query rows per register chunk
constexpr unsigned kSatLimit = 32767 - 127;

// Interleave a group's 128 sequences position-major (res[j * 128 + s]),
// 64 positions at a time through an LDS tile: a wave reads 64 consecutive
// residues of one sequence and writes one 128-byte row per position.
__global__ void __launch_bounds__(256) db_pack_kernel(const uint8_t *codes, const int64_t *offs, const int32_t *perm,
                                                      const DbGroup *groups, uint8_t pad, uint8_t *res)
{
    __shared__ uint8_t tile[64][132];   // [position][sequence]; the odd dword stride avoids bank conflicts
    __shared__ int64_t sbase[128];
    __shared__ int64_t slen[128];
    const DbGroup g = groups[blockIdx.x];
    const int tid = threadIdx.x;
    if (tid < 128) {
        const int32_t idx = perm[g.first + tid];
        sbase[tid] = idx >= 0 ? offs[idx] : 0;
        slen[tid] = idx >= 0 ? offs[idx + 1] - offs[idx] : 0;
    }
    __syncthreads();
    uint8_t *out = res + g.offset;
    for (int64_t j0 = 0; j0 < g.maxlen; j0 += 64) {
        for (int k = tid; k < 64 * 128; k += 256) {
            const int s = k >> 6, jj = k & 63;
            const int64_t j = j0 + jj;
            tile[jj][s] = j < slen[s] ? codes[sbase[s] + j] : pad;
        }
        __syncthreads();
        const int rows = (int)min<int64_t>(64, (int64_t)g.maxlen - j0);
        for (int k = tid; k < rows * 128; k += 256) {
            const int jj = k >> 7, s = k & 127;
            out[(j0 + jj) * 128 + s] = tile[jj][s];
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(64) db_search_kernel(DbSearchArgs a)
{
    __shared__ __align__(16) int prof[33 * 16];   // (asize + 1) symbols x 32 int16 scores
    const int lane = threadIdx.x;
    const int pad = a.asize;
    uint2 *border = reinterpret_cast<uint2 *>(a.border) + (size_t)blockIdx.x * a.max_len * 64;
    const u16x2 o2 = as16((unsigned)a.o | ((unsigned)a.o << 16));
    const u16x2 e2 = as16((unsigned)a.e | ((unsigned)a.e << 16));

    for (;;) {
        const int tv = __hip_atomic_fetch_add(a.ticket, lane == 0 ? 1 : 0, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
        const int w = __builtin_amdgcn_readfirstlane(tv);
        if (w >= a.nwork) break;
        // cancellation (pinned host flag, read uncached): no further unit is run
        if (a.cancel &&
            __builtin_amdgcn_readfirstlane(__hip_atomic_load(a.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)))
            break;
        const DbWork wk = a.work[w];
        const DbGroup g = a.groups[wk.g];
        const int64_t q0 = a.qoff[wk.q];
        const int n = (int)(a.qoff[wk.q + 1] - q0);
        const uint8_t *qc = a.qcodes + q0;
        const uint8_t *res = a.res + g.offset;
        const int maxlen = g.maxlen;
        u16x2 best = as16(0u);

        const int nchunks = (n + kChunk - 1) / kChunk;
        for (int c = 0; c < nchunks; ++c) {
            __syncthreads();
            if (lane <= pad) {
#pragma unroll
                for (int w = 0; w < 16; ++w) {
                    unsigned word = 0;
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        const int row = c * kChunk + 2 * w + b;
                        const int qv = row < n ? (int)qc[row] : pad;
                        const int s = (qv >= pad || lane >= pad) ? -128 : (int)a.mat[qv * a.asize + lane];
                        word |= (unsigned)(s & 0xFFFF) << (16 * b);
                    }
                    prof[lane * 16 + w] = (int)word;
                }
            }
            __syncthreads();

            u16x2 H[kChunk], E[kChunk];
#pragma unroll
            for (int k = 0; k < kChunk; ++k) {
                H[k] = as16(0u);
                E[k] = as16(0u);
            }
            u16x2 diag0 = as16(0u);                        // H(row0 - 1, j - 1)
            const bool first = c == 0, last = c == nchunks - 1;
            unsigned cn = *reinterpret_cast<const unsigned short *>(res + 2 * lane);
            uint2 tn = first ? make_uint2(0u, 0u) : border[lane];
#pragma unroll 2
            for (int j = 0; j < maxlen; ++j) {
                const unsigned cab = cn;
                const uint2 top = tn;
                if (j + 1 < maxlen) {
                    cn = *reinterpret_cast<const unsigned short *>(res + (int64_t)(j + 1) * 128 + 2 * lane);
                    if (!first) tn = border[(int64_t)(j + 1) * 64 + lane];
                }
                const int ca = (int)(cab & 0xFF), cb = (int)(cab >> 8);
                unsigned wa[16], wb[16];
#pragma unroll
                for (int q4 = 0; q4 < 4; ++q4) {
                    const int4 x = reinterpret_cast<const int4 *>(prof + ca * 16)[q4];
                    const int4 y = reinterpret_cast<const int4 *>(prof + cb * 16)[q4];
                    wa[4 * q4] = (unsigned)x.x; wa[4 * q4 + 1] = (unsigned)x.y;
                    wa[4 * q4 + 2] = (unsigned)x.z; wa[4 * q4 + 3] = (unsigned)x.w;
                    wb[4 * q4] = (unsigned)y.x; wb[4 * q4 + 1] = (unsigned)y.y;
                    wb[4 * q4 + 2] = (unsigned)y.z; wb[4 * q4 + 3] = (unsigned)y.w;
                }
                u16x2 diag = diag0;
                u16x2 f = as16(top.y);
#pragma unroll
                for (int k = 0; k < kChunk; ++k) {
                    // row k's int16 score of each sequence into the two halves
                    const unsigned sel = (k & 1) ? 0x07060302u : 0x05040100u;
                    const i16x2 sk = __builtin_bit_cast(i16x2, __builtin_amdgcn_perm(wb[k >> 1], wa[k >> 1], sel));
                    const u16x2 h = smax3(sadds(diag, sk), E[k], f);
                    const u16x2 hop = subs(h, o2);
                    f = vmax(subs(f, e2), hop);
                    E[k] = vmax(subs(E[k], e2), hop);
                    diag = H[k];
                    H[k] = h;
                    best = vmax(best, h);
                }
                diag0 = as16(top.x);
                if (!last) border[(int64_t)j * 64 + lane] = make_uint2(as32(H[kChunk - 1]), as32(f));
            }
        }

        const unsigned bv = as32(best);
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int32_t idx = a.perm[g.first + 2 * lane + half];
            if (idx >= 0) {
                const unsigned v = half ? (bv >> 16) : (bv & 0xFFFF);
                int32_t *dst = a.scores + (int64_t)wk.q * a.ndb + idx;
                if (v >= kSatLimit) {
                    *dst = -1;
                    const int slot = atomicAdd(a.nredo, 1);
                    if (slot < a.redo_cap) {
                        a.redo[2 * slot] = wk.q;
                        a.redo[2 * slot + 1] = idx;
                    }
                } else {
                    *dst = (int32_t)v;
                }
            }
        }
    }
}

// ---- the pipelined form: W waves share one unit --------------------------
//
// With few queries there are fewer (query, group) units than SIMDs.  Here a
// work-group of W waves takes units from the ticket and cuts each into its
// 32-row chunks; the work-group numbers all chunks of its units in one
// sequence and wave w runs chunks w, w + W, w + 2W, ...  So consecutive
// chunks of a unit run on neighbouring waves, one behind the other, and a
// chunk's bottom row (H, F and the running maximum, per column) reaches the
// next chunk through a ring of kRing columns in LDS between neighbouring
// waves; from the last wave back to the first (one round of chunks later) it
// goes through a per-work-group ring in global memory that holds a whole row
// plus slack, so the last wave never waits for room on it.
//
// Every hand-over is a single-producer single-consumer ring with cumulative
// counters in LDS: the producer publishes how many columns it has written,
// the consumer how many it has read.  Units enter a table of kTable entries:
// the wave that owns a unit's first chunk takes the ticket and publishes the
// entry; it waits before reusing an entry until every wave has moved past
// it.  The consumer reads column j + 1 while computing column j.  Each wait
// is bounded: on expiry the kernel sets the abort flag and every wave leaves.
constexpr int kRing = 8;        // columns per LDS ring
constexpr int kTable = 32;      // unit-table entries
constexpr int kWrapPub = 16;    // the last wave publishes its global-ring progress every 16 columns

__device__ __forceinline__ int lds_get(const int *p)
{
    return __builtin_amdgcn_readfirstlane(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
}

__device__ __forceinline__ void lds_put(int *p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Spin until ok() holds; false when the wait expired or another wave gave up.
template <class Pred>
__device__ __forceinline__ bool pipe_wait(const DbSearchArgs &a, Pred ok)
{
    if (ok()) return true;
    const uint64_t t0 = wall_clock64();
    for (;;) {
        __builtin_amdgcn_s_sleep(1);
        if (ok()) return true;
        if (__builtin_amdgcn_readfirstlane(
                __hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)))
            return false;
        if (wall_clock64() - t0 > a.wait_ticks) {
            __hip_atomic_store(a.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
}

struct PipeRings {
    uint4 *lds_in, *lds_out;       // this wave's LDS rings (input: from wave w-1, output: to wave w+1)
    uint4 *glob;                   // the work-group's global ring (last wave -> first wave)
    int *prod_in, *cons_in;        // counters of the input ring
    int *prod_out, *cons_out;      // counters of the output ring
};

// One 32-row chunk of a unit.  IN_G / OUT_G: the input / output ring is the
// global one.  in_seq / out_seq: columns this wave has read from / written to
// its rings so far; avail / room: cached counter values.
template <bool IN_G, bool OUT_G>
__device__ __forceinline__ bool pipe_chunk(const DbSearchArgs &a, const PipeRings &r, int *pw, int lane, int c,
                                           int nc, const DbWork wk, int &in_seq, int &out_seq, int &avail, int &room)
{
    const int pad = a.asize;
    const int cap_in = IN_G ? a.wrap_cap : kRing;
    const int cap_out = OUT_G ? a.wrap_cap : kRing;
    const DbGroup g = a.groups[wk.g];
    const int64_t q0 = a.qoff[wk.q];
    const int n = (int)(a.qoff[wk.q + 1] - q0);
    const uint8_t *qc = a.qcodes + q0;
    const uint8_t *res = a.res + g.offset;
    const int maxlen = g.maxlen;
    const bool has_in = c > 0, has_out = c < nc - 1;
    const u16x2 o2 = as16((unsigned)a.o | ((unsigned)a.o << 16));
    const u16x2 e2 = as16((unsigned)a.e | ((unsigned)a.e << 16));

    // this chunk's query profile (the previous chunk's reads have all returned)
    if (lane <= pad) {
#pragma unroll
        for (int w = 0; w < 16; ++w) {
            unsigned word = 0;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int row = c * kChunk + 2 * w + b;
                const int qv = row < n ? (int)qc[row] : pad;
                const int s = (qv >= pad || lane >= pad) ? -128 : (int)a.mat[qv * a.asize + lane];
                word |= (unsigned)(s & 0xFFFF) << (16 * b);
            }
            pw[lane * 16 + w] = (int)word;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    u16x2 H[kChunk], E[kChunk];
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
        H[k] = as16(0u);
        E[k] = as16(0u);
    }
    u16x2 diag0 = as16(0u);
    u16x2 best = as16(0u);
    const int in_base = in_seq, out_base = out_seq;
    int islot = in_base % cap_in, oslot = out_base % cap_out;

    auto wait_in = [&](int need) -> bool {
        if (avail >= need) return true;
        const bool ok = pipe_wait(a, [&] {
            avail = lds_get(r.prod_in);
            return avail >= need;
        });
        if (IN_G)
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        else
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
        return ok;
    };
    auto read_in = [&](int slot) -> uint4 {
        return IN_G ? r.glob[(size_t)slot * 64 + lane] : r.lds_in[slot * 64 + lane];
    };

    unsigned cn = *reinterpret_cast<const unsigned short *>(res + 2 * lane);   // (the layout ends in 256 spare bytes)
    uint4 tn = make_uint4(0u, 0u, 0u, 0u);
    if (has_in && maxlen > 0) {   // a group of empty sequences has no columns to hand over
        if (!wait_in(in_base + 1)) return false;
        tn = read_in(islot);
    }
    for (int j = 0; j < maxlen; ++j) {
        const unsigned cab = cn;
        const uint4 top = tn;
        if (j + 1 < maxlen) {
            cn = *reinterpret_cast<const unsigned short *>(res + (int64_t)(j + 1) * 128 + 2 * lane);
            if (has_in) {
                if (!wait_in(in_base + j + 2)) return false;
                islot = islot + 1 == cap_in ? 0 : islot + 1;
                tn = read_in(islot);
            }
        }
        const int ca = (int)(cab & 0xFF), cb = (int)(cab >> 8);
        unsigned wa[16], wb[16];
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
            const int4 x = reinterpret_cast<const int4 *>(pw + ca * 16)[q4];
            const int4 y = reinterpret_cast<const int4 *>(pw + cb * 16)[q4];
            wa[4 * q4] = (unsigned)x.x; wa[4 * q4 + 1] = (unsigned)x.y;
            wa[4 * q4 + 2] = (unsigned)x.z; wa[4 * q4 + 3] = (unsigned)x.w;
            wb[4 * q4] = (unsigned)y.x; wb[4 * q4 + 1] = (unsigned)y.y;
            wb[4 * q4 + 2] = (unsigned)y.z; wb[4 * q4 + 3] = (unsigned)y.w;
        }
        u16x2 diag = diag0;
        u16x2 f = as16(top.y);
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
            const unsigned sel = (k & 1) ? 0x07060302u : 0x05040100u;
            const i16x2 sk = __builtin_bit_cast(i16x2, __builtin_amdgcn_perm(wb[k >> 1], wa[k >> 1], sel));
            const u16x2 h = smax3(sadds(diag, sk), E[k], f);
            const u16x2 hop = subs(h, o2);
            f = vmax(subs(f, e2), hop);
            E[k] = vmax(subs(E[k], e2), hop);
            diag = H[k];
            H[k] = h;
            best = vmax(best, h);
        }
        best = vmax(best, as16(top.z));      // the maximum of the chunks above
        diag0 = as16(top.x);
        if (has_out) {
            const int seq = out_base + j;
            if (seq >= room) {
                int seen = 0;
                if (!pipe_wait(a, [&] {
                        seen = lds_get(r.cons_out);
                        return seq < seen + cap_out;
                    }))
                    return false;
                room = seen + cap_out;
            }
            const uint4 v = make_uint4(as32(H[kChunk - 1]), as32(f), as32(best), 0u);
            if (OUT_G)
                r.glob[(size_t)oslot * 64 + lane] = v;
            else
                r.lds_out[oslot * 64 + lane] = v;
            oslot = oslot + 1 == cap_out ? 0 : oslot + 1;
            if (OUT_G) {
                if ((j % kWrapPub) == kWrapPub - 1 || j == maxlen - 1) {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    lds_put(r.prod_out, seq + 1);
                }
            } else if ((j & 1) || j == maxlen - 1) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
                lds_put(r.prod_out, seq + 1);
            }
        }
        if (has_in && ((j & 1) || j == maxlen - 1)) {
            // the slots up to column j have been read (their values are in use above)
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            lds_put(r.cons_in, in_base + j + 1);
        }
    }
    if (has_in) in_seq += maxlen;
    if (has_out) out_seq += maxlen;

    if (c == nc - 1) {
        const DbGroup gg = g;
        const unsigned bv = as32(best);
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int32_t idx = a.perm[gg.first + 2 * lane + half];
            if (idx >= 0) {
                const unsigned v = half ? (bv >> 16) : (bv & 0xFFFF);
                int32_t *dst = a.scores + (int64_t)wk.q * a.ndb + idx;
                if (v >= kSatLimit) {
                    *dst = -1;
                    const int slot = atomicAdd(a.nredo, 1);
                    if (slot < a.redo_cap) {
                        a.redo[2 * slot] = wk.q;
                        a.redo[2 * slot + 1] = idx;
                    }
                } else {
                    *dst = (int32_t)v;
                }
            }
        }
    }
    return true;
}

// Three waves per SIMD: a chunk's rows, E and H take 64 registers and the
// profile words, ring values and addresses about 70 more, so 168 registers
// per wave hold the column loop without spills (at four waves per SIMD, 128
// registers, the loop reloaded spilled values from scratch every column and
// ran about 5% slower with four waves per unit, 25% with sixteen).  Sixteen
// waves per work-group still force four per SIMD.
template <int W>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(3)))
db_pipe_kernel(DbSearchArgs a)
{
    static_assert(W >= 2, "the pipelined form needs two waves or more");
    __shared__ __align__(16) int prof[W][33 * 16];
    __shared__ __align__(16) uint4 ring[W - 1][kRing * 64];
    __shared__ int prod[W], cons[W], wave_unit[W];
    __shared__ int table[kTable][4];
    __shared__ int npub;

    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (threadIdx.x < W) {
        prod[threadIdx.x] = 0;
        cons[threadIdx.x] = 0;
        wave_unit[threadIdx.x] = 0;
    }
    if (threadIdx.x == 0) npub = 0;
    __syncthreads();

    PipeRings r;
    r.glob = reinterpret_cast<uint4 *>(a.border) + (size_t)blockIdx.x * a.wrap_cap * 64;
    const int inr = w == 0 ? W - 1 : w - 1;
    r.lds_in = w == 0 ? nullptr : ring[w - 1];
    r.lds_out = w == W - 1 ? nullptr : ring[w];
    r.prod_in = prod + inr;
    r.cons_in = cons + inr;
    r.prod_out = prod + w;
    r.cons_out = cons + w;
    int *pw = prof[w];

    int G = w, u = -1, ug0 = 0, unc = 0, uw = 0;
    int in_seq = 0, out_seq = 0, avail = 0;
    int room = w == W - 1 ? a.wrap_cap : kRing;
    bool ok = true;
    for (;;) {
        // find the unit that holds chunk G (entries are published in order)
        while (u < 0 || G >= ug0 + unc) {
            const int nu = u + 1;
            const int start = u < 0 ? 0 : ug0 + unc;
            if (lds_get(&npub) > nu) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
                const int *e = table[nu % kTable];
                uw = __builtin_amdgcn_readfirstlane(e[1]);
                ug0 = __builtin_amdgcn_readfirstlane(e[2]);
                unc = __builtin_amdgcn_readfirstlane(e[3]);
                u = nu;
                lds_put(&wave_unit[w], nu);
                continue;
            }
            if (G == start) {
                // this wave runs the unit's first chunk: it takes the ticket
                const int tv = __builtin_amdgcn_readfirstlane(
                    __hip_atomic_fetch_add(a.ticket, lane == 0 ? 1 : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                int work = -1, nc = 1 << 30;
                const bool stop =
                    tv >= a.nwork ||
                    (a.cancel && __builtin_amdgcn_readfirstlane(
                                     __hip_atomic_load(a.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)));
                if (!stop) {
                    const DbWork wk = a.work[tv];
                    const int len = (int)(a.qoff[wk.q + 1] - a.qoff[wk.q]);
                    work = tv;
                    nc = max(1, (len + kChunk - 1) / kChunk);
                }
                ok = pipe_wait(a, [&] {
                    int m = nu;
                    for (int k = 0; k < W; ++k) m = min(m, lds_get(&wave_unit[k]));
                    return m >= nu - kTable + 1;
                });
                if (!ok) break;
                if (lane == 0) {
                    int *e = table[nu % kTable];
                    e[0] = nu;
                    e[1] = work;
                    e[2] = start;
                    e[3] = nc;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
                lds_put(&npub, nu + 1);
                continue;
            }
            ok = pipe_wait(a, [&] { return lds_get(&npub) > nu; });
            if (!ok) break;
        }
        if (!ok || uw < 0) break;
        const DbWork wk = a.work[uw];
        const int c = G - ug0;
        if (w == 0)
            ok = pipe_chunk<true, false>(a, r, pw, lane, c, unc, wk, in_seq, out_seq, avail, room);
        else if (w == W - 1)
            ok = pipe_chunk<false, true>(a, r, pw, lane, c, unc, wk, in_seq, out_seq, avail, room);
        else
            ok = pipe_chunk<false, false>(a, r, pw, lane, c, unc, wk, in_seq, out_seq, avail, room);
        if (!ok) break;
        G += W;
    }
}

// Top-k of one row segment: each thread keeps its best k of a strided
// subset in a sorted list, then k rounds of a block-wide arg-best pick the
// heads.  Order: score desc, then index asc.
constexpr int kTopMax = 32;
constexpr int kTopThreads = 256;

__device__ __forceinline__ bool better(int32_t s1, int64_t i1, int32_t s2, int64_t i2)
{
    return s1 > s2 || (s1 == s2 && i1 < i2);
}

__global__ void __launch_bounds__(kTopThreads) topk_kernel(const int32_t *scores, const int32_t *cidx, int64_t rowlen,
                                                           int64_t seglen, int32_t nseg, int32_t k,
                                                           int32_t *out_score, int32_t *out_idx, int64_t *final_idx)
{
    __shared__ int32_t sh_s[kTopThreads];
    __shared__ int64_t sh_i[kTopThreads];
    __shared__ int sh_t[kTopThreads];
    const int row = blockIdx.y, seg = blockIdx.x;
    const int64_t b = (int64_t)seg * seglen, e = min(rowlen, b + seglen);
    const int32_t *rs = scores + (int64_t)row * rowlen;
    const int32_t *ri = cidx ? cidx + (int64_t)row * rowlen : nullptr;
    int32_t ls[kTopMax];
    int64_t li[kTopMax];
    int cnt = 0;
    for (int64_t x = b + threadIdx.x; x < e; x += blockDim.x) {
        const int32_t s = rs[x];
        const int64_t id = ri ? (int64_t)ri[x] : x;
        if (id < 0) continue;
        if (cnt < k || better(s, id, ls[cnt - 1], li[cnt - 1])) {
            int p = cnt < k ? cnt++ : k - 1;
            while (p > 0 && better(s, id, ls[p - 1], li[p - 1])) {
                ls[p] = ls[p - 1];
                li[p] = li[p - 1];
                --p;
            }
            ls[p] = s;
            li[p] = id;
        }
    }
    int head = 0;
    for (int r = 0; r < k; ++r) {
        sh_s[threadIdx.x] = head < cnt ? ls[head] : INT32_MIN;
        sh_i[threadIdx.x] = head < cnt ? li[head] : INT64_MAX;
        sh_t[threadIdx.x] = threadIdx.x;
        __syncthreads();
        for (int wdt = kTopThreads / 2; wdt >= 1; wdt >>= 1) {
            if ((int)threadIdx.x < wdt) {
                const int o = threadIdx.x + wdt;
                if (better(sh_s[o], sh_i[o], sh_s[threadIdx.x], sh_i[threadIdx.x])) {
                    sh_s[threadIdx.x] = sh_s[o];
                    sh_i[threadIdx.x] = sh_i[o];
                    sh_t[threadIdx.x] = sh_t[o];
                }
            }
            __syncthreads();
        }
        const int32_t ws = sh_s[0];
        const int64_t wi = sh_i[0];
        const int wt = sh_t[0];
        __syncthreads();
        if ((int)threadIdx.x == wt && head < cnt) ++head;
        if (threadIdx.x == 0) {
            const int64_t o = ((int64_t)row * nseg + seg) * k + r;
            const bool valid = wi != INT64_MAX;
            if (final_idx) {
                final_idx[o] = valid ? wi : -1;
                out_score[o] = valid ? ws : -1;
            } else {
                out_idx[o] = valid ? (int32_t)wi : -1;
                out_score[o] = valid ? ws : -1;
            }
        }
    }
}

__global__ void scatter_kernel(const int64_t *pos, const int32_t *val, int64_t n, int32_t *dst)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[pos[i]] = val[i];
}

// dst[pos[i]] = score of the i-th strip-kernel problem (BestCell: score first)
__global__ void scatter_best_kernel(const int64_t *pos, const int32_t *best, int64_t n, int32_t stride,
                                    int32_t *dst)
{
    const int64_t gs = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gs) dst[pos[i]] = best[i * stride];
}

__global__ void fill_i32_kernel(int32_t *dst, int64_t n, int32_t v)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = v;
}

}  // namespace

hipError_t launch_scatter(const int64_t *pos, const int32_t *val, int64_t n, int32_t *dst, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t g = std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)g), dim3(256), 0, st, pos, val, n, dst);
    return hipGetLastError();
}

hipError_t launch_scatter_best(const int64_t *pos, const int32_t *best, int64_t n, int32_t stride, int32_t *dst,
                               hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t g = std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(scatter_best_kernel, dim3((unsigned)g), dim3(256), 0, st, pos, best, n, stride, dst);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *dst, int64_t n, int32_t v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t g = std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)g), dim3(256), 0, st, dst, n, v);
    return hipGetLastError();
}

hipError_t launch_db_pack(const uint8_t *codes, const int64_t *offs, const int32_t *perm, const DbGroup *groups,
                          int32_t ngroups, uint8_t pad, uint8_t *res, hipStream_t st)
{
    if (ngroups <= 0) return hipSuccess;
    hipLaunchKernelGGL(db_pack_kernel, dim3(ngroups), dim3(256), 0, st, codes, offs, perm, groups, pad, res);
    return hipGetLastError();
}

hipError_t launch_db_search(const DbSearchArgs &a, int waves, int grid, hipStream_t st)
{
    switch (waves) {
    case 1: hipLaunchKernelGGL(db_search_kernel, dim3(grid), dim3(64), 0, st, a); break;
    case 2: hipLaunchKernelGGL(db_pipe_kernel<2>, dim3(grid), dim3(128), 0, st, a); break;
    case 4: hipLaunchKernelGGL(db_pipe_kernel<4>, dim3(grid), dim3(256), 0, st, a); break;
    case 8: hipLaunchKernelGGL(db_pipe_kernel<8>, dim3(grid), dim3(512), 0, st, a); break;
    case 12: hipLaunchKernelGGL(db_pipe_kernel<12>, dim3(grid), dim3(768), 0, st, a); break;
    case 16: hipLaunchKernelGGL(db_pipe_kernel<16>, dim3(grid), dim3(1024), 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int db_search_grid_limit(int device, int waves)
{
    const void *fn = waves == 1   ? reinterpret_cast<const void *>(&db_search_kernel)
                     : waves == 2 ? reinterpret_cast<const void *>(&db_pipe_kernel<2>)
                     : waves == 4 ? reinterpret_cast<const void *>(&db_pipe_kernel<4>)
                     : waves == 8 ? reinterpret_cast<const void *>(&db_pipe_kernel<8>)
                     : waves == 12 ? reinterpret_cast<const void *>(&db_pipe_kernel<12>)
                                   : reinterpret_cast<const void *>(&db_pipe_kernel<16>);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * waves, 0) != hipSuccess || per_cu < 1)
        per_cu = waves == 1 ? 4 : 1;
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return per_cu * 256;
    return per_cu * p.multiProcessorCount;
}

size_t topk_scratch_entries(int32_t nq, int64_t ndb, int32_t k)
{
    const int64_t seglen = 8192;
    const int64_t nseg = (ndb + seglen - 1) / seglen;
    return (size_t)nq * (size_t)(nseg > 0 ? nseg : 1) * (size_t)k;
}

hipError_t launch_topk(const int32_t *scores, int32_t nq, int64_t ndb, int32_t k, int32_t *cand_idx,
                       int32_t *cand_score, int64_t *out_idx, int32_t *out_score, hipStream_t st)
{
    if (nq <= 0 || k <= 0) return hipSuccess;
    if (k > kTopMax) return hipErrorInvalidValue;
    const int64_t seglen = 8192;
    const int32_t nseg = (int32_t)std::max<int64_t>(1, (ndb + seglen - 1) / seglen);
    hipLaunchKernelGGL(topk_kernel, dim3(nseg, nq), dim3(kTopThreads), 0, st, scores, (const int32_t *)nullptr, ndb,
                       seglen, nseg, k, cand_score, cand_idx, (int64_t *)nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t clen = (int64_t)nseg * k;
    hipLaunchKernelGGL(topk_kernel, dim3(1, nq), dim3(kTopThreads), 0, st, cand_score, cand_idx, clen, clen, 1, k,
                       out_score, (int32_t *)nullptr, out_idx);
    return hipGetLastError();
}

}  // namespace swh
