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

hipError_t launch_db_search(const DbSearchArgs &a, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(db_search_kernel, dim3(grid), dim3(64), 0, st, a);
    return hipGetLastError();
}

int db_search_grid_limit(int device)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(&db_search_kernel), 64,
                                                     0) != hipSuccess ||
        per_cu < 1)
        per_cu = 4;
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
