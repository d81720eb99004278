// tb_kernels.hip -- kernels of the reconstruction phase (the paper's SW#
// "reconstruction": the optimal path, found with space-efficient methods).
//
// The traceback is a frontier-seeded divide and conquer over the aligned
// rectangle (global Gotoh DP, no zero clamp).  A split runs a forward pass
// from the subproblem's top frontier to the mid row and a backward pass from
// its end node up to the row below (both on the strip kernel in global mode),
// then the crossing scan below finds the frontier columns an optimal path can
// cross at.  Leaves run the full DP with per-cell tie flags and walk back.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "tb_kernels.h"

namespace swh {

namespace {

constexpr int kDppWaveShr1 = 0x138;   // lane i reads lane i-1 (lane 0: keeps old)

__device__ __forceinline__ int shr1(int old, int src)
{
    return __builtin_amdgcn_update_dpp(old, src, kDppWaveShr1, 0xF, 0xF, false);
}

__global__ void gather_kernel(const GatherDesc *descs, uint8_t pad)
{
    const GatherDesc d = descs[blockIdx.x];
    for (int64_t i = threadIdx.x; i < d.padded; i += blockDim.x) {
        uint8_t v = pad;
        const int64_t k = i - d.first_pad;
        if (k >= 0 && k < d.count) v = d.src[d.start + (int64_t)d.step * k];
        d.dst[i] = v;
    }
}

// Synthetic codes for timing runs: splitmix64 of (seed + position) mod asize;
// the pad code asize beyond n.
__global__ void random_codes_kernel(uint8_t *dst, int64_t n, int64_t padded, int32_t asize, uint64_t seed)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < padded; i += stride) {
        uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        dst[i] = i < n ? (uint8_t)(z % (uint64_t)asize) : (uint8_t)asize;
    }
}

__global__ void border_init_kernel(const BorderInit *descs, int32_t o, int32_t e)
{
    const BorderInit d = descs[blockIdx.x];
    for (int64_t c = threadIdx.x; c < d.padded; c += blockDim.x) {
        Border v{kNeg, kNeg};
        if (c < d.count) {
            if (d.kind == 0) {
                v = d.src[c];
            } else if (d.kind == 1) {
                const int32_t g = c == 0 ? 0 : (int32_t)(-(int64_t)o - (c - 1) * (int64_t)e);
                v = Border{g, g - o};
            } else if (d.kind == 2) {
                v = Border{kNeg, c == 0 ? -o : kNeg};
            } else if (d.kind == 3) {
                if (c == 0) v = Border{d.seed_h, d.seed_f};
            } else {
                v = Border{0, -o};
            }
        }
        d.dst[c] = v;
    }
}

__global__ void __launch_bounds__(256) row_pick_kernel(const Border *row, int64_t count, int32_t target, int32_t mode,
                                                       unsigned long long *out)
{
    unsigned long long best = mode == 0 ? 0ull : ~0ull;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < count; j += stride) {
        const int32_t h = row[j].h;
        if (mode == 0) {
            const unsigned long long key = ((unsigned long long)(uint32_t)(h + (1 << 30)) << 32) |
                                           (unsigned long long)(0xFFFFFFFFu - (uint32_t)j);
            best = key > best ? key : best;
        } else if (j >= 1 && h == target) {
            best = (unsigned long long)j < best ? (unsigned long long)j : best;
        }
    }
    if (mode == 0)
        atomicMax(out, best);
    else
        atomicMin(out, best);
}

__global__ void __launch_bounds__(256) row_pick_multi_kernel(const RowPickDesc *descs, unsigned long long *out)
{
    __shared__ unsigned long long s_best;
    const RowPickDesc d = descs[blockIdx.x];
    const unsigned long long init = d.mode == 0 ? 0ull : ~0ull;
    if (threadIdx.x == 0) s_best = init;
    __syncthreads();
    unsigned long long best = init;
    for (int64_t j = threadIdx.x; j < d.count; j += blockDim.x) {
        const int32_t h = d.row[j].h;
        if (d.mode == 0) {
            const unsigned long long key = ((unsigned long long)(uint32_t)(h + (1 << 30)) << 32) |
                                           (unsigned long long)(0xFFFFFFFFu - (uint32_t)j);
            best = key > best ? key : best;
        } else if (j >= 1 && h == d.target) {
            best = (unsigned long long)j < best ? (unsigned long long)j : best;
        }
    }
    if (d.mode == 0)
        atomicMax(&s_best, best);
    else
        atomicMin(&s_best, best);
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = s_best;
}

// A path from the frontier to the end crosses from mid row r into row r+1
// through exactly one edge: vertical into F(r+1, j) (forward value D(j),
// backward value from F(r+1, j) = D'+o) or diagonal G(r, j-1) -> G(r+1, j).
// The edge is on an optimal path iff forward + edge + backward == V.
__global__ void __launch_bounds__(256) cross_kernel(const CrossDesc *descs, const int8_t *mat, int32_t asize,
                                                    int32_t o, int32_t e, CrossOut *outs)
{
    __shared__ int32_t s_cmin, s_count, s_key;
    const CrossDesc d = descs[blockIdx.x];
    if (threadIdx.x == 0) {
        s_cmin = INT32_MAX;
        s_count = 0;
        s_key = INT32_MAX;
    }
    __syncthreads();
    const int64_t w = d.J - d.L + 1;
    const int arow = *d.arow;
    int cmin = INT32_MAX, count = 0, key = INT32_MAX;
    for (int64_t k = threadIdx.x; k < w; k += blockDim.x) {
        const int64_t j = d.L + k;
        const Border fw = d.fwd[k];
        const Border bw = d.bwd[w - 1 - k];
        if ((int64_t)fw.f + bw.f + o == d.V) {
            cmin = min(cmin, (int)j);
            ++count;
            key = min(key, (int)(j << 1) | 1);
        }
        if (k >= 1 && j >= 1) {
            const int s = mat[arow * asize + d.bpad[j]];
            if ((int64_t)d.fwd[k - 1].h + s + bw.h == d.V) {
                cmin = min(cmin, (int)(j - 1));
                ++count;
                key = min(key, (int)(j << 1));
            }
        }
    }
    if (count) {
        atomicMin(&s_cmin, cmin);
        atomicAdd(&s_count, count);
        atomicMin(&s_key, key);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        CrossOut r;
        r.cmin = s_count ? s_cmin : -1;
        r.count = s_count;
        r.key = s_key;
        r.exit_col = -1;
        r.exit_state = 0;
        r.exit_val = 0;
        r.pad_[0] = r.pad_[1] = 0;
        if (s_count == 1) {
            const int64_t j = s_key >> 1;
            if (s_key & 1) {
                // vertical edge: the walk leaves F(r+1, j) upwards and closes the
                // gap at G(r, j) when that is optimal, else extends into F(r, j)
                const Border fw = d.fwd[j - d.L];
                const bool close = fw.h - o == fw.f;
                r.exit_col = (int32_t)j;
                r.exit_state = close ? 0 : 1;
                r.exit_val = close ? fw.h : fw.f + e;
            } else {
                r.exit_col = (int32_t)(j - 1);
                r.exit_state = 0;
                r.exit_val = d.fwd[j - 1 - d.L].h;
            }
        }
        outs[blockIdx.x] = r;
    }
}

__global__ void __launch_bounds__(256) cut_scan_kernel(const CutDesc *descs, const int8_t *mat, int32_t asize,
                                                       int32_t o, int32_t *counts, int32_t *keys)
{
    __shared__ int32_t s_count, s_key;
    const CutDesc d = descs[blockIdx.y];
    if (threadIdx.x == 0) {
        s_count = 0;
        s_key = INT32_MAX;
    }
    __syncthreads();
    const int8_t *mrow = mat + (int)*d.arow * asize;
    const uint8_t *tc = d.tc;
    const int64_t te = d.te;
    const int32_t S = d.S;
    int count = 0, key = INT32_MAX;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j <= te; j += stride) {
        // the rest of the path after a node in column j uses columns j+1 ..:
        // reverse record of column j+1 (none after the last column)
        const Border rv = (j < te || d.global) ? d.rev[te - j - 1] : Border{0, kNeg};
        if ((int64_t)d.fwd[j].f + rv.f + o == S) {
            ++count;
            key = min(key, (int)(j << 1) | 1);
        }
        const int64_t hd = (j >= 1 || d.global) ? d.fwd[j - 1].h : 0;
        if (hd + mrow[tc[j]] + rv.h == S) {
            ++count;
            key = min(key, (int)(j << 1));
        }
    }
    if (count) {
        atomicAdd(&s_count, count);
        atomicMin(&s_key, key);
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_count) {
        atomicAdd(counts + blockIdx.y, s_count);
        atomicMin(keys + blockIdx.y, s_key);
    }
}

__global__ void cut_resolve_kernel(const CutDesc *descs, int32_t nd, const int32_t *counts, const int32_t *keys,
                                   int32_t o, int32_t e, CutOut *outs)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nd) return;
    const CutDesc d = descs[k];
    CutOut r;
    r.count = counts[k];
    r.key = keys[k];
    r.clean = 0;
    r.col = -1;
    r.state = 0;
    r.val = 0;
    r.seed_h = r.seed_f = kNeg;
    if (r.count == 1) {
        const int j = r.key >> 1;
        if (r.key & 1) {
            const Border fw = d.fwd[j];
            // (global: a vertical crossing in the last column is left
            // unresolved; the path then runs down that column to the corner)
            if (fw.h - o != fw.f && !(d.global && j == d.te)) {
                r.clean = 1;
                r.col = j;
                r.state = 1;
                r.val = fw.f + e;
                r.seed_f = fw.f;
            }
        } else if (j >= 1) {
            const Border fw = d.fwd[j - 1];
            r.clean = 1;
            r.col = j - 1;
            r.state = 0;
            r.val = fw.h;
            r.seed_h = fw.h;
        }
    }
    outs[k] = r;
}

// Small leaves (flags in LDS): one wave per leaf.  Rows are processed 64 at a
// time, lane = row, with a one-column skew per lane; H and the F handed down
// pass between lanes by a DPP shift, and between row groups through a row
// buffer in LDS.  Each cell stores its tie flags:
//   bit 0  H == H(i-1,j-1) + s   bit 1  H == F
//   bit 2  F == H(i-1,j) - o     bit 3  E == H(i,j-1) - o
// Lane 0 then walks back from the end: at H prefer the diagonal, then F,
// then E; inside a gap prefer closing it.
__global__ void __launch_bounds__(64) leaf_kernel(const LeafDesc *descs, const int8_t *mat, int32_t asize, int32_t o,
                                                  int32_t e, LeafOut *outs)
{
    extern __shared__ uint8_t lds[];
    const LeafDesc d = descs[blockIdx.x];
    const int lane = threadIdx.x;
    const int P = d.P, w = d.w;
    int8_t *smat = reinterpret_cast<int8_t *>(lds);                 // 1024 bytes
    Border *row = reinterpret_cast<Border *>(lds + 1024);           // w entries
    uint8_t *fl = lds + 1024 + (size_t)8 * w;                      // P*w tie flags

    __shared__ int32_t s_endv;
    for (int k = lane; k < asize * asize; k += 64) smat[k] = mat[k];
    for (int k = lane; k < w; k += 64) row[k] = d.front[k];
    if (lane == 0) s_endv = kNeg;
    __syncthreads();

    const int nstr = (P + 63) / 64;
    for (int st = 0; st < nstr; ++st) {
        const int i = st * 64 + lane + 1;          // 1-based leaf row
        const bool real = i <= P;
        const int qcode = real ? d.arows[i - 1] : 0;
        int hprev = kNeg, E = kNeg, hup_prev = kNeg, hbot = kNeg, fbot = kNeg;
        for (int t = 0; t < w + 63; ++t) {
            const int c = t - lane;
            const Border in = t < w ? row[t] : Border{kNeg, kNeg};
            const int hup = shr1(in.h, hbot);
            const int fin = shr1(in.f, fbot);
            const bool valid = real && c >= 0 && c < w;
            int h = kNeg, fdown = kNeg, En = kNeg;
            if (valid) {
                const int code = d.bcols[c];
                const int s = code >= asize ? kNeg : (int)smat[qcode * asize + code];
                const int dg = c == 0 ? kNeg : hup_prev;
                const int t1 = dg + s;
                h = max(t1, max(E, fin));
                const int flag = (h == t1 ? 1 : 0) | (h == fin ? 2 : 0) | (fin == hup - o ? 4 : 0) |
                                 (E == hprev - o ? 8 : 0);
                fl[(i - 1) * w + c] = (uint8_t)flag;
                fdown = max(fin - e, h - o);
                En = max(E - e, h - o);
                if (i == P && c == w - 1) s_endv = d.end_state ? fin : h;
            }
            hbot = h;
            fbot = fdown;
            hprev = h;
            E = En;
            hup_prev = hup;
            if (lane == 63 && valid) row[c] = Border{h, fdown};
        }
        __syncthreads();
    }

    if (lane == 0) {
        int i = P, c = w - 1, state = d.end_state, n = 0, err = 0;
        while (i > 0) {
            if (c < 0 || n >= d.ops_cap) { err = 1; break; }
            const int f = fl[(i - 1) * w + c];
            if (state == 0) {
                if (f & 1) { d.ops[n++] = 'M'; --i; --c; }
                else state = (f & 2) ? 1 : 2;
            } else if (state == 1) {
                d.ops[n++] = 'I';
                if (f & 4) state = 0;
                --i;
            } else {
                d.ops[n++] = 'D';
                if (f & 8) state = 0;
                --c;
            }
        }
        if (c < 0 || state == 2) err = err ? err : 2;
        if (s_endv != d.V) err = 3;
        LeafOut r;
        r.nops = n;
        r.exit_col = c;
        r.exit_state = state;
        r.exit_val = (!err && c >= 0) ? (state == 0 ? d.front[c].h : d.front[c].f + e) : 0;
        r.err = err;
        r.pad_[0] = r.pad_[1] = r.pad_[2] = 0;
        outs[blockIdx.x] = r;
    }
}

// Large leaves (flags in global memory): one wave per leaf, kLeafR rows per
// lane (64 kLeafR rows per group), the strip kernel's layout: the lane's rows
// in registers, a one-column skew per lane, the row above handed over by a
// DPP shift, a per-lane int8 score profile of its rows in LDS.  The four tie
// flags of each cell (as in leaf_kernel) take a nibble; the lane's kLeafR
// cells of one step make one dword, and the 64 dwords of a step one
// coalesced store at flags[(group * (w + 63) + step) * 64 + lane].  Lane 0
// then walks back as in leaf_kernel.
__device__ __forceinline__ uint32_t big_flag(const uint32_t *fl, int w, int64_t r, int64_t c)
{
    constexpr int64_t G = 64 * kLeafR;
    const int64_t g = r / G, lr = r - g * G, ln = lr / kLeafR, k = lr - ln * kLeafR;
    return (fl[(g * (w + 63) + c + ln) * 64 + ln] >> (4 * k)) & 15u;
}

template <bool CAPTURE>
__device__ __forceinline__ void big_step(int (&hp)[kLeafR], int (&E)[kLeafR], const int (&sc)[kLeafR / 4], int dg,
                                         int hup, int &f, int o, int e, uint32_t &flags, int kstar, int end_state,
                                         int32_t *endv)
{
    int habove = hup;
    flags = 0;
#pragma unroll
    for (int k = 0; k < kLeafR; ++k) {
        const int t1 = dg + (int)(signed char)(sc[k >> 2] >> (8 * (k & 3)));
        const int h = max(max(t1, E[k]), f);
        const uint32_t fb = (h == t1 ? 1u : 0u) | (h == f ? 2u : 0u) | (f == habove - o ? 4u : 0u) |
                            (E[k] == hp[k] - o ? 8u : 0u);
        flags |= fb << (4 * k);
        if (CAPTURE && k == kstar) *endv = end_state ? f : h;
        const int hop = h - o;
        const int fn = max(f - e, hop);
        E[k] = max(E[k] - e, hop);
        dg = hp[k];
        hp[k] = h;
        habove = h;
        f = fn;
    }
}

__global__ void __launch_bounds__(64) leaf_big_kernel(const LeafDesc *descs, const int8_t *mat, int32_t asize,
                                                      int32_t o, int32_t e, LeafOut *outs)
{
    extern __shared__ uint8_t lds[];
    constexpr int R = kLeafR, W = kLeafR / 4;
    const LeafDesc d = descs[blockIdx.x];
    const int lane = threadIdx.x;
    const int P = d.P, w = d.w;
    const int A1 = asize + 1;
    int8_t *smat = reinterpret_cast<int8_t *>(lds);                                  // 1024 bytes
    int *prof = reinterpret_cast<int *>(lds + 1024);                                  // A1 * 64 * W words
    Border *row = reinterpret_cast<Border *>(lds + 1024 + (size_t)A1 * 64 * W * 4);   // w entries
    uint8_t *bc = reinterpret_cast<uint8_t *>(row + w);                               // w column codes
    uint32_t *fl = reinterpret_cast<uint32_t *>(d.gflags);
    __shared__ int32_t s_endv;
    for (int k = lane; k < asize * asize; k += 64) smat[k] = mat[k];
    for (int k = lane; k < w; k += 64) {
        row[k] = d.front[k];
        bc[k] = d.bcols[k];
    }
    if (lane == 0) s_endv = kNeg;
    __syncthreads();

    const int ngroups = (P + 64 * R - 1) / (64 * R);
    // the lane and row (within the lane) of the end cell (P, w-1)
    const int gend = (P - 1) / (64 * R), lend = ((P - 1) - gend * 64 * R) / R, kend = (P - 1) - gend * 64 * R - lend * R;
    for (int g = 0; g < ngroups; ++g) {
        const int r0 = g * 64 * R + lane * R;   // the lane's first row (from 0)
        for (int cd = 0; cd < A1; ++cd)
#pragma unroll
            for (int wd = 0; wd < W; ++wd) {
                uint32_t word = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int r = r0 + 4 * wd + b;
                    const int q = r < P ? (int)d.arows[r] : asize;
                    const int v = (q >= asize || cd >= asize) ? -128 : (int)smat[q * asize + cd];
                    word |= (uint32_t)(v & 0xFF) << (8 * b);
                }
                prof[(cd * 64 + lane) * W + wd] = (int)word;
            }
        int hp[R], E[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            hp[k] = kNeg;
            E[k] = kNeg;
        }
        int hup_prev = kNeg, hbot = kNeg, fbot = kNeg;
        uint32_t *flg = fl + (size_t)g * (w + 63) * 64 + lane;
        const bool rows_real = r0 < P;
        const int tcap = g == gend ? w - 1 + lend : -1;   // the step that holds the end cell
        for (int t = 0; t < w + 63; ++t) {
            const int c = t - lane;
            const Border in = t < w ? row[t] : Border{kNeg, kNeg};
            const int hup = shr1(in.h, hbot);
            int f = shr1(in.f, fbot);
            if (rows_real && c >= 0 && c < w) {
                const int code = bc[c];
                int sc[W];
                const int *pp = prof + (code * 64 + lane) * W;
#pragma unroll
                for (int wd = 0; wd < W; ++wd) sc[wd] = pp[wd];
                const int dg = c == 0 ? kNeg : hup_prev;
                uint32_t flags;
                if (t == tcap)
                    big_step<true>(hp, E, sc, dg, hup, f, o, e, flags, lane == lend ? kend : -1, d.end_state,
                                   &s_endv);
                else
                    big_step<false>(hp, E, sc, dg, hup, f, o, e, flags, -1, 0, nullptr);
                flg[(size_t)t * 64] = flags;
                hbot = hp[R - 1];
                fbot = f;
                if (lane == 63) row[c] = Border{hbot, fbot};
            }
            hup_prev = hup;
        }
        __syncthreads();
    }

    if (lane == 0) {
        int i = P, c = w - 1, state = d.end_state, n = 0, err = 0;
        while (i > 0) {
            if (c < 0 || n >= d.ops_cap) { err = 1; break; }
            const uint32_t f = big_flag(fl, w, i - 1, c);
            if (state == 0) {
                if (f & 1) { d.ops[n++] = 'M'; --i; --c; }
                else state = (f & 2) ? 1 : 2;
            } else if (state == 1) {
                d.ops[n++] = 'I';
                if (f & 4) state = 0;
                --i;
            } else {
                d.ops[n++] = 'D';
                if (f & 8) state = 0;
                --c;
            }
        }
        if (c < 0 || state == 2) err = err ? err : 2;
        if (s_endv != d.V) err = 3;
        LeafOut r;
        r.nops = n;
        r.exit_col = c;
        r.exit_state = state;
        r.exit_val = (!err && c >= 0) ? (state == 0 ? d.front[c].h : d.front[c].f + e) : 0;
        r.err = err;
        r.pad_[0] = r.pad_[1] = r.pad_[2] = 0;
        outs[blockIdx.x] = r;
    }
}

}  // namespace

hipError_t launch_random_codes(uint8_t *dst, int64_t n, int64_t padded, int32_t asize, uint64_t seed, hipStream_t st)
{
    if (padded <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((padded + 255) / 256, 65536);
    hipLaunchKernelGGL(random_codes_kernel, dim3((unsigned)blocks), dim3(256), 0, st, dst, n, padded, asize, seed);
    return hipGetLastError();
}

hipError_t launch_row_pick(const Border *row, int64_t count, int32_t target, int32_t mode, uint64_t *out,
                           hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((count + 255) / 256, 1024));
    hipLaunchKernelGGL(row_pick_kernel, dim3((unsigned)blocks), dim3(256), 0, st, row, count, target, mode,
                       reinterpret_cast<unsigned long long *>(out));
    return hipGetLastError();
}

hipError_t launch_row_pick_multi(const RowPickDesc *d, int32_t nd, uint64_t *out, hipStream_t st)
{
    if (nd <= 0) return hipSuccess;
    hipLaunchKernelGGL(row_pick_multi_kernel, dim3((unsigned)nd), dim3(256), 0, st, d,
                       reinterpret_cast<unsigned long long *>(out));
    return hipGetLastError();
}

hipError_t launch_gather(const GatherDesc *d, int32_t nd, uint8_t pad, hipStream_t st)
{
    if (nd <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_kernel, dim3(nd), dim3(256), 0, st, d, pad);
    return hipGetLastError();
}

hipError_t launch_border_init(const BorderInit *d, int32_t nd, int32_t o, int32_t e, hipStream_t st)
{
    if (nd <= 0) return hipSuccess;
    hipLaunchKernelGGL(border_init_kernel, dim3(nd), dim3(256), 0, st, d, o, e);
    return hipGetLastError();
}


hipError_t launch_cross(const CrossDesc *d, int32_t nd, const int8_t *mat, int32_t asize, int32_t o, int32_t e,
                        CrossOut *out, hipStream_t st)
{
    if (nd <= 0) return hipSuccess;
    hipLaunchKernelGGL(cross_kernel, dim3(nd), dim3(256), 0, st, d, mat, asize, o, e, out);
    return hipGetLastError();
}

hipError_t launch_cut_scan(const CutDesc *d, int32_t nd, int64_t max_te, const int8_t *mat, int32_t asize,
                           int32_t o, int32_t *counts, int32_t *keys, hipStream_t st)
{
    if (nd <= 0 || max_te < 0) return hipSuccess;
    // about 16 K columns per workgroup, enough workgroups per cut to fill the GPU
    const int64_t chunks = std::max<int64_t>(1, std::min<int64_t>((max_te + 1 + 16383) / 16384, 1024));
    for (int32_t k0 = 0; k0 < nd; k0 += 65535) {   // grid y is at most 65,535
        const int32_t n = std::min<int32_t>(nd - k0, 65535);
        hipLaunchKernelGGL(cut_scan_kernel, dim3((unsigned)chunks, (unsigned)n), dim3(256), 0, st, d + k0, mat, asize,
                           o, counts + k0, keys + k0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_cut_resolve(const CutDesc *d, int32_t nd, const int32_t *counts, const int32_t *keys, int32_t o,
                              int32_t e, CutOut *out, hipStream_t st)
{
    if (nd <= 0) return hipSuccess;
    hipLaunchKernelGGL(cut_resolve_kernel, dim3((unsigned)((nd + 255) / 256)), dim3(256), 0, st, d, nd, counts, keys,
                       o, e, out);
    return hipGetLastError();
}

hipError_t launch_leaf(const LeafDesc *d, int32_t nd, const int8_t *mat, int32_t asize, int32_t o, int32_t e,
                       size_t lds_bytes, LeafOut *out, hipStream_t st)
{
    if (nd <= 0) return hipSuccess;
    hipLaunchKernelGGL(leaf_kernel, dim3(nd), dim3(64), lds_bytes, st, d, mat, asize, o, e, out);
    return hipGetLastError();
}

hipError_t launch_leaf_big(const LeafDesc *d, int32_t nd, const int8_t *mat, int32_t asize, int32_t o, int32_t e,
                           int32_t max_w, LeafOut *out, hipStream_t st)
{
    if (nd <= 0) return hipSuccess;
    hipLaunchKernelGGL(leaf_big_kernel, dim3(nd), dim3(64), leaf_big_lds(asize, max_w), st, d, mat, asize, o, e, out);
    return hipGetLastError();
}

}  // namespace swh
