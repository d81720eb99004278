// mlp_kernels.hip -- the learned prefilter on CDNA4.
//
// The network's matrix products are dense contractions, so they run on the
// matrix cores: v_mfma_f32_16x16x32_bf16 (bfloat16 operands, float32
// accumulation).  Lane l of a wave supplies A[m = l % 16][k = 8 (l / 16) ..
// +7] and B[k = 8 (l / 16) .. +7][n = l % 16] and receives
// D[m = 4 (l / 16) + r][n = l % 16], r = 0..3.  Everything else (features,
// reductions, Adam, selection) is plain VALU code laid out for coalescing.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mlp_kernels.h"

namespace swh {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);   // nearest, ties to even (finite inputs)
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ bf16x8 as_bf(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ uint32_t order_key(float v)
{
    const uint32_t u = __float_as_uint(v);
    return (u >> 31) ? ~u : (u | 0x80000000u);
}

// ------------------------------------------------------------------ features

__global__ void __launch_bounds__(256) dipeptide_kernel(const uint8_t *codes, const int64_t *off, int64_t nseq,
                                                        const int32_t *dst_row, int32_t *counts, float *freq32,
                                                        uint16_t *freqbf, int32_t *lens)
{
    __shared__ int32_t c[4][kNDip];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t s = (int64_t)blockIdx.x * 4 + w;
    for (int k = lane; k < kNDip; k += 64) c[w][k] = 0;
    __syncthreads();
    int64_t L = 0;
    if (s < nseq) {
        const int64_t o = off[s];
        L = off[s + 1] - o;
        for (int64_t i = lane; i + 1 < L; i += 64) {
            const int a = codes[o + i], b = codes[o + i + 1];
            if (a < kNStd && b < kNStd) atomicAdd(&c[w][kNStd * a + b], 1);
        }
    }
    __syncthreads();
    if (s >= nseq) return;
    const int64_t r = dst_row ? dst_row[s] : s;
    if (r < 0) return;
    for (int k = lane; k < kKPad; k += 64) {
        const int32_t v = k < kNDip ? c[w][k] : 0;
        const float f = L >= 2 ? (float)v / (float)(L - 1) : 0.0f;
        if (k < kNDip) {
            if (counts) counts[r * kNDip + k] = v;
            if (freq32) freq32[r * kNDip + k] = f;
        }
        if (freqbf) freqbf[r * kKPad + k] = k < kNDip ? f2bf(f) : 0;
    }
    if (lens && lane == 0) lens[r] = (int32_t)L;
}

__device__ __forceinline__ float log_len(int32_t a, int32_t b) { return logf((float)max(1, min(a, b))); }

// One block per chunk of pairs, thread k < 401 accumulates feature k in float64.
__global__ void __launch_bounds__(512) pair_stats_kernel(const float *f, const int32_t *lens, const int32_t *rows,
                                                         const int32_t *cols, int64_t npairs, int64_t chunk,
                                                         double *partial)
{
    const int k = threadIdx.x;
    if (k >= kNIn) return;
    const int64_t p0 = (int64_t)blockIdx.x * chunk, p1 = min(npairs, p0 + chunk);
    double s = 0.0, ss = 0.0;
    for (int64_t p = p0; p < p1; ++p) {
        const int32_t r = rows[p], c = cols[p];
        const float x = k < kNDip ? f[(int64_t)r * kNDip + k] * f[(int64_t)c * kNDip + k] : log_len(lens[r], lens[c]);
        s += x;
        ss += (double)x * x;
    }
    partial[(int64_t)blockIdx.x * 2 * kNIn + k] = s;
    partial[(int64_t)blockIdx.x * 2 * kNIn + kNIn + k] = ss;
}

__global__ void pair_stats_final_kernel(const double *partial, int nblocks, double *sum, double *sumsq)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kNIn) return;
    double s = 0.0, ss = 0.0;
    for (int b = 0; b < nblocks; ++b) {
        s += partial[(int64_t)b * 2 * kNIn + k];
        ss += partial[(int64_t)b * 2 * kNIn + kNIn + k];
    }
    sum[k] = s;
    sumsq[k] = ss;
}

__global__ void __launch_bounds__(448) pair_z_kernel(const float *f, const int32_t *lens, const int32_t *rows,
                                                     const int32_t *cols, const float *mu, const float *sd,
                                                     uint16_t *Z)
{
    const int64_t p = blockIdx.x;
    const int k = threadIdx.x;
    if (k >= kKPad) return;
    const int32_t r = rows[p], c = cols[p];
    float z = 0.0f;
    if (k < kNIn) {
        const float x = k < kNDip ? f[(int64_t)r * kNDip + k] * f[(int64_t)c * kNDip + k] : log_len(lens[r], lens[c]);
        z = (x - mu[k]) / sd[k];
    }
    Z[p * kKPad + k] = f2bf(z);
}

__global__ void labels_kernel(const int32_t *s, int64_t n, float *y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = log1pf((float)s[i]);
}

__global__ void __launch_bounds__(448) z_to_bf16_kernel(const float *z, uint16_t *Z)
{
    const int64_t r = blockIdx.x;
    const int k = threadIdx.x;
    if (k < kKPad) Z[r * kKPad + k] = k < kNIn ? f2bf(z[r * kNIn + k]) : 0;
}

__global__ void __launch_bounds__(64) gather_rows_kernel(const uint16_t *Z, const float *y, const int32_t *idx,
                                                         const int32_t *ctr, uint16_t *Xb, float *yb)
{
    const int i = blockIdx.x;
    const int64_t src = idx[(ctr ? (int64_t)ctr[0] * gridDim.x : 0) + i];
    const u32x4 *s = (const u32x4 *)(Z + src * kKPad);
    u32x4 *d = (u32x4 *)(Xb + (int64_t)i * kKPad);
    for (int t = threadIdx.x; t < kKPad / 8; t += 64) d[t] = s[t];
    if (threadIdx.x == 0) yb[i] = y[src];
}

// ------------------------------------------------------------------ GEMM

// 64 x 64 output tile per workgroup, four waves of 32 x 32 (2 x 2 MFMA
// tiles), K in steps of 32 staged through LDS with k contiguous per row.
template <bool AT, bool BT>
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[64][40];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[64][40];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const u32x4 zero = {0u, 0u, 0u, 0u};
    const int kslice = g.K / gridDim.z;   // a multiple of 32 (checked by the launcher)
    const int kbeg = blockIdx.z * kslice, kend = kbeg + kslice;
    for (int k0 = kbeg; k0 < kend; k0 += 32) {
        if (!AT) {
            const int m = tid >> 2, kk = (tid & 3) * 8;
            u32x4 v = zero;
            if (m0 + m < g.mload) v = *(const u32x4 *)(g.A + (int64_t)(m0 + m) * g.lda + k0 + kk);
            *(u32x4 *)&As[m][kk] = v;
        } else {
            const int kk = tid >> 3, m = (tid & 7) * 8;
            u32x4 v = zero;
            if (m0 + m < g.mload) v = *(const u32x4 *)(g.A + (int64_t)(k0 + kk) * g.lda + m0 + m);
            const uint16_t *e = (const uint16_t *)&v;
            for (int i = 0; i < 8; ++i) As[m + i][kk] = e[i];
        }
        if (BT) {
            const int n = tid >> 2, kk = (tid & 3) * 8;
            u32x4 v = zero;
            if (n0 + n < g.nload) v = *(const u32x4 *)(g.B + (int64_t)(n0 + n) * g.ldb + k0 + kk);
            *(u32x4 *)&Bs[n][kk] = v;
        } else {
            const int kk = tid >> 3, n = (tid & 7) * 8;
            u32x4 v = zero;
            if (n0 + n < g.nload) v = *(const u32x4 *)(g.B + (int64_t)(k0 + kk) * g.ldb + n0 + n);
            const uint16_t *e = (const uint16_t *)&v;
            for (int i = 0; i < 8; ++i) Bs[n + i][kk] = e[i];
        }
        __syncthreads();
        bf16x8 a[2], b[2];
        for (int i = 0; i < 2; ++i) a[i] = as_bf(*(const u32x4 *)&As[wm + 16 * i + (lane & 15)][8 * (lane >> 4)]);
        for (int j = 0; j < 2; ++j) b[j] = as_bf(*(const u32x4 *)&Bs[wn + 16 * j + (lane & 15)][8 * (lane >> 4)]);
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) acc[i][j] = mfma(a[i], b[j], acc[i][j]);
        __syncthreads();
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
                const int n = n0 + wn + 16 * j + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                const float c = acc[i][j][r];
                const int64_t o = (int64_t)m * g.ldc + n;
                if (gridDim.z > 1) {
                    g.partial[((int64_t)blockIdx.z * g.M + m) * g.N + n] = c;
                } else if (g.epi == kEpiF32) {
                    g.out32[o] = c;
                } else if (g.epi == kEpiBiasReluBf) {
                    g.outbf[o] = f2bf(fmaxf(c + g.bias[n], 0.0f));
                } else if (g.epi == kEpiBiasReluF32) {
                    g.out32[o] = fmaxf(c + g.bias[n], 0.0f);
                } else {
                    const float v = bf2f(g.mask[o]) > 0.0f ? c : 0.0f;
                    g.out32[o] = v;
                    g.outbf[o] = f2bf(v);
                }
            }
}

__global__ void splitk_reduce_kernel(const float *partial, int splits, int M, int N, float *out, int64_t ldc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)M * N) return;
    float acc = 0.0f;
    for (int s = 0; s < splits; ++s) acc += partial[(int64_t)s * M * N + i];
    out[(i / N) * ldc + i % N] = acc;
}

// ------------------------------------------------------------------ training reductions

__global__ void __launch_bounds__(256) head_kernel(const float *H2, const float *y, const float *theta, int B,
                                                   float *d, float *dz2, uint16_t *dz2bf, double *loss)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int b = blockIdx.x * 4 + w;
    if (b >= B) return;
    const float *h = H2 + (int64_t)b * kNH;
    const float *w3 = theta + kOffW3;
    float hv[4], s = 0.0f;
    for (int t = 0; t < 4; ++t) {
        hv[t] = h[4 * lane + t];
        s += hv[t] * w3[4 * lane + t];
    }
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    const float r = s + theta[kOffB3] - y[b];
    const float dd = 2.0f * r / (float)B;
    for (int t = 0; t < 4; ++t) {
        const float v = hv[t] > 0.0f ? dd * w3[4 * lane + t] : 0.0f;
        dz2[(int64_t)b * kNH + 4 * lane + t] = v;
        dz2bf[(int64_t)b * kNH + 4 * lane + t] = f2bf(v);
    }
    if (lane == 0) {
        d[b] = dd;
        atomicAdd(loss, (double)r * (double)r);
    }
}

constexpr int kColSlices = 32;

__global__ void colsum_kernel(const float *X, int64_t ldx, int rows, int cols, const float *scale, float *partial)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= cols) return;
    const int s = blockIdx.y;
    const int r0 = (int)((int64_t)rows * s / kColSlices), r1 = (int)((int64_t)rows * (s + 1) / kColSlices);
    float acc = 0.0f;
    for (int r = r0; r < r1; ++r) acc += X[(int64_t)r * ldx + n] * (scale ? scale[r] : 1.0f);
    partial[(int64_t)s * cols + n] = acc;
}

__global__ void colsum_final_kernel(const float *partial, int cols, float *out)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= cols) return;
    float acc = 0.0f;
    for (int s = 0; s < kColSlices; ++s) acc += partial[(int64_t)s * cols + n];
    out[n] = acc;
}

__global__ void adam_kernel(float *theta, float *m, float *v, const float *g, int64_t n, float lr, float b1, float b2,
                            float eps, float bc1, float bc2, const int32_t *ctr)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (ctr) {   // step number from the device counter (graph replays)
        const float t = (float)(ctr[1] + 1);
        bc1 = 1.0f - powf(b1, t);
        bc2 = 1.0f - powf(b2, t);
    }
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

__global__ void pack_weights_kernel(const float *theta, uint16_t *W1bf, uint16_t *W2bf)
{
    const int n = blockIdx.x;   // 256 rows
    for (int k = threadIdx.x; k < kKPad; k += blockDim.x)
        W1bf[n * kKPad + k] = k < kNIn ? f2bf(theta[kOffW1 + (int64_t)n * kNIn + k]) : 0;
    for (int k = threadIdx.x; k < kNH; k += blockDim.x) W2bf[n * kNH + k] = f2bf(theta[kOffW2 + (int64_t)n * kNH + k]);
}

// ------------------------------------------------------------------ inference

__global__ void __launch_bounds__(256) fold_const_kernel(const float *theta, const float *mu, const float *sd,
                                                         float *cvec, float *w1x)
{
    __shared__ float part[256];
    const int n = blockIdx.x;
    float acc = 0.0f;
    for (int k = threadIdx.x; k < kNDip; k += 256) acc += theta[kOffW1 + (int64_t)n * kNIn + k] * (mu[k] / sd[k]);
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cvec[n] = theta[kOffB1 + n] - part[0];
        w1x[n] = theta[kOffW1 + (int64_t)n * kNIn + kNDip] / sd[kNDip];
    }
}

__global__ void __launch_bounds__(448) fold_query_kernel(const float *theta, const float *fq, const float *sd,
                                                         uint16_t *Aq)
{
    const int q = blockIdx.y, n = blockIdx.x, k = threadIdx.x;
    if (k >= kKPad) return;
    float v = 0.0f;
    if (k < kNDip) v = theta[kOffW1 + (int64_t)n * kNIn + k] * fq[(int64_t)q * kNDip + k] / sd[k];
    Aq[((int64_t)q * kNH + n) * kKPad + k] = f2bf(v);
}

// 64 database rows x one query per workgroup; wave w owns hidden units
// [64 w, 64 w + 64) of both layers.  Layer-1 activations go through LDS.
__global__ void __launch_bounds__(256) infer_kernel(InferArgs a)
{
    __shared__ __attribute__((aligned(16))) uint16_t H1[64][kNH + 8];
    __shared__ float part[4][64];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int64_t row0 = (int64_t)blockIdx.x * 64;
    const int q = blockIdx.y;
    const int li = lane & 15, lk = 8 * (lane >> 4);
    const uint16_t *Aq = a.Aq + (int64_t)q * kNH * kKPad;

    f32x4 acc[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const uint16_t *frow[4];
    for (int i = 0; i < 4; ++i) {
        const int64_t r = min(row0 + 16 * i + li, a.nrows - 1);
        frow[i] = a.F + r * kKPad + lk;
    }
    const uint16_t *arow[4];
    for (int j = 0; j < 4; ++j) arow[j] = Aq + (int64_t)(64 * w + 16 * j + li) * kKPad + lk;
    for (int kk = 0; kk < kKPad; kk += 32) {
        bf16x8 fa[4], fb[4];
        for (int i = 0; i < 4; ++i) fa[i] = as_bf(*(const u32x4 *)(frow[i] + kk));
        for (int j = 0; j < 4; ++j) fb[j] = as_bf(*(const u32x4 *)(arow[j] + kk));
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) acc[i][j] = mfma(fa[i], fb[j], acc[i][j]);
    }
    const int32_t Lq = a.qlen[q];
    for (int i = 0; i < 4; ++i)
        for (int r = 0; r < 4; ++r) {
            const int lr = 16 * i + 4 * (lane >> 4) + r;
            const int64_t row = min(row0 + lr, a.nrows - 1);
            const float x400 = log_len(Lq, a.row_len[row]) - a.mu400;   // w1x already holds the 1 / sd
            for (int j = 0; j < 4; ++j) {
                const int n = 64 * w + 16 * j + li;
                const float z = acc[i][j][r] + a.cvec[n] + a.w1x[n] * x400;
                H1[lr][n] = f2bf(fmaxf(z, 0.0f));
            }
        }
    __syncthreads();

    const float *b2 = a.theta + kOffB2;
    const float *w3 = a.theta + kOffW3;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const uint16_t *wrow[4];
    for (int j = 0; j < 4; ++j) wrow[j] = a.W2bf + (int64_t)(64 * w + 16 * j + li) * kNH + lk;
    for (int kk = 0; kk < kNH; kk += 32) {
        bf16x8 ha[4], wb[4];
        for (int i = 0; i < 4; ++i) ha[i] = as_bf(*(const u32x4 *)&H1[16 * i + li][kk + lk]);
        for (int j = 0; j < 4; ++j) wb[j] = as_bf(*(const u32x4 *)(wrow[j] + kk));
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) acc[i][j] = mfma(ha[i], wb[j], acc[i][j]);
    }
    for (int i = 0; i < 4; ++i)
        for (int r = 0; r < 4; ++r) {
            float s = 0.0f;
            for (int j = 0; j < 4; ++j) {
                const int n = 64 * w + 16 * j + li;
                s += fmaxf(acc[i][j][r] + b2[n], 0.0f) * w3[n];
            }
            for (int o = 8; o >= 1; o >>= 1) s += __shfl_xor(s, o);
            if (li == 0) part[w][16 * i + 4 * (lane >> 4) + r] = s;
        }
    __syncthreads();
    if (tid < 64) {
        const int64_t row = row0 + tid;
        if (row < a.nrows) {
            const float y = a.theta[kOffB3] + part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
            a.pred[(int64_t)q * a.nrows + row] = a.row_db[row] >= 0 ? y : -INFINITY;
        }
    }
}

// All queries over 128 database rows per workgroup.  The rows' frequency tile
// is staged in LDS once (108.5 KB) and serves every query, so the feature
// matrix is read from memory once per search instead of once per query.  Both
// layers are computed transposed -- hidden (or output) units along the MFMA's
// M dimension, database rows along N -- so that a lane's four accumulator
// values are four consecutive units of one row: the layer-1 epilogue stores
// them as one 8-byte LDS write, and its length term is a single per-row value.
// The hidden layer is produced in two halves of 128 units (34 KB of LDS each
// time); layer 2 accumulates over both halves.  Wave w owns hidden units
// [128 h + 32 w, +32) of half h and output units [64 w, +64).
constexpr int kInferRows = 128;
constexpr int kFStride = kKPad + 8;   // bf16 per LDS row of the F tile (rows stay 16-byte aligned)
constexpr int kHalf = kNH / 2;        // hidden units per half
constexpr int kH2Stride = kHalf + 8;  // bf16 per LDS row of a half of the activations
constexpr size_t kInferLds = (size_t)kInferRows * (kFStride + kH2Stride) * 2;

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// two floats to two bfloat16 (nearest, ties to even: one v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi)
{
    const bf16x2 v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, v);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) infer_all_kernel(InferArgs a)
{
    extern __shared__ __attribute__((aligned(16))) uint16_t sm[];
    uint16_t *Ft = sm;                                  // [rows][kFStride]
    uint16_t *Hh = sm + kInferRows * kFStride;          // [rows][kH2Stride]
    __shared__ float rowlog[kInferRows];
    __shared__ float part[4][kInferRows];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lg = lane >> 4, lk = 8 * lg;
    const int64_t row0 = (int64_t)blockIdx.x * kInferRows;
    for (int c = tid; c < kInferRows * (kKPad / 8); c += 256) {
        const int r = c / (kKPad / 8), k8 = c - r * (kKPad / 8);
        const int64_t row = min(row0 + r, a.nrows - 1);
        *(u32x4 *)&Ft[r * kFStride + 8 * k8] = *(const u32x4 *)(a.F + row * kKPad + 8 * k8);
    }
    // ln(max(1, min(Lq, L))) = min(ln max(1, Lq), ln max(1, L)): the row's half here
    if (tid < kInferRows) rowlog[tid] = logf((float)max(1, a.row_len[min(row0 + tid, a.nrows - 1)]));
    __syncthreads();

    const float *b2 = a.theta + kOffB2;
    const float *w3 = a.theta + kOffW3;
    float b2v[4][4], w3v[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = 64 * w + 16 * i + 4 * lg + r;
            b2v[i][r] = b2[m];
            w3v[i][r] = w3[m];
        }
    const float b3 = a.theta[kOffB3];

    for (int q = 0; q < a.nq; ++q) {
        const uint16_t *Aq = a.Aq + (int64_t)q * kNH * kKPad;
        const float lq = logf((float)max(1, a.qlen[q]));
        f32x4 acc2[4][8];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j) acc2[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

        for (int h = 0; h < 2; ++h) {
            // ---- layer 1 (transposed): D[hidden][row] = A_q[hidden][:] . F[row][:]
            f32x4 acc1[2][8];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 8; ++j) acc1[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
            const uint16_t *arow[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) arow[i] = Aq + (int64_t)(kHalf * h + 32 * w + 16 * i + li) * kKPad + lk;
            // A fragments two K steps ahead (they come from L2)
            bf16x8 fa[2], f1[2], f2[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                fa[i] = as_bf(*(const u32x4 *)arow[i]);
                f1[i] = as_bf(*(const u32x4 *)(arow[i] + 32));
            }
#pragma unroll
            for (int kk = 0; kk < kKPad; kk += 32) {
                if (kk + 64 < kKPad)
#pragma unroll
                    for (int i = 0; i < 2; ++i) f2[i] = as_bf(*(const u32x4 *)(arow[i] + kk + 64));
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const bf16x8 fb = as_bf(*(const u32x4 *)&Ft[(16 * j + li) * kFStride + kk + lk]);
#pragma unroll
                    for (int i = 0; i < 2; ++i) acc1[i][j] = mfma(fa[i], fb, acc1[i][j]);
                }
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    fa[i] = f1[i];
                    f1[i] = f2[i];
                }
            }
            // ---- bias, length term, ReLU: four consecutive hidden units of one row per lane
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int m0 = kHalf * h + 32 * w + 16 * i + 4 * lg;
                const float4 cv = *(const float4 *)(a.cvec + m0);
                const float4 wx = *(const float4 *)(a.w1x + m0);
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int n = 16 * j + li;
                    const float xr = fminf(lq, rowlog[n]) - a.mu400;   // w1x holds the 1 / sd
                    const float z0 = fmaxf(acc1[i][j][0] + cv.x + wx.x * xr, 0.0f);
                    const float z1 = fmaxf(acc1[i][j][1] + cv.y + wx.y * xr, 0.0f);
                    const float z2 = fmaxf(acc1[i][j][2] + cv.z + wx.z * xr, 0.0f);
                    const float z3 = fmaxf(acc1[i][j][3] + cv.w + wx.w * xr, 0.0f);
                    *(uint2 *)&Hh[n * kH2Stride + 32 * w + 16 * i + 4 * lg] =
                        make_uint2(pack_bf16(z0, z1), pack_bf16(z2, z3));
                }
            }
            __syncthreads();
            // ---- layer 2 (transposed) over this half: D[out][row] += W2[out][half] . H[row][half]
            const uint16_t *wrow[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) wrow[i] = a.W2bf + (int64_t)(64 * w + 16 * i + li) * kNH + kHalf * h + lk;
            bf16x8 wa[4], wn[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) wa[i] = as_bf(*(const u32x4 *)wrow[i]);
#pragma unroll
            for (int kk = 0; kk < kHalf; kk += 32) {
                if (kk + 32 < kHalf)
#pragma unroll
                    for (int i = 0; i < 4; ++i) wn[i] = as_bf(*(const u32x4 *)(wrow[i] + kk + 32));
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const bf16x8 hb = as_bf(*(const u32x4 *)&Hh[(16 * j + li) * kH2Stride + kk + lk]);
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc2[i][j] = mfma(wa[i], hb, acc2[i][j]);
                }
                if (kk + 32 < kHalf)
#pragma unroll
                    for (int i = 0; i < 4; ++i) wa[i] = wn[i];
            }
            __syncthreads();   // the next half overwrites the activations
        }
        // ---- output: y[row] = b3 + sum over outputs of relu(. + b2) w3
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            float sum = 0.0f;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) sum += fmaxf(acc2[i][j][r] + b2v[i][r], 0.0f) * w3v[i][r];
            sum += __shfl_xor(sum, 16);
            sum += __shfl_xor(sum, 32);
            if (lg == 0) part[w][16 * j + li] = sum;
        }
        __syncthreads();
        if (tid < kInferRows) {
            const int64_t row = row0 + tid;
            if (row < a.nrows) {
                const float y = b3 + part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
                a.pred[(int64_t)q * a.nrows + row] = a.row_db[row] >= 0 ? y : -INFINITY;
            }
        }
        // part is written again only after the next query's two barriers
    }
}

// ------------------------------------------------------------------ selection

constexpr int kHistRows = 16384;

__global__ void __launch_bounds__(256) key_hist_kernel(const float *pred, int64_t nrows, int level,
                                                       const uint32_t *prefix, uint32_t *hist)
{
    __shared__ uint32_t h[2048];
    const int q = blockIdx.y;
    for (int b = threadIdx.x; b < 2048; b += 256) h[b] = 0;
    __syncthreads();
    const int64_t r0 = (int64_t)blockIdx.x * kHistRows, r1 = min(nrows, r0 + kHistRows);
    const uint32_t pre = prefix ? prefix[q] : 0u;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
        const uint32_t key = order_key(pred[(int64_t)q * nrows + r]);
        if (level == 0) {
            atomicAdd(&h[key >> 21], 1u);
        } else if (level == 1) {
            if ((key >> 21) == pre) atomicAdd(&h[(key >> 10) & 0x7FFu], 1u);
        } else {
            if ((key >> 10) == pre) atomicAdd(&h[key & 0x3FFu], 1u);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < 2048; b += 256)
        if (h[b]) atomicAdd(&hist[(int64_t)q * 2048 + b], h[b]);
}

// Audit draw of (query, database index): splitmix64 of
// seed + golden * (q * 2^32 + index + 1); audited when the high half < threshold.
__device__ __forceinline__ bool audited(uint64_t seed, int q, int32_t idx, uint32_t threshold)
{
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (((uint64_t)(uint32_t)q << 32) + (uint64_t)idx + 1ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (uint32_t)(z >> 32) < threshold;
}

__global__ void __launch_bounds__(256) mark_kernel(const float *pred, int64_t nrows, const uint32_t *thr,
                                                   const int32_t *row_db, uint64_t seed, uint32_t audit_threshold,
                                                   uint8_t *marks, int32_t *chunk_counts)
{
    __shared__ int32_t cnt;
    const int q = blockIdx.y;
    const int64_t r = (int64_t)blockIdx.x * kMarkChunk + threadIdx.x;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    uint8_t mk = 0;
    if (r < nrows) {
        const int32_t idx = row_db[r];
        if (idx >= 0) {
            if (order_key(pred[(int64_t)q * nrows + r]) >= thr[q])
                mk = 1;
            else if (audited(seed, q, idx, audit_threshold))
                mk = 2;
        }
        marks[(int64_t)q * nrows + r] = mk;
    }
    if (mk) atomicAdd(&cnt, 1);
    __syncthreads();
    if (threadIdx.x == 0) chunk_counts[(int64_t)q * gridDim.x + blockIdx.x] = cnt;
}

__global__ void __launch_bounds__(256) compact_kernel(const uint8_t *marks, int64_t nrows, const int64_t *chunk_base,
                                                      int32_t *out_rows, uint8_t *out_kind)
{
    __shared__ int32_t wsum[4];
    const int q = blockIdx.y;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * kMarkChunk + threadIdx.x;
    const uint8_t mk = r < nrows ? marks[(int64_t)q * nrows + r] : 0;
    const uint64_t bal = __ballot(mk != 0);
    const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0));
    if (lane == 0) wsum[w] = __popcll(bal);
    __syncthreads();
    int base = 0;
    for (int i = 0; i < w; ++i) base += wsum[i];
    if (mk) {
        const int64_t o = chunk_base[(int64_t)q * gridDim.x + blockIdx.x] + base + below;
        out_rows[o] = (int32_t)r;
        out_kind[o] = mk;
    }
}

// Length-group excess: the database rows are stored length-sorted, 128 to a
// group, so the mean prediction of a group's sequences estimates what a
// sequence of that length scores against the query by chance; each
// prediction becomes its excess over that mean.  One block per (group, query).
__global__ void __launch_bounds__(128) excess_kernel(float *pred, int64_t nrows, const int32_t *row_db,
                                                     int standardise)
{
    __shared__ float psum[2], psq[2];
    __shared__ int pcnt[2];
    const int q = blockIdx.y;
    const int64_t r = (int64_t)blockIdx.x * 128 + threadIdx.x;
    const bool valid = r < nrows && row_db[r] >= 0;
    float v = valid ? pred[(int64_t)q * nrows + r] : 0.0f;
    int c = valid ? 1 : 0;
    float sum = v, sq = v * v;
    for (int off = 32; off >= 1; off >>= 1) {
        sum += __shfl_xor(sum, off);
        sq += __shfl_xor(sq, off);
        c += __shfl_xor(c, off);
    }
    if ((threadIdx.x & 63) == 0) {
        psum[threadIdx.x >> 6] = sum;
        psq[threadIdx.x >> 6] = sq;
        pcnt[threadIdx.x >> 6] = c;
    }
    __syncthreads();
    const int n = pcnt[0] + pcnt[1];
    const float mean = n ? (psum[0] + psum[1]) / (float)n : 0.0f;
    float scale = 1.0f;
    if (standardise && n > 1) {
        const float var = fmaxf((psq[0] + psq[1]) / (float)n - mean * mean, 0.0f);
        scale = 1.0f / fmaxf(sqrtf(var), 1e-3f);
    }
    if (valid) pred[(int64_t)q * nrows + r] = (v - mean) * scale;
}

__global__ void step_end_kernel(int32_t *ctr)
{
    if (threadIdx.x == 0) {
        ctr[0] += 1;
        ctr[1] += 1;
    }
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)std::max<int64_t>(1, (n + per - 1) / per); }

}  // namespace

hipError_t launch_dipeptides(const uint8_t *codes, const int64_t *off, int64_t nseq, const int32_t *dst_row,
                             int32_t *counts, float *freq32, uint16_t *freqbf, int32_t *lens, hipStream_t st)
{
    if (nseq <= 0) return hipSuccess;
    hipLaunchKernelGGL(dipeptide_kernel, dim3(blocks_for(nseq, 4)), dim3(256), 0, st, codes, off, nseq, dst_row,
                       counts, freq32, freqbf, lens);
    return hipGetLastError();
}

hipError_t launch_pair_stats(const float *freq32, const int32_t *lens, const int32_t *rows, const int32_t *cols,
                             int64_t npairs, double *sum, double *sumsq, hipStream_t st)
{
    // partial sums live behind sum: the caller reserves 2 * 401 * 1025 doubles there
    const int64_t chunk = std::max<int64_t>(1, (npairs + 1023) / 1024);
    const int nblocks = (int)std::max<int64_t>(1, (npairs + chunk - 1) / chunk);
    double *partial = sum + 2 * kNIn;
    hipLaunchKernelGGL(pair_stats_kernel, dim3(nblocks), dim3(512), 0, st, freq32, lens, rows, cols, npairs, chunk,
                       partial);
    hipLaunchKernelGGL(pair_stats_final_kernel, dim3(2), dim3(256), 0, st, partial, nblocks, sum, sumsq);
    return hipGetLastError();
}

hipError_t launch_pair_z(const float *freq32, const int32_t *lens, const int32_t *rows, const int32_t *cols,
                         int64_t npairs, const float *mu, const float *sd, uint16_t *Z, hipStream_t st)
{
    if (npairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(pair_z_kernel, dim3((unsigned)npairs), dim3(448), 0, st, freq32, lens, rows, cols, mu, sd, Z);
    return hipGetLastError();
}

hipError_t launch_labels(const int32_t *scores, int64_t n, float *y, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(labels_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, scores, n, y);
    return hipGetLastError();
}

hipError_t launch_z_to_bf16(const float *z, int64_t B, uint16_t *Z, hipStream_t st)
{
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(z_to_bf16_kernel, dim3((unsigned)B), dim3(448), 0, st, z, Z);
    return hipGetLastError();
}

hipError_t launch_gather_rows(const uint16_t *Z, const float *y, const int32_t *idx, const int32_t *ctr, int B,
                              uint16_t *Xb, float *yb, hipStream_t st)
{
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)B), dim3(64), 0, st, Z, y, idx, ctr, Xb, yb);
    return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs &g, bool at, bool bt, hipStream_t st)
{
    const int splits = g.splits > 1 ? g.splits : 1;
    if (g.K % (32 * splits) != 0 || (splits > 1 && (g.epi != kEpiF32 || !g.partial))) return hipErrorInvalidValue;
    const dim3 grid(blocks_for(g.N, 64), blocks_for(g.M, 64), (unsigned)splits);
    if (!at && !bt) gemm_kernel<false, false><<<grid, dim3(256), 0, st>>>(g);
    if (!at && bt) gemm_kernel<false, true><<<grid, dim3(256), 0, st>>>(g);
    if (at && !bt) gemm_kernel<true, false><<<grid, dim3(256), 0, st>>>(g);
    if (at && bt) gemm_kernel<true, true><<<grid, dim3(256), 0, st>>>(g);
    if (splits > 1)
        hipLaunchKernelGGL(splitk_reduce_kernel, dim3(blocks_for((int64_t)g.M * g.N, 256)), dim3(256), 0, st,
                           g.partial, splits, g.M, g.N, g.out32, g.ldc);
    return hipGetLastError();
}

hipError_t launch_head(const float *H2, const float *y, const float *theta, int B, float *d, float *dz2,
                       uint16_t *dz2bf, double *loss, hipStream_t st)
{
    hipLaunchKernelGGL(head_kernel, dim3(blocks_for(B, 4)), dim3(256), 0, st, H2, y, theta, B, d, dz2, dz2bf, loss);
    return hipGetLastError();
}

hipError_t launch_colsum(const float *X, int64_t ldx, int rows, int cols, const float *scale, float *partial,
                         float *out, hipStream_t st)
{
    hipLaunchKernelGGL(colsum_kernel, dim3(blocks_for(cols, 256), kColSlices), dim3(256), 0, st, X, ldx, rows, cols,
                       scale, partial);
    hipLaunchKernelGGL(colsum_final_kernel, dim3(blocks_for(cols, 256)), dim3(256), 0, st, partial, cols, out);
    return hipGetLastError();
}

hipError_t launch_adam(float *theta, float *m, float *v, const float *g, int64_t n, float lr, float b1, float b2,
                       float eps, float bc1, float bc2, const int32_t *ctr, hipStream_t st)
{
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, theta, m, v, g, n, lr, b1, b2, eps,
                       bc1, bc2, ctr);
    return hipGetLastError();
}

hipError_t launch_step_end(int32_t *ctr, hipStream_t st)
{
    hipLaunchKernelGGL(step_end_kernel, dim3(1), dim3(64), 0, st, ctr);
    return hipGetLastError();
}

hipError_t launch_pack_weights(const float *theta, uint16_t *W1bf, uint16_t *W2bf, hipStream_t st)
{
    hipLaunchKernelGGL(pack_weights_kernel, dim3(kNH), dim3(256), 0, st, theta, W1bf, W2bf);
    return hipGetLastError();
}

hipError_t launch_fold_const(const float *theta, const float *mu, const float *sd, float *cvec, float *w1x,
                             hipStream_t st)
{
    hipLaunchKernelGGL(fold_const_kernel, dim3(kNH), dim3(256), 0, st, theta, mu, sd, cvec, w1x);
    return hipGetLastError();
}

hipError_t launch_fold_query(const float *theta, const float *fq, int nq, const float *sd, uint16_t *Aq,
                             hipStream_t st)
{
    if (nq <= 0) return hipSuccess;
    hipLaunchKernelGGL(fold_query_kernel, dim3(kNH, nq), dim3(448), 0, st, theta, fq, sd, Aq);
    return hipGetLastError();
}

hipError_t launch_infer(const InferArgs &a, hipStream_t st)
{
    if (a.nrows <= 0 || a.nq <= 0) return hipSuccess;
    // the all-queries kernel needs 143 KB of dynamic LDS per workgroup; otherwise the 64-row one
    int dev = 0, lds_wg = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&lds_wg, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        (size_t)lds_wg >= kInferLds + sizeof(float) * 5 * kInferRows) {
        hipLaunchKernelGGL(infer_all_kernel, dim3(blocks_for(a.nrows, kInferRows)), dim3(256), kInferLds, st, a);
        return hipGetLastError();
    }
    (void)hipGetLastError();
    hipLaunchKernelGGL(infer_kernel, dim3(blocks_for(a.nrows, 64), a.nq), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_key_hist(const float *pred, int64_t nrows, int nq, int level, const uint32_t *prefix,
                           uint32_t *hist, hipStream_t st)
{
    hipLaunchKernelGGL(key_hist_kernel, dim3(blocks_for(nrows, kHistRows), nq), dim3(256), 0, st, pred, nrows, level,
                       prefix, hist);
    return hipGetLastError();
}

hipError_t launch_mark(const float *pred, int64_t nrows, int nq, const uint32_t *thr, const int32_t *row_db,
                       uint64_t seed, uint32_t audit_threshold, uint8_t *marks, int32_t *chunk_counts,
                       hipStream_t st)
{
    hipLaunchKernelGGL(mark_kernel, dim3(blocks_for(nrows, kMarkChunk), nq), dim3(256), 0, st, pred, nrows, thr,
                       row_db, seed, audit_threshold, marks, chunk_counts);
    return hipGetLastError();
}

hipError_t launch_excess(float *pred, int64_t nrows, int nq, const int32_t *row_db, bool standardise,
                         hipStream_t st)
{
    if (nrows <= 0 || nq <= 0) return hipSuccess;
    hipLaunchKernelGGL(excess_kernel, dim3((unsigned)((nrows + 127) / 128), nq), dim3(128), 0, st, pred, nrows,
                       row_db, standardise ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_compact(const uint8_t *marks, int64_t nrows, int nq, const int64_t *chunk_base, int32_t *out_rows,
                          uint8_t *out_kind, hipStream_t st)
{
    hipLaunchKernelGGL(compact_kernel, dim3(blocks_for(nrows, kMarkChunk), nq), dim3(256), 0, st, marks, nrows,
                       chunk_base, out_rows, out_kind);
    return hipGetLastError();
}

}  // namespace swh
