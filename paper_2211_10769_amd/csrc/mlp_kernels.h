// mlp_kernels.h -- kernels of the learned prefilter (mlp_kernels.hip):
// dipeptide features, bfloat16 MFMA products with fused epilogues, the
// training step's reductions and Adam, the folded inference network and the
// candidate selection.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swh {

constexpr int kNStd = 20;                 // standard residues (codes 0..19)
constexpr int kNDip = kNStd * kNStd;      // 400 dipeptides
constexpr int kNIn = kNDip + 1;           // + log length
constexpr int kKPad = 416;                // input width padded to a multiple of 32
constexpr int kNH = 256;                  // hidden width
// flat parameter layout: W1 [256 x 401] | b1 | W2 [256 x 256] | b2 | w3 | b3
constexpr int64_t kOffW1 = 0;
constexpr int64_t kOffB1 = kOffW1 + (int64_t)kNH * kNIn;
constexpr int64_t kOffW2 = kOffB1 + kNH;
constexpr int64_t kOffB2 = kOffW2 + (int64_t)kNH * kNH;
constexpr int64_t kOffW3 = kOffB2 + kNH;
constexpr int64_t kOffB3 = kOffW3 + kNH;
constexpr int64_t kNParams = kOffB3 + 1;  // 168,961

// Dipeptide counts / frequencies of nseq sequences (codes, offsets).  Output
// row of sequence i: dst_row ? dst_row[i] : i (negative: skipped).  Any of the
// outputs may be NULL: counts [row][400] int32, freq32 [row][400],
// freqbf [row][416] bfloat16 (zero padding), lens [row].
hipError_t launch_dipeptides(const uint8_t *codes, const int64_t *off, int64_t nseq, const int32_t *dst_row,
                             int32_t *counts, float *freq32, uint16_t *freqbf, int32_t *lens, hipStream_t st);

// Training features.  Sums and sums of squares (float64) of the 401 pair
// features over all pairs, then the normalised bfloat16 rows [pair][416].
hipError_t launch_pair_stats(const float *freq32, const int32_t *lens, const int32_t *rows, const int32_t *cols,
                             int64_t npairs, double *sum, double *sumsq, hipStream_t st);
hipError_t launch_pair_z(const float *freq32, const int32_t *lens, const int32_t *rows, const int32_t *cols,
                         int64_t npairs, const float *mu, const float *sd, uint16_t *Z, hipStream_t st);
// y = ln(1 + S)
hipError_t launch_labels(const int32_t *scores, int64_t n, float *y, hipStream_t st);
// float rows [B][401] -> bfloat16 [B][416]
hipError_t launch_z_to_bf16(const float *z, int64_t B, uint16_t *Z, hipStream_t st);
// Xb[i] = Z[j], yb[i] = y[j] with j = idx[b B + i] for i < B, b = ctr ? ctr[0] : 0
hipError_t launch_gather_rows(const uint16_t *Z, const float *y, const int32_t *idx, const int32_t *ctr, int B,
                              uint16_t *Xb, float *yb, hipStream_t st);

// C = A B (bfloat16 operands, float32 accumulation).  A(m,k) = at ? A[k lda + m]
// : A[m lda + k]; B(k,n) = bt ? B[n ldb + k] : B[k ldb + n].  K % 32 == 0;
// loads read rows m < mload, columns n < nload (multiples of 8, zero
// beyond); results are stored for m < M, n < N.
enum GemmEpilogue {
    kEpiF32 = 0,          // out32 = C
    kEpiBiasReluBf = 1,   // outbf = bf16(relu(C + bias[n]))
    kEpiBiasReluF32 = 2,  // out32 = relu(C + bias[n])
    kEpiMask = 3,         // v = C * (mask[m][n] > 0): out32 = v, outbf = bf16(v)
};
struct GemmArgs {
    const uint16_t *A, *B;
    int64_t lda, ldb;
    int M, N, K, mload, nload;
    int epi;
    float *out32;
    uint16_t *outbf;
    int64_t ldc;
    const float *bias;
    const uint16_t *mask;   // bfloat16, leading dimension ldc
    // split-K (kEpiF32 only): splits > 1 sums K in `splits` slices into
    // partial [splits][M][N] and then into out32
    int splits;
    float *partial;
};
hipError_t launch_gemm(const GemmArgs &g, bool at, bool bt, hipStream_t st);

// Output head and its backward: yhat = H2 w3 + b3, d = 2 (yhat - y) / B,
// loss += sum (yhat - y)^2 (float64), dz2 = d w3 (H2 > 0) as float and bf16.
hipError_t launch_head(const float *H2, const float *y, const float *theta, int B, float *d, float *dz2,
                       uint16_t *dz2bf, double *loss, hipStream_t st);
// out[n] = sum_r X[r][n] * (scale ? scale[r] : 1) for n < cols (deterministic, two stages)
hipError_t launch_colsum(const float *X, int64_t ldx, int rows, int cols, const float *scale, float *partial,
                         float *out, hipStream_t st);
// Adam on the flat parameters; bc1 = 1 - b1^t, bc2 = 1 - b2^t, or with ctr
// t = ctr[1] + 1 read on the device (a captured step replays unchanged)
hipError_t launch_adam(float *theta, float *m, float *v, const float *g, int64_t n, float lr, float b1, float b2,
                       float eps, float bc1, float bc2, const int32_t *ctr, hipStream_t st);
// ctr[0] (batch within the epoch) and ctr[1] (Adam step) advance by one
hipError_t launch_step_end(int32_t *ctr, hipStream_t st);
// bfloat16 copies of W1 ([256][416], zero padding) and W2 ([256][256])
hipError_t launch_pack_weights(const float *theta, uint16_t *W1bf, uint16_t *W2bf, hipStream_t st);

// Inference, query folded into the first layer.
// cvec[n] = b1[n] - sum_k W1[n][k] mu_k / sd_k (k < 400); w1x[n] = W1[n][400] / sd_400
hipError_t launch_fold_const(const float *theta, const float *mu, const float *sd, float *cvec, float *w1x,
                             hipStream_t st);
// Aq[q][n][k] = bf16(W1[n][k] fq[q][k] / sd_k), k < 400; 0 for 400 <= k < 416
hipError_t launch_fold_query(const float *theta, const float *fq, int nq, const float *sd, uint16_t *Aq,
                             hipStream_t st);
struct InferArgs {
    const uint16_t *F;       // database rows [nrows][416] bfloat16 frequencies
    const int32_t *row_len;  // residues per row (0: empty slot)
    const int32_t *row_db;   // database index per row (-1: empty slot)
    int64_t nrows;
    const uint16_t *Aq;      // [nq][256][416]
    const int32_t *qlen;     // [nq]
    int nq;
    const float *cvec, *w1x;    // folded bias; W1[:,400] / sd_400
    float mu400;
    const uint16_t *W2bf;    // [256][256]
    const float *theta;      // b2, w3, b3
    float *pred;             // [nq][nrows]; -inf for empty slots
};
hipError_t launch_infer(const InferArgs &a, hipStream_t st);

// Selection of the largest predictions: radix histograms of order-preserving
// keys (11, 11, 10 bits), then marks (1 = candidate: key >= thr[q];
// 2 = audited non-candidate) and an ordered compaction of marked rows.
hipError_t launch_key_hist(const float *pred, int64_t nrows, int nq, int level, const uint32_t *prefix,
                           uint32_t *hist, hipStream_t st);
hipError_t launch_mark(const float *pred, int64_t nrows, int nq, const uint32_t *thr, const int32_t *row_db,
                       uint64_t seed, uint32_t audit_threshold, uint8_t *marks, int32_t *chunk_counts,
                       hipStream_t st);
constexpr int kMarkChunk = 256;
// pred[q][r] -= mean of pred[q][.] over the valid rows (row_db >= 0) of r's
// group of 128 rows; standardise: then divided by their deviation
hipError_t launch_excess(float *pred, int64_t nrows, int nq, const int32_t *row_db, bool standardise,
                         hipStream_t st);
hipError_t launch_compact(const uint8_t *marks, int64_t nrows, int nq, const int64_t *chunk_base, int32_t *out_rows,
                          uint8_t *out_kind, hipStream_t st);

}  // namespace swh
