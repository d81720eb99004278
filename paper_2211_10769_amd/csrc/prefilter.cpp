// prefilter.cpp -- learned prefilter for the database search.
//
// A small network (401 -> 256 -> 256 -> 1) predicts ln(1 + S) of a (query,
// database sequence) pair from the product of their dipeptide frequencies and
// the log of the shorter length.  It is trained on exact scores that the
// engine computes itself, on the GPU (bfloat16 MFMA products, float32
// accumulation, Adam on float32 master weights).  A search predicts every
// pair, keeps the best-ranked fraction of the database per query, rescores
// those exactly with the database kernels, audits a sample of the rest and
// falls back to the exhaustive search for a query whose audit finds a better
// hit: every reported score is exact.
//
// Inference folds the query into the first layer: with the query fixed the
// normalised feature k is affine in the database frequency f_t[k], so
//   W1 z = (W1 diag(f_q / sd)) f_t + (b1 - W1 (mu / sd)) + W1[:,400] z_400
// and one bfloat16 GEMM per query scores the whole database.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "batch.h"
#include "db.h"
#include "db_kernels.h"
#include "mlp_kernels.h"
#include "prefilter.h"
#include "strips.h"

namespace swh {

namespace {

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t0) { return std::chrono::duration<double, std::milli>(Clock::now() - t0).count(); }

void free_buf(DevBuf &b)
{
    if (b.p) hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

uint64_t splitmix(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename T>
swh_status upload(swh_ctx *ctx, DevBuf &buf, const T *v, size_t n, hipStream_t st, const char *what)
{
    swh_status s = ensure(ctx, buf, n * sizeof(T) + 16, what);
    if (s != SWH_OK) return s;
    if (n == 0) return SWH_OK;
    hipError_t e = hipMemcpyAsync(buf.p, v, n * sizeof(T), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(ctx, e, what);
    return SWH_OK;
}

// Weight gradients reduce over the batch (K = B, M x N = 256 x 256 or 401):
// split K so that the grid holds enough workgroups.
constexpr int kSplitMax = 16;

// Device buffers of one training call (or one gradient evaluation).
struct TrainWs {
    DevBuf Xb, yb, H1bf, H2, d, dz2, dz2bf, dz1, dz1bf, grad, colpart, splitk;
    double *loss = nullptr;   // one double, device
    ~TrainWs()
    {
        for (DevBuf *b : {&Xb, &yb, &H1bf, &H2, &d, &dz2, &dz2bf, &dz1, &dz1bf, &grad, &colpart, &splitk})
            free_buf(*b);
        if (loss) hipFree(loss);
    }
};

swh_status ws_alloc(swh_ctx *ctx, TrainWs &w, int B)
{
    swh_status s;
    const size_t hb = (size_t)B * kNH;
    if ((s = ensure(ctx, w.Xb, (size_t)B * kKPad * 2, "batch inputs")) != SWH_OK ||
        (s = ensure(ctx, w.yb, (size_t)B * 4, "batch labels")) != SWH_OK ||
        (s = ensure(ctx, w.H1bf, hb * 2, "hidden 1")) != SWH_OK || (s = ensure(ctx, w.H2, hb * 4, "hidden 2")) != SWH_OK ||
        (s = ensure(ctx, w.d, (size_t)B * 4, "output gradient")) != SWH_OK ||
        (s = ensure(ctx, w.dz2, hb * 4, "gradient 2")) != SWH_OK ||
        (s = ensure(ctx, w.dz2bf, hb * 2, "gradient 2 (bf16)")) != SWH_OK ||
        (s = ensure(ctx, w.dz1, hb * 4, "gradient 1")) != SWH_OK ||
        (s = ensure(ctx, w.dz1bf, hb * 2, "gradient 1 (bf16)")) != SWH_OK ||
        (s = ensure(ctx, w.grad, (size_t)kNParams * 4, "parameter gradient")) != SWH_OK ||
        (s = ensure(ctx, w.colpart, (size_t)32 * kNH * 4, "column sums")) != SWH_OK ||
        (s = ensure(ctx, w.splitk, (size_t)kSplitMax * kNH * kKPad * 4, "split-K partial sums")) != SWH_OK)
        return s;
    if (!w.loss && hipMalloc((void **)&w.loss, 8) != hipSuccess) return fail(ctx, SWH_E_NOMEM, "loss accumulator");
    return SWH_OK;
}

int splits_for(int B)
{
    int s = kSplitMax;
    while (s > 1 && (B % (32 * s) != 0 || B / s < 128)) s /= 2;
    return s;
}

GemmArgs gemm(const uint16_t *A, int64_t lda, const uint16_t *B, int64_t ldb, int M, int N, int K, int mload,
              int nload, int epi, int64_t ldc)
{
    GemmArgs g{};
    g.A = A;
    g.B = B;
    g.lda = lda;
    g.ldb = ldb;
    g.M = M;
    g.N = N;
    g.K = K;
    g.mload = mload;
    g.nload = nload;
    g.epi = epi;
    g.ldc = ldc;
    return g;
}

// Forward and backward of the batch in w.Xb / w.yb; gradient in w.grad, the
// sum of squared residuals added to *w.loss.
hipError_t forward_backward(swh_model *m, TrainWs &w, int B, hipStream_t st)
{
    float *theta = (float *)m->theta.p;
    float *grad = (float *)w.grad.p;
    const uint16_t *Xb = (const uint16_t *)w.Xb.p;
    uint16_t *H1 = (uint16_t *)w.H1bf.p;
    float *H2 = (float *)w.H2.p;
    hipError_t e;
    GemmArgs g = gemm(Xb, kKPad, (const uint16_t *)m->W1bf.p, kKPad, B, kNH, kKPad, B, kNH, kEpiBiasReluBf, kNH);
    g.bias = theta + kOffB1;
    g.outbf = H1;
    if ((e = launch_gemm(g, false, true, st)) != hipSuccess) return e;
    g = gemm(H1, kNH, (const uint16_t *)m->W2bf.p, kNH, B, kNH, kNH, B, kNH, kEpiBiasReluF32, kNH);
    g.bias = theta + kOffB2;
    g.out32 = H2;
    if ((e = launch_gemm(g, false, true, st)) != hipSuccess) return e;
    if ((e = launch_head(H2, (const float *)w.yb.p, theta, B, (float *)w.d.p, (float *)w.dz2.p,
                         (uint16_t *)w.dz2bf.p, w.loss, st)) != hipSuccess)
        return e;
    // dW2 = dz2^T h1
    g = gemm((const uint16_t *)w.dz2bf.p, kNH, H1, kNH, kNH, kNH, B, kNH, kNH, kEpiF32, kNH);
    g.out32 = grad + kOffW2;
    g.splits = splits_for(B);
    g.partial = (float *)w.splitk.p;
    if ((e = launch_gemm(g, true, false, st)) != hipSuccess) return e;
    // dz1 = (dz2 W2) * (h1 > 0)
    g = gemm((const uint16_t *)w.dz2bf.p, kNH, (const uint16_t *)m->W2bf.p, kNH, B, kNH, kNH, B, kNH, kEpiMask, kNH);
    g.mask = H1;
    g.out32 = (float *)w.dz1.p;
    g.outbf = (uint16_t *)w.dz1bf.p;
    if ((e = launch_gemm(g, false, false, st)) != hipSuccess) return e;
    // dW1 = dz1^T x
    g = gemm((const uint16_t *)w.dz1bf.p, kNH, Xb, kKPad, kNH, kNIn, B, kNH, kKPad, kEpiF32, kNIn);
    g.out32 = grad + kOffW1;
    g.splits = splits_for(B);
    g.partial = (float *)w.splitk.p;
    if ((e = launch_gemm(g, true, false, st)) != hipSuccess) return e;
    float *cp = (float *)w.colpart.p;
    if ((e = launch_colsum((const float *)w.dz1.p, kNH, B, kNH, nullptr, cp, grad + kOffB1, st)) != hipSuccess ||
        (e = launch_colsum((const float *)w.dz2.p, kNH, B, kNH, nullptr, cp, grad + kOffB2, st)) != hipSuccess ||
        (e = launch_colsum(H2, kNH, B, kNH, (const float *)w.d.p, cp, grad + kOffW3, st)) != hipSuccess ||
        (e = launch_colsum((const float *)w.d.p, 1, B, 1, nullptr, cp, grad + kOffB3, st)) != hipSuccess)
        return e;
    return hipSuccess;
}

// Adam step; with ctr the step number is read on the device (graph replays).
hipError_t adam_update(swh_model *m, TrainWs &w, double lr, hipStream_t st, const int32_t *ctr = nullptr)
{
    const double b1 = 0.9, b2 = 0.999;
    if (!ctr) m->steps += 1;
    const float bc1 = (float)(1.0 - std::pow(b1, (double)m->steps));
    const float bc2 = (float)(1.0 - std::pow(b2, (double)m->steps));
    hipError_t e;
    if ((e = launch_adam((float *)m->theta.p, (float *)m->adam_m.p, (float *)m->adam_v.p, (const float *)w.grad.p,
                         kNParams, (float)lr, (float)b1, (float)b2, 1e-8f, bc1, bc2, ctr, st)) != hipSuccess)
        return e;
    return launch_pack_weights((const float *)m->theta.p, (uint16_t *)m->W1bf.p, (uint16_t *)m->W2bf.p, st);
}

// Inference constants of the current weights.
hipError_t refresh_fold(swh_model *m, hipStream_t st)
{
    return launch_fold_const((const float *)m->theta.p, (const float *)m->mu_d.p, (const float *)m->sd_d.p,
                             (float *)m->cvec.p, (float *)m->w1x.p, st);
}

swh_status model_alloc(swh_ctx *ctx, swh_model *m)
{
    swh_status s;
    if ((s = ensure(ctx, m->theta, kNParams * 4, "parameters")) != SWH_OK ||
        (s = ensure(ctx, m->adam_m, kNParams * 4, "Adam moments")) != SWH_OK ||
        (s = ensure(ctx, m->adam_v, kNParams * 4, "Adam moments")) != SWH_OK ||
        (s = ensure(ctx, m->W1bf, (size_t)kNH * kKPad * 2, "W1 (bf16)")) != SWH_OK ||
        (s = ensure(ctx, m->W2bf, (size_t)kNH * kNH * 2, "W2 (bf16)")) != SWH_OK ||
        (s = ensure(ctx, m->cvec, kNH * 4, "folded bias")) != SWH_OK ||
        (s = ensure(ctx, m->w1x, kNH * 4, "folded length weight")) != SWH_OK ||
        (s = ensure(ctx, m->mu_d, kNIn * 4, "feature means")) != SWH_OK ||
        (s = ensure(ctx, m->sd_d, kNIn * 4, "feature deviations")) != SWH_OK)
        return s;
    return SWH_OK;
}

// Upload parameters and normalisation, reset Adam, derive the bf16 copies and
// the inference constants.
swh_status model_install(swh_ctx *ctx, swh_model *m, const float *theta, const float *mu, const float *sd)
{
    hipStream_t st = ctx->own_stream;
    hipError_t e;
    m->mu.assign(mu, mu + kNIn);
    m->sd.assign(sd, sd + kNIn);
    for (float &x : m->sd)
        if (!(x > 0.0f)) x = 1.0f;
    m->steps = 0;
    if ((e = hipMemcpyAsync(m->theta.p, theta, kNParams * 4, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(m->mu_d.p, m->mu.data(), kNIn * 4, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(m->sd_d.p, m->sd.data(), kNIn * 4, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemsetAsync(m->adam_m.p, 0, kNParams * 4, st)) != hipSuccess ||
        (e = hipMemsetAsync(m->adam_v.p, 0, kNParams * 4, st)) != hipSuccess ||
        (e = launch_pack_weights((const float *)m->theta.p, (uint16_t *)m->W1bf.p, (uint16_t *)m->W2bf.p, st)) !=
            hipSuccess ||
        (e = refresh_fold(m, st)) != hipSuccess || (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, "model upload");
    return SWH_OK;
}

// He-normal initial weights from a splitmix64 stream (Box-Muller), zero biases.
void init_params(uint64_t seed, std::vector<float> &theta)
{
    theta.assign(kNParams, 0.0f);
    uint64_t s = seed;
    auto normal = [&]() {
        const double u1 = ((splitmix(s) >> 11) + 1.0) * (1.0 / 9007199254740993.0);
        const double u2 = (splitmix(s) >> 11) * (1.0 / 9007199254740992.0);
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    };
    for (int64_t i = 0; i < (int64_t)kNH * kNIn; ++i) theta[kOffW1 + i] = (float)(normal() * std::sqrt(2.0 / kNIn));
    for (int64_t i = 0; i < (int64_t)kNH * kNH; ++i) theta[kOffW2 + i] = (float)(normal() * std::sqrt(2.0 / kNH));
    for (int64_t i = 0; i < kNH; ++i) theta[kOffW3 + i] = (float)(normal() * std::sqrt(1.0 / kNH));
}

// Encode host sequences (cat, off with nseq entries) into dst codes; offsets rebased.
swh_status encode_pool(swh_ctx *ctx, const Scoring &sc, int64_t nseq, const char *cat, const int64_t *off,
                       DevBuf &raw, DevBuf &codes, DevBuf &offs_d, std::vector<int64_t> &h_off, const char *what)
{
    hipStream_t st = ctx->own_stream;
    for (int64_t i = 0; i < nseq; ++i)
        if (off[i + 1] < off[i]) return fail(ctx, SWH_E_INVAL, std::string(what) + ": offsets must not decrease");
    const int64_t base = nseq ? off[0] : 0, total = nseq ? off[nseq] - base : 0;
    h_off.resize((size_t)nseq + 1);
    for (int64_t i = 0; i <= nseq; ++i) h_off[i] = nseq ? off[i] - base : 0;
    swh_status s;
    if ((s = ensure(ctx, raw, (size_t)total + 16, what)) != SWH_OK ||
        (s = ensure(ctx, codes, (size_t)total + 16, what)) != SWH_OK ||
        (s = ensure(ctx, ctx->lut, 256, "symbol table")) != SWH_OK ||
        (s = ensure(ctx, ctx->misc, 64, "scratch words")) != SWH_OK)
        return s;
    if ((s = upload(ctx, offs_d, h_off.data(), h_off.size(), st, what)) != SWH_OK) return s;
    hipError_t e;
    const int32_t init = INT32_MAX;
    if ((total && (e = hipMemcpyAsync(raw.p, cat + base, (size_t)total, hipMemcpyHostToDevice, st)) != hipSuccess) ||
        (e = hipMemcpyAsync(ctx->lut.p, sc.lut, 256, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(ctx->misc.p, &init, 4, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = launch_encode((const char *)raw.p, total, (uint8_t *)codes.p, total, (const uint8_t *)ctx->lut.p,
                           (uint8_t)sc.asize, (int32_t *)ctx->misc.p, st)) != hipSuccess)
        return hip_fail(ctx, e, what);
    int32_t bad = 0;
    if ((e = hipMemcpyAsync(&bad, ctx->misc.p, 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, what);
    if (bad != INT32_MAX) {
        const int64_t i = (int64_t)(std::upper_bound(h_off.begin(), h_off.end(), (int64_t)bad) - h_off.begin()) - 1;
        return fail(ctx, SWH_E_ALPHABET, std::string(what) + " " + std::to_string(i) + ": byte at position " +
                                             std::to_string(bad - h_off[i]) + " is not in the alphabet");
    }
    return SWH_OK;
}

// Per-database feature rows: the inter-task slots in sorted order (empty
// slots included), then the long sequences.
swh_status ensure_db_features(swh_ctx *ctx, swh_db *db)
{
    if (db->pf_ready) return SWH_OK;
    hipStream_t st = ctx->own_stream;
    const int64_t nslots = (int64_t)db->h_perm.size(), nlong = (int64_t)db->long_idx.size();
    const int64_t nrows = nslots + nlong;
    db->h_row_db.assign((size_t)nrows, -1);
    db->h_row_len.assign((size_t)nrows, 0);
    std::vector<int32_t> dst_row((size_t)db->ndb, -1);
    for (int64_t r = 0; r < nrows; ++r) {
        const int32_t idx = r < nslots ? db->h_perm[r] : db->long_idx[r - nslots];
        db->h_row_db[r] = idx;
        if (idx >= 0) {
            db->h_row_len[r] = (int32_t)(db->h_off[idx + 1] - db->h_off[idx]);
            dst_row[idx] = (int32_t)r;
        }
    }
    swh_status s;
    hipError_t e;
    if ((s = ensure(ctx, db->pf_F, (size_t)std::max<int64_t>(nrows, 1) * kKPad * 2, "database features")) != SWH_OK ||
        (s = upload(ctx, db->pf_row_db, db->h_row_db.data(), db->h_row_db.size(), st, "row table")) != SWH_OK ||
        (s = upload(ctx, db->pf_row_len, db->h_row_len.data(), db->h_row_len.size(), st, "row lengths")) != SWH_OK ||
        (s = upload(ctx, ctx->tb_misc, dst_row.data(), dst_row.size(), st, "row map")) != SWH_OK)
        return s;
    if ((e = hipMemsetAsync(db->pf_F.p, 0, (size_t)std::max<int64_t>(nrows, 1) * kKPad * 2, st)) != hipSuccess ||
        (e = launch_dipeptides((const uint8_t *)db->codes.p, (const int64_t *)db->offs.p, db->ndb,
                               (const int32_t *)ctx->tb_misc.p, nullptr, nullptr, (uint16_t *)db->pf_F.p, nullptr,
                               st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, "database features");
    db->pf_nrows = nrows;
    db->pf_nslots = nslots;
    db->pf_ready = true;
    return SWH_OK;
}

// Predictions [nq][nrows] of encoded queries (prepare_queries) into ctx->pf_pred.
swh_status predict_rows(swh_ctx *ctx, const swh_model *m, swh_db *db, const QuerySet &qs, PrefilterStats *ps)
{
    hipStream_t st = ctx->own_stream;
    auto t0 = Clock::now();
    swh_status s;
    if ((s = ensure_db_features(ctx, db)) != SWH_OK) return s;
    const int nq = qs.nq;
    if ((s = ensure(ctx, ctx->pf_fq, (size_t)nq * kNDip * 4 + 16, "query features")) != SWH_OK ||
        (s = ensure(ctx, ctx->pf_qlen, (size_t)nq * 4 + 16, "query lengths")) != SWH_OK ||
        (s = ensure(ctx, ctx->pf_Aq, (size_t)nq * kNH * kKPad * 2 + 16, "folded queries")) != SWH_OK ||
        (s = ensure(ctx, ctx->pf_pred, (size_t)nq * db->pf_nrows * 4 + 16, "predictions")) != SWH_OK)
        return s;
    hipError_t e;
    if ((e = launch_dipeptides((const uint8_t *)ctx->qc.p, (const int64_t *)ctx->qoff.p, nq, nullptr, nullptr,
                               (float *)ctx->pf_fq.p, nullptr, (int32_t *)ctx->pf_qlen.p, st)) != hipSuccess ||
        (e = launch_fold_query((const float *)m->theta.p, (const float *)ctx->pf_fq.p, nq, (const float *)m->sd_d.p,
                               (uint16_t *)ctx->pf_Aq.p, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, "query features");
    if (ps) ps->ms_features += ms_since(t0);
    t0 = Clock::now();
    InferArgs a;
    a.F = (const uint16_t *)db->pf_F.p;
    a.row_len = (const int32_t *)db->pf_row_len.p;
    a.row_db = (const int32_t *)db->pf_row_db.p;
    a.nrows = db->pf_nrows;
    a.Aq = (const uint16_t *)ctx->pf_Aq.p;
    a.qlen = (const int32_t *)ctx->pf_qlen.p;
    a.nq = nq;
    a.cvec = (const float *)m->cvec.p;
    a.w1x = (const float *)m->w1x.p;
    a.mu400 = m->mu[kNDip];
    a.W2bf = (const uint16_t *)m->W2bf.p;
    a.theta = (const float *)m->theta.p;
    a.pred = (float *)ctx->pf_pred.p;
    hipEventRecord(ctx->ev[2], st);
    if ((e = launch_infer(a, st)) != hipSuccess) return hip_fail(ctx, e, "inference launch");
    hipEventRecord(ctx->ev[3], st);
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(ctx, e, "inference");
    float ms = 0.f;
    hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]);
    ctx->pf_infer_ms = ms;
    if (ps) ps->ms_predict += ms_since(t0);
    return SWH_OK;
}

// Order-preserving key of the n-th largest prediction of each query (radix
// select over 11 + 11 + 10 bits).
swh_status select_thresholds(swh_ctx *ctx, int nq, int64_t nrows, int64_t n, std::vector<uint32_t> &thr)
{
    hipStream_t st = ctx->own_stream;
    swh_status s;
    hipError_t e;
    if ((s = ensure(ctx, ctx->pf_hist, (size_t)nq * 2048 * 4 + 16, "histograms")) != SWH_OK ||
        (s = ensure(ctx, ctx->pf_prefix, (size_t)nq * 4 + 16, "prefixes")) != SWH_OK)
        return s;
    std::vector<uint32_t> prefix((size_t)nq, 0), hist((size_t)nq * 2048);
    std::vector<int64_t> need((size_t)nq, n);
    const int bits[3] = {11, 11, 10};
    for (int level = 0; level < 3; ++level) {
        if ((e = hipMemsetAsync(ctx->pf_hist.p, 0, (size_t)nq * 2048 * 4, st)) != hipSuccess ||
            (e = hipMemcpyAsync(ctx->pf_prefix.p, prefix.data(), (size_t)nq * 4, hipMemcpyHostToDevice, st)) !=
                hipSuccess ||
            (e = launch_key_hist((const float *)ctx->pf_pred.p, nrows, nq, level,
                                 level ? (const uint32_t *)ctx->pf_prefix.p : nullptr, (uint32_t *)ctx->pf_hist.p,
                                 st)) != hipSuccess ||
            (e = hipMemcpyAsync(hist.data(), ctx->pf_hist.p, (size_t)nq * 2048 * 4, hipMemcpyDeviceToHost, st)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess)
            return hip_fail(ctx, e, "radix select");
        for (int q = 0; q < nq; ++q) {
            int64_t acc = 0;
            int b = (1 << bits[level]) - 1;
            for (; b > 0; --b) {
                const int64_t c = hist[(size_t)q * 2048 + b];
                if (acc + c >= need[q]) break;
                acc += c;
            }
            need[q] -= acc;
            prefix[q] = (prefix[q] << bits[level]) | (uint32_t)b;
        }
    }
    thr = prefix;
    return SWH_OK;
}

}  // namespace

// ---------------------------------------------------------------- model handle

swh_status model_create(swh_ctx *ctx, const Scoring &sc, const float *theta, const float *mu, const float *sd,
                        uint64_t seed, swh_model **out)
{
    if (sc.asize < kNStd) return fail(ctx, SWH_E_INVAL, "the prefilter needs an alphabet of at least 20 symbols");
    swh_model *m = new (std::nothrow) swh_model();
    if (!m) return fail(ctx, SWH_E_NOMEM, "model handle");
    m->device = ctx->device;
    m->asize = sc.asize;
    swh_status s = model_alloc(ctx, m);
    std::vector<float> th, z(kNIn, 0.0f), one(kNIn, 1.0f);
    if (!theta) init_params(seed, th);
    if (s == SWH_OK) s = model_install(ctx, m, theta ? theta : th.data(), mu ? mu : z.data(), sd ? sd : one.data());
    if (s != SWH_OK) {
        model_destroy(m);
        return s;
    }
    *out = m;
    return SWH_OK;
}

void model_destroy(swh_model *m)
{
    if (!m) return;
    hipSetDevice(m->device);
    hipDeviceSynchronize();
    for (DevBuf *b : {&m->theta, &m->adam_m, &m->adam_v, &m->W1bf, &m->W2bf, &m->cvec, &m->w1x, &m->mu_d, &m->sd_d})
        free_buf(*b);
    delete m;
}

swh_status model_get(swh_ctx *ctx, const swh_model *m, float *theta, float *mu, float *sd)
{
    hipError_t e;
    if (theta && ((e = hipMemcpy(theta, m->theta.p, kNParams * 4, hipMemcpyDeviceToHost)) != hipSuccess))
        return hip_fail(ctx, e, "parameters");
    if (mu) std::memcpy(mu, m->mu.data(), kNIn * 4);
    if (sd) std::memcpy(sd, m->sd.data(), kNIn * 4);
    return SWH_OK;
}

swh_status model_set(swh_ctx *ctx, swh_model *m, const float *theta, const float *mu, const float *sd)
{
    std::vector<float> th(kNParams);
    if (!theta) {
        swh_status s = model_get(ctx, m, th.data(), nullptr, nullptr);
        if (s != SWH_OK) return s;
    }
    return model_install(ctx, m, theta ? theta : th.data(), mu ? mu : m->mu.data(), sd ? sd : m->sd.data());
}

namespace {
const char kMagic[8] = {'S', 'W', 'H', 'M', 'L', 'P', '0', '1'};
}

swh_status model_save(swh_ctx *ctx, const swh_model *m, const char *path)
{
    std::vector<float> th(kNParams);
    swh_status s = model_get(ctx, m, th.data(), nullptr, nullptr);
    if (s != SWH_OK) return s;
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(ctx, SWH_E_INVAL, std::string("cannot open ") + path + " for writing");
    const int32_t hdr[2] = {m->asize, (int32_t)kNParams};
    bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(hdr, 4, 2, f) == 2 &&
              std::fwrite(th.data(), 4, kNParams, f) == (size_t)kNParams &&
              std::fwrite(m->mu.data(), 4, kNIn, f) == (size_t)kNIn && std::fwrite(m->sd.data(), 4, kNIn, f) == (size_t)kNIn;
    ok = (std::fclose(f) == 0) && ok;
    return ok ? SWH_OK : fail(ctx, SWH_E_INVAL, std::string("write to ") + path + " failed");
}

swh_status model_load(swh_ctx *ctx, const char *path, swh_model **out)
{
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(ctx, SWH_E_INVAL, std::string("cannot open ") + path);
    char magic[8];
    int32_t hdr[2];
    std::vector<float> th(kNParams), mu(kNIn), sd(kNIn);
    const bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0 &&
                    std::fread(hdr, 4, 2, f) == 2 && hdr[1] == (int32_t)kNParams && hdr[0] >= kNStd && hdr[0] <= 32 &&
                    std::fread(th.data(), 4, kNParams, f) == (size_t)kNParams &&
                    std::fread(mu.data(), 4, kNIn, f) == (size_t)kNIn && std::fread(sd.data(), 4, kNIn, f) == (size_t)kNIn;
    std::fclose(f);
    if (!ok) return fail(ctx, SWH_E_INVAL, std::string(path) + " is not a prefilter model file");
    Scoring sc;
    sc.asize = hdr[0];
    return model_create(ctx, sc, th.data(), mu.data(), sd.data(), 0, out);
}

// ---------------------------------------------------------------- training

swh_status dipeptide_counts(swh_ctx *ctx, const Scoring &sc, int64_t nseq, const char *cat, const int64_t *off,
                            int32_t *counts)
{
    hipStream_t st = ctx->own_stream;
    std::vector<int64_t> h_off;
    DevBuf raw, codes, offs, cnt;
    swh_status s = encode_pool(ctx, sc, nseq, cat, off, raw, codes, offs, h_off, "sequence");
    if (s == SWH_OK) s = ensure(ctx, cnt, (size_t)std::max<int64_t>(nseq, 1) * kNDip * 4, "counts");
    hipError_t e = hipSuccess;
    if (s == SWH_OK && nseq > 0 &&
        ((e = launch_dipeptides((const uint8_t *)codes.p, (const int64_t *)offs.p, nseq, nullptr, (int32_t *)cnt.p,
                                nullptr, nullptr, nullptr, st)) != hipSuccess ||
         (e = hipMemcpyAsync(counts, cnt.p, (size_t)nseq * kNDip * 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
         (e = hipStreamSynchronize(st)) != hipSuccess))
        s = hip_fail(ctx, e, "dipeptide counts");
    for (DevBuf *b : {&raw, &codes, &offs, &cnt}) free_buf(*b);
    return s;
}

swh_status mlp_grad(swh_ctx *ctx, swh_model *m, int32_t B, const float *z, const float *y, double *loss, float *grad)
{
    hipStream_t st = ctx->own_stream;
    TrainWs w;
    DevBuf zf;
    swh_status s = ws_alloc(ctx, w, B);
    if (s == SWH_OK) s = upload(ctx, zf, z, (size_t)B * kNIn, st, "inputs");
    if (s != SWH_OK) {
        free_buf(zf);
        return s;
    }
    hipError_t e;
    double lsum = 0.0;
    if ((e = hipMemcpyAsync(w.yb.p, y, (size_t)B * 4, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemsetAsync(w.loss, 0, 8, st)) != hipSuccess ||
        (e = launch_z_to_bf16((const float *)zf.p, B, (uint16_t *)w.Xb.p, st)) != hipSuccess ||
        (e = forward_backward(m, w, B, st)) != hipSuccess ||
        (e = hipMemcpyAsync(grad, w.grad.p, kNParams * 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipMemcpyAsync(&lsum, w.loss, 8, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        s = hip_fail(ctx, e, "gradient");
    free_buf(zf);
    if (loss) *loss = lsum / B;
    return s;
}

swh_status mlp_train_steps(swh_ctx *ctx, swh_model *m, int32_t B, const float *z, const float *y, int32_t steps,
                           double lr)
{
    hipStream_t st = ctx->own_stream;
    TrainWs w;
    DevBuf zf;
    swh_status s = ws_alloc(ctx, w, B);
    if (s == SWH_OK) s = upload(ctx, zf, z, (size_t)B * kNIn, st, "inputs");
    hipError_t e = hipSuccess;
    if (s == SWH_OK && ((e = hipMemcpyAsync(w.yb.p, y, (size_t)B * 4, hipMemcpyHostToDevice, st)) != hipSuccess ||
                        (e = launch_z_to_bf16((const float *)zf.p, B, (uint16_t *)w.Xb.p, st)) != hipSuccess))
        s = hip_fail(ctx, e, "inputs");
    for (int32_t i = 0; s == SWH_OK && i < steps; ++i)
        if ((e = hipMemsetAsync(w.loss, 0, 8, st)) != hipSuccess || (e = forward_backward(m, w, B, st)) != hipSuccess ||
            (e = adam_update(m, w, lr, st)) != hipSuccess)
            s = hip_fail(ctx, e, "training step");
    if (s == SWH_OK && ((e = refresh_fold(m, st)) != hipSuccess || (e = hipStreamSynchronize(st)) != hipSuccess))
        s = hip_fail(ctx, e, "training steps");
    free_buf(zf);
    return s;
}

swh_status prefilter_train(swh_ctx *ctx, const Scoring &sc, int64_t nseq, const char *cat, const int64_t *off,
                           int64_t npairs, const int32_t *rows, const int32_t *cols, const int32_t *scores,
                           int32_t epochs, int32_t batch, double lr, uint64_t seed, swh_model *model,
                           int32_t *labels_out, TrainStats &ts)
{
    hipStream_t st = ctx->own_stream;
    swh_status s;
    hipError_t e;
    for (int64_t p = 0; p < npairs; ++p)
        if (rows[p] < 0 || rows[p] >= nseq || cols[p] < 0 || cols[p] >= nseq)
            return fail(ctx, SWH_E_INVAL, "pair " + std::to_string(p) + " indexes outside the sequence pool");
    auto t0 = Clock::now();
    std::vector<int64_t> h_off;
    DevBuf raw, codes, offs, freq, lens, drows, dcols, Z, y, lab, statbuf, perm;
    struct Free {
        std::vector<DevBuf *> v;
        ~Free()
        {
            for (DevBuf *b : v) free_buf(*b);
        }
    } guard{{&raw, &codes, &offs, &freq, &lens, &drows, &dcols, &Z, &y, &lab, &statbuf, &perm}};
    if ((s = encode_pool(ctx, sc, nseq, cat, off, raw, codes, offs, h_off, "sequence")) != SWH_OK) return s;

    // ---- labels: exact local scores of every pair (or the caller's)
    std::vector<int32_t> labels((size_t)npairs);
    if (scores) {
        std::copy(scores, scores + npairs, labels.begin());
    } else {
        if (ctx->mat.cap < 1024 && (s = ensure(ctx, ctx->mat, 1024, "matrix")) != SWH_OK) return s;
        if ((e = hipMemcpyAsync(ctx->mat.p, sc.mat, (size_t)sc.asize * sc.asize, hipMemcpyHostToDevice, st)) !=
            hipSuccess)
            return hip_fail(ctx, e, "matrix upload");
        std::vector<PairPass> ps((size_t)npairs);
        const uint8_t *c = (const uint8_t *)codes.p;
        for (int64_t p = 0; p < npairs; ++p) {
            const int32_t r = rows[p], q = cols[p];
            ps[p] = PairPass{c + h_off[r], h_off[r + 1] - h_off[r], c + h_off[q], h_off[q + 1] - h_off[q], 1};
            ts.cells_label += (double)ps[p].n * (double)ps[p].m;
            const int64_t sabs = std::max(1, std::max(sc.smax, -sc.smin));
            if (std::min(ps[p].n, ps[p].m) * sabs >= ((int64_t)1 << 26))
                return fail(ctx, SWH_E_RANGE, "pair " + std::to_string(p) + " is too long to label");
        }
        std::vector<BestCell> best;
        double ms = 0.0;
        if ((s = score_passes(ctx, ps, sc, st, best, ms)) != SWH_OK) return s;
        for (int64_t p = 0; p < npairs; ++p) labels[p] = best[p].score;
    }
    if (labels_out) std::copy(labels.begin(), labels.end(), labels_out);
    ts.ms_label = ms_since(t0);

    // ---- features: frequencies per sequence, statistics and normalised rows per pair
    t0 = Clock::now();
    if ((s = ensure(ctx, freq, (size_t)std::max<int64_t>(nseq, 1) * kNDip * 4, "frequencies")) != SWH_OK ||
        (s = ensure(ctx, lens, (size_t)std::max<int64_t>(nseq, 1) * 4, "lengths")) != SWH_OK ||
        (s = upload(ctx, drows, rows, (size_t)npairs, st, "pairs")) != SWH_OK ||
        (s = upload(ctx, dcols, cols, (size_t)npairs, st, "pairs")) != SWH_OK ||
        (s = upload(ctx, lab, labels.data(), labels.size(), st, "labels")) != SWH_OK ||
        (s = ensure(ctx, Z, (size_t)npairs * kKPad * 2 + 16, "training inputs")) != SWH_OK ||
        (s = ensure(ctx, y, (size_t)npairs * 4 + 16, "training targets")) != SWH_OK ||
        (s = ensure(ctx, statbuf, sizeof(double) * 2 * kNIn * 1026, "feature statistics")) != SWH_OK)
        return s;
    std::vector<double> sums(2 * kNIn);
    if ((e = launch_dipeptides((const uint8_t *)codes.p, (const int64_t *)offs.p, nseq, nullptr, nullptr,
                               (float *)freq.p, nullptr, (int32_t *)lens.p, st)) != hipSuccess ||
        (e = launch_pair_stats((const float *)freq.p, (const int32_t *)lens.p, (const int32_t *)drows.p,
                               (const int32_t *)dcols.p, npairs, (double *)statbuf.p, (double *)statbuf.p + kNIn,
                               st)) != hipSuccess ||
        (e = hipMemcpyAsync(sums.data(), statbuf.p, sizeof(double) * 2 * kNIn, hipMemcpyDeviceToHost, st)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, "feature statistics");
    std::vector<float> mu(kNIn), sd(kNIn);
    for (int k = 0; k < kNIn; ++k) {
        const double mean = sums[k] / (double)npairs;
        const double var = std::max(0.0, sums[kNIn + k] / (double)npairs - mean * mean);
        mu[k] = (float)mean;
        sd[k] = var > 0.0 ? (float)std::sqrt(var) : 1.0f;
    }
    std::vector<float> th(kNParams);
    if ((s = model_get(ctx, model, th.data(), nullptr, nullptr)) != SWH_OK ||
        (s = model_install(ctx, model, th.data(), mu.data(), sd.data())) != SWH_OK)
        return s;
    if ((e = launch_pair_z((const float *)freq.p, (const int32_t *)lens.p, (const int32_t *)drows.p,
                           (const int32_t *)dcols.p, npairs, (const float *)model->mu_d.p,
                           (const float *)model->sd_d.p, (uint16_t *)Z.p, st)) != hipSuccess ||
        (e = launch_labels((const int32_t *)lab.p, npairs, (float *)y.p, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, "training inputs");
    ts.ms_features = ms_since(t0);

    // ---- Adam over shuffled batches (the incomplete last batch of an epoch is dropped)
    t0 = Clock::now();
    TrainWs w;
    if ((s = ws_alloc(ctx, w, batch)) != SWH_OK) return s;
    if ((s = ensure(ctx, perm, (size_t)npairs * 4 + 16, "batch order")) != SWH_OK) return s;
    const int64_t nb = npairs / batch;
    std::vector<int32_t> order((size_t)npairs);
    uint64_t rs = seed ^ 0x5eedf00dull;
    // One step = gather, forward, backward, Adam, bf16 copies, counter bump.
    // It is captured once in a HIP graph and replayed: the batch index and
    // the Adam step live in device counters, so every replay is identical.
    DevBuf ctrbuf;
    guard.v.push_back(&ctrbuf);
    if ((s = ensure(ctx, ctrbuf, 64, "step counters")) != SWH_OK) return s;
    int32_t *ctr = (int32_t *)ctrbuf.p;
    const int32_t ctr0[2] = {0, (int32_t)model->steps};
    if ((e = hipMemcpyAsync(ctr, ctr0, 8, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, "step counters");
    auto step = [&](hipStream_t s2) -> hipError_t {
        hipError_t e2;
        if ((e2 = launch_gather_rows((const uint16_t *)Z.p, (const float *)y.p, (const int32_t *)perm.p, ctr, batch,
                                     (uint16_t *)w.Xb.p, (float *)w.yb.p, s2)) != hipSuccess ||
            (e2 = forward_backward(model, w, batch, s2)) != hipSuccess ||
            (e2 = adam_update(model, w, lr, s2, ctr)) != hipSuccess)
            return e2;
        return launch_step_end(ctr, s2);
    };
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (nb > 0 && ctx->opt.graph != 0) {
        if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            const hipError_t ce = step(st);
            const hipError_t ee = hipStreamEndCapture(st, &graph);
            if (ce != hipSuccess || ee != hipSuccess || !graph ||
                hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
                if (graph) hipGraphDestroy(graph);
                graph = nullptr;
                exec = nullptr;
            }
        }
        (void)hipGetLastError();
    }
    struct GraphGuard {
        hipGraph_t &g;
        hipGraphExec_t &x;
        ~GraphGuard()
        {
            if (x) hipGraphExecDestroy(x);
            if (g) hipGraphDestroy(g);
        }
    } gguard{graph, exec};
    ts.graph = exec != nullptr;
    for (int32_t ep = 0; ep < epochs; ++ep) {
        std::iota(order.begin(), order.end(), 0);
        for (int64_t i = npairs - 1; i > 0; --i) std::swap(order[i], order[splitmix(rs) % (uint64_t)(i + 1)]);
        if ((e = hipMemcpyAsync(perm.p, order.data(), (size_t)npairs * 4, hipMemcpyHostToDevice, st)) != hipSuccess ||
            (e = hipMemsetAsync(w.loss, 0, 8, st)) != hipSuccess || (e = hipMemsetAsync(ctr, 0, 4, st)) != hipSuccess)
            return hip_fail(ctx, e, "epoch setup");
        for (int64_t b = 0; b < nb; ++b) {
            if (cancelled(ctx)) {
                (void)hipStreamSynchronize(st);
                return cancel_status(ctx);
            }
            if ((e = exec ? hipGraphLaunch(exec, st) : step(st)) != hipSuccess) return hip_fail(ctx, e, "training step");
            ++ts.steps;
            ++model->steps;
        }
        double lsum = 0.0;
        if ((e = hipMemcpyAsync(&lsum, w.loss, 8, hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess)
            return hip_fail(ctx, e, "epoch loss");
        const double l = nb ? lsum / (double)(nb * batch) : 0.0;
        if (ep == 0) ts.first_loss = l;
        ts.final_loss = l;
    }
    if ((e = refresh_fold(model, st)) != hipSuccess || (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, "training");
    ts.ms_train = ms_since(t0);
    return SWH_OK;
}

// ---------------------------------------------------------------- search

swh_status prefilter_predict(swh_ctx *ctx, const swh_model *m, swh_db *db, int32_t nq, const char *q_cat,
                             const int64_t *q_off, float *pred)
{
    if (nq == 0 || db->ndb == 0) return SWH_OK;
    QuerySet qs;
    swh_status s = prepare_queries(ctx, db->sc, nq, q_cat, q_off, qs);
    if (s != SWH_OK) return s;
    if ((s = predict_rows(ctx, m, db, qs, nullptr)) != SWH_OK) return s;
    const int64_t nrows = db->pf_nrows;
    std::vector<float> h((size_t)nq * nrows);
    hipError_t e;
    if ((e = hipMemcpy(h.data(), ctx->pf_pred.p, h.size() * 4, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(ctx, e, "predictions");
    for (int32_t q = 0; q < nq; ++q)
        for (int64_t r = 0; r < nrows; ++r)
            if (db->h_row_db[r] >= 0) pred[(int64_t)q * db->ndb + db->h_row_db[r]] = h[(size_t)q * nrows + r];
    return SWH_OK;
}

swh_status prefilter_search(swh_ctx *ctx, const swh_model *m, swh_db *db, int32_t nq, const char *q_cat,
                            const int64_t *q_off, int32_t k, double rescore_frac, double audit_frac,
                            uint64_t audit_seed, swh_hit *hits, PrefilterStats &ps)
{
    hipStream_t st = ctx->own_stream;
    swh_status s;
    hipError_t e;
    if (nq == 0) return SWH_OK;
    if (db->ndb == 0) {
        for (int64_t i = 0; i < (int64_t)nq * k; ++i) hits[i] = swh_hit{-1, -1, 0};
        return SWH_OK;
    }
    QuerySet qs;
    if ((s = prepare_queries(ctx, db->sc, nq, q_cat, q_off, qs)) != SWH_OK) return s;
    if ((s = predict_rows(ctx, m, db, qs, &ps)) != SWH_OK) return s;
    const int64_t nrows = db->pf_nrows, ndb = db->ndb;

    // ---- candidates: predictions (or their excess over the mean of sequences
    // of the same length) at or above each query's n-th largest
    auto t0 = Clock::now();
    if (ctx->opt.pf_rank > 0 &&
        (e = launch_excess((float *)ctx->pf_pred.p, nrows, nq, (const int32_t *)db->pf_row_db.p, ctx->opt.pf_rank == 2,
                           st)) != hipSuccess)
        return hip_fail(ctx, e, "length-group excess");
    const int64_t want = std::min<int64_t>(ndb, std::max<int64_t>(k, (int64_t)std::ceil(rescore_frac * (double)ndb)));
    std::vector<uint32_t> thr;
    if ((s = select_thresholds(ctx, nq, nrows, want, thr)) != SWH_OK) return s;
    const int64_t nchunks = (nrows + kMarkChunk - 1) / kMarkChunk;
    const uint32_t audit_thr = (uint32_t)std::min(4294967295.0, std::floor(audit_frac * 4294967296.0));
    if ((s = ensure(ctx, ctx->pf_marks, (size_t)nq * nrows + 16, "marks")) != SWH_OK ||
        (s = ensure(ctx, ctx->pf_chunk, (size_t)nq * nchunks * 8 + 16, "chunk counts")) != SWH_OK ||
        (s = upload(ctx, ctx->pf_prefix, thr.data(), thr.size(), st, "thresholds")) != SWH_OK)
        return s;
    std::vector<int32_t> cc((size_t)nq * nchunks);
    if ((e = launch_mark((const float *)ctx->pf_pred.p, nrows, nq, (const uint32_t *)ctx->pf_prefix.p,
                         (const int32_t *)db->pf_row_db.p, audit_seed, audit_thr, (uint8_t *)ctx->pf_marks.p,
                         (int32_t *)ctx->pf_chunk.p, st)) != hipSuccess ||
        (e = hipMemcpyAsync(cc.data(), ctx->pf_chunk.p, cc.size() * 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, "marks");
    std::vector<int64_t> base(cc.size()), qbase((size_t)nq + 1, 0);
    int64_t tot = 0;
    for (int32_t q = 0; q < nq; ++q) {
        qbase[q] = tot;
        for (int64_t c = 0; c < nchunks; ++c) {
            base[(size_t)q * nchunks + c] = tot;
            tot += cc[(size_t)q * nchunks + c];
        }
    }
    qbase[nq] = tot;
    std::vector<int32_t> crow((size_t)tot);
    std::vector<uint8_t> ckind((size_t)tot);
    if ((s = upload(ctx, ctx->pf_chunk, base.data(), base.size(), st, "chunk offsets")) != SWH_OK ||
        (s = ensure(ctx, ctx->pf_cand, (size_t)tot * 5 + 16, "candidates")) != SWH_OK)
        return s;
    int32_t *dcrow = (int32_t *)ctx->pf_cand.p;
    uint8_t *dckind = (uint8_t *)(dcrow + tot);
    if ((e = launch_compact((const uint8_t *)ctx->pf_marks.p, nrows, nq, (const int64_t *)ctx->pf_chunk.p, dcrow,
                            dckind, st)) != hipSuccess ||
        (tot && (e = hipMemcpyAsync(crow.data(), dcrow, (size_t)tot * 4, hipMemcpyDeviceToHost, st)) != hipSuccess) ||
        (tot && (e = hipMemcpyAsync(ckind.data(), dckind, (size_t)tot, hipMemcpyDeviceToHost, st)) != hipSuccess) ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, "compaction");

    // ---- rescoring units: per query, its candidate slots in groups of 128
    //      (slots are length-sorted already) and its long candidates as pairs
    std::vector<DbGroup> groups;
    std::vector<int32_t> gperm;
    gperm.reserve((size_t)tot + 128 * (size_t)nq);
    std::vector<DbWork> work;
    std::vector<std::pair<int32_t, int32_t>> long_pairs;
    std::vector<std::vector<int32_t>> audit_idx((size_t)nq);   // sorted after the loop
    std::vector<int64_t> ncand((size_t)nq, 0);
    int64_t res_bytes = 0;
    for (int32_t q = 0; q < nq; ++q) {
        const int64_t Lq = qs.qo[q + 1] - qs.qo[q];
        const size_t first_slot = gperm.size();
        for (int64_t i = qbase[q]; i < qbase[q + 1]; ++i) {
            const int32_t r = crow[i];
            const int32_t idx = db->h_row_db[r];
            if (ckind[i] == 1) {
                ++ncand[q];
            } else {
                audit_idx[q].push_back(idx);
            }
            ps.cells_rescored += (double)Lq * (double)db->h_row_len[r];
            if (Lq == 0) continue;
            if (r < db->pf_nslots) {
                gperm.push_back(idx);
            } else {
                long_pairs.push_back({q, idx});
            }
        }
        ps.candidates += ncand[q];
        ps.audited += (int64_t)audit_idx[q].size();
        std::sort(audit_idx[q].begin(), audit_idx[q].end());
        // groups of 128 slots; slots are in ascending length, so a group's
        // longest member is its last one
        const size_t nslot = gperm.size() - first_slot;
        for (size_t i = 0; i < nslot; i += 128) {
            const size_t last = std::min(nslot, i + 128) - 1;
            const int32_t idx_last = gperm[first_slot + last];
            const int32_t maxlen = (int32_t)(db->h_off[idx_last + 1] - db->h_off[idx_last]);
            work.push_back(DbWork{q, (int32_t)groups.size()});
            groups.push_back(DbGroup{res_bytes, maxlen, (int32_t)(first_slot + i)});
            res_bytes += (int64_t)maxlen * 128;
        }
        gperm.resize(first_slot + (nslot + 127) / 128 * 128, -1);
        ps.cells_exhaustive += (double)Lq * (double)db->total_residues;
    }
    if ((s = ensure(ctx, ctx->pf_res, (size_t)res_bytes + 256, "candidate layout")) != SWH_OK ||
        (s = upload(ctx, ctx->pf_groups, groups.data(), groups.size(), st, "candidate groups")) != SWH_OK ||
        (s = upload(ctx, ctx->pf_perm, gperm.data(), gperm.size(), st, "candidate order")) != SWH_OK ||
        (s = ensure(ctx, ctx->db_scores, sizeof(int32_t) * (size_t)std::max<int64_t>(1, (int64_t)nq * ndb) + 64,
                    "score matrix")) != SWH_OK)
        return s;
    if ((!groups.empty() &&
         (e = launch_db_pack((const uint8_t *)db->codes.p, (const int64_t *)db->offs.p,
                             (const int32_t *)ctx->pf_perm.p, (const DbGroup *)ctx->pf_groups.p,
                             (int32_t)groups.size(), (uint8_t)db->sc.asize, (uint8_t *)ctx->pf_res.p, st)) !=
             hipSuccess) ||
        (e = launch_fill_i32((int32_t *)ctx->db_scores.p, (int64_t)nq * ndb, -1, st)) != hipSuccess)
        return hip_fail(ctx, e, "candidate layout");
    // an empty query aligns with nothing: every score is 0, as in the exhaustive search
    for (int32_t q = 0; q < nq; ++q)
        if (qs.qo[q + 1] == qs.qo[q] &&
            (e = launch_fill_i32((int32_t *)ctx->db_scores.p + (int64_t)q * ndb, ndb, 0, st)) != hipSuccess)
            return hip_fail(ctx, e, "score fill");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(ctx, e, "candidate layout");
    ps.ms_select += ms_since(t0);

    t0 = Clock::now();
    int32_t *scores = (int32_t *)ctx->db_scores.p;
    DbStats ds;
    GroupSet gs{(const uint8_t *)ctx->pf_res.p, (const DbGroup *)ctx->pf_groups.p, (const int32_t *)ctx->pf_perm.p,
                &groups};
    if ((s = score_units(ctx, db, qs, gs, std::move(work), long_pairs, scores, ds)) != SWH_OK) return s;
    ps.ms_rescore += ms_since(t0);

    // ---- top-k, audit, fallback
    auto topk = [&](std::vector<int64_t> &hi, std::vector<int32_t> &hs) -> swh_status {
        t0 = Clock::now();
        const size_t cand = topk_scratch_entries(nq, ndb, k);
        swh_status s2 = ensure(ctx, ctx->db_topk, cand * 8 + (size_t)nq * k * 12 + 256, "top-k scratch");
        if (s2 != SWH_OK) return s2;
        int32_t *cidx = (int32_t *)ctx->db_topk.p;
        int32_t *cscore = cidx + cand;
        int64_t *oidx = (int64_t *)(((uintptr_t)(cscore + cand) + 15) & ~(uintptr_t)15);
        int32_t *oscore = (int32_t *)(oidx + (size_t)nq * k);
        hi.resize((size_t)nq * k);
        hs.resize((size_t)nq * k);
        hipError_t e2;
        if ((e2 = launch_topk(scores, nq, ndb, k, cidx, cscore, oidx, oscore, st)) != hipSuccess ||
            (e2 = hipMemcpyAsync(hi.data(), oidx, sizeof(int64_t) * hi.size(), hipMemcpyDeviceToHost, st)) !=
                hipSuccess ||
            (e2 = hipMemcpyAsync(hs.data(), oscore, sizeof(int32_t) * hs.size(), hipMemcpyDeviceToHost, st)) !=
                hipSuccess ||
            (e2 = hipStreamSynchronize(st)) != hipSuccess)
            return hip_fail(ctx, e2, "top-k");
        ps.ms_topk += ms_since(t0);
        return SWH_OK;
    };
    std::vector<int64_t> hi;
    std::vector<int32_t> hs;
    if (nq > 0 && (s = topk(hi, hs)) != SWH_OK) return s;
    std::vector<int32_t> fb;
    for (int32_t q = 0; q < nq; ++q) {
        if (qs.qo[q + 1] == qs.qo[q]) continue;
        bool need = ncand[q] < std::min<int64_t>(k, ndb);
        for (int32_t j = 0; j < k && !need; ++j) {
            const int64_t idx = hi[(size_t)q * k + j];
            if (idx >= 0 && std::binary_search(audit_idx[q].begin(), audit_idx[q].end(), (int32_t)idx)) need = true;
        }
        if (need) fb.push_back(q);
    }
    if (!fb.empty()) {
        t0 = Clock::now();
        ps.fallbacks = (int64_t)fb.size();
        std::vector<DbWork> fw;
        std::vector<std::pair<int32_t, int32_t>> flong;
        for (int32_t q : fb) {
            for (size_t g = 0; g < db->h_groups.size(); ++g) fw.push_back(DbWork{q, (int32_t)g});
            for (int32_t d : db->long_idx) flong.push_back({q, d});
        }
        GroupSet all{(const uint8_t *)db->res.p, (const DbGroup *)db->groups.p, (const int32_t *)db->perm.p,
                     &db->h_groups};
        if ((s = score_units(ctx, db, qs, all, std::move(fw), flong, scores, ds)) != SWH_OK) return s;
        ps.ms_fallback += ms_since(t0);
        if ((s = topk(hi, hs)) != SWH_OK) return s;
    }
    for (size_t i = 0; i < hi.size(); ++i) {
        hits[i].db_index = hi[i];
        hits[i].score = hi[i] >= 0 ? hs[i] : -1;
        hits[i].reserved = 0;
    }
    return SWH_OK;
}

}  // namespace swh
