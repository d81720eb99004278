// prefilter.h -- the learned prefilter: model handle, training, inference,
// candidate selection and exact rescoring (prefilter.cpp).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "context.h"

struct swh_model {
    int device = 0;
    int asize = 0;                    // alphabet size of the scoring it was built for
    std::vector<float> mu, sd;        // feature normalisation (401 each)
    swh::DevBuf theta, adam_m, adam_v, W1bf, W2bf, cvec, w1x, mu_d, sd_d;
    int64_t steps = 0;                // Adam steps taken
};

namespace swh {

swh_status model_create(swh_ctx *ctx, const Scoring &sc, const float *theta, const float *mu, const float *sd,
                        uint64_t seed, swh_model **out);
void model_destroy(swh_model *m);
swh_status model_get(swh_ctx *ctx, const swh_model *m, float *theta, float *mu, float *sd);
swh_status model_set(swh_ctx *ctx, swh_model *m, const float *theta, const float *mu, const float *sd);
swh_status model_save(swh_ctx *ctx, const swh_model *m, const char *path);
swh_status model_load(swh_ctx *ctx, const char *path, swh_model **out);

struct TrainStats {
    double first_loss = 0.0, final_loss = 0.0;
    double ms_label = 0.0, ms_features = 0.0, ms_train = 0.0;
    double cells_label = 0.0;
    int64_t steps = 0;
    bool graph = false;   // the step ran as a replayed HIP graph
};
swh_status prefilter_train(swh_ctx *ctx, const Scoring &sc, int64_t nseq, const char *cat, const int64_t *off,
                           int64_t npairs, const int32_t *rows, const int32_t *cols, const int32_t *scores,
                           int32_t epochs, int32_t batch, double lr, uint64_t seed, swh_model *model,
                           int32_t *labels_out, TrainStats &ts);

// One forward and backward pass of a batch of normalised inputs z [B][401].
swh_status mlp_grad(swh_ctx *ctx, swh_model *m, int32_t B, const float *z, const float *y, double *loss,
                    float *grad);
// Adam steps on one fixed batch.
swh_status mlp_train_steps(swh_ctx *ctx, swh_model *m, int32_t B, const float *z, const float *y, int32_t steps,
                           double lr);

swh_status dipeptide_counts(swh_ctx *ctx, const Scoring &sc, int64_t nseq, const char *cat, const int64_t *off,
                            int32_t *counts);

struct PrefilterStats {
    int64_t candidates = 0, audited = 0, fallbacks = 0;
    double cells_rescored = 0.0, cells_exhaustive = 0.0;
    double ms_features = 0.0, ms_predict = 0.0, ms_select = 0.0, ms_rescore = 0.0, ms_topk = 0.0,
           ms_fallback = 0.0;
};
swh_status prefilter_predict(swh_ctx *ctx, const swh_model *m, swh_db *db, int32_t nq, const char *q_cat,
                             const int64_t *q_off, float *pred);
swh_status prefilter_search(swh_ctx *ctx, const swh_model *m, swh_db *db, int32_t nq, const char *q_cat,
                            const int64_t *q_off, int32_t k, double rescore_frac, double audit_frac,
                            uint64_t audit_seed, swh_hit *hits, PrefilterStats &ps);

}  // namespace swh
