// tune.hip -- launch shapes of the batched paths, picked by measurement.
//
// Two shapes are tuned on the caller's own workload:
//   train_threads    workgroup of the large-cluster trainer (256, 512, 1024
//                    threads); the LDS footprint keeps one workgroup per CU,
//                    so more threads trade barrier cost for parallel work in
//                    each elimination step.
//   eval_persistent  the FP32/FP64 evaluation either launches one wavefront
//                    per 64-query chunk (0) or keeps 1, 2 or 4 persistent
//                    wavefronts per SIMD taking chunks from a counter.
// Each candidate runs three times after one warm-up run; the median of the
// HIP-event times on the context stream decides.
#include "gpdf_internal.hpp"

#include <algorithm>
#include <vector>

using namespace gpdf;

namespace {

const int kTrainCand[] = {256, 512, 1024};
const int kEvalCand[] = {0, 1, 2, 4};

template <class F>
gpdf_status time_median(gpdf_ctx *c, F &&call, float *ms) {
    hipEvent_t a, b;
    hipError_t e;
    if ((e = hipEventCreate(&a)) != hipSuccess) return hip_fail(c, e, "autotune: event");
    if ((e = hipEventCreate(&b)) != hipSuccess) {
        (void)hipEventDestroy(a);
        return hip_fail(c, e, "autotune: event");
    }
    std::vector<float> t;
    gpdf_status st = GPDF_OK;
    for (int rep = 0; rep < 4 && st == GPDF_OK; ++rep) {
        (void)hipEventRecord(a, c->stream);
        st = call();
        (void)hipEventRecord(b, c->stream);
        if (st != GPDF_OK) break;
        if ((e = hipEventSynchronize(b)) != hipSuccess) {
            st = hip_fail(c, e, "autotune: sync");
            break;
        }
        float x = 0.f;
        (void)hipEventElapsedTime(&x, a, b);
        if (rep > 0) t.push_back(x);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != GPDF_OK) return st;
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
    return GPDF_OK;
}

}  // namespace

extern "C" gpdf_status gpdf_set_tuning(gpdf_ctx *c, int32_t train_threads, int32_t eval_persistent) {
    if (!c) return GPDF_E_INVALID_ARG;
    if (std::find(std::begin(kTrainCand), std::end(kTrainCand), train_threads) == std::end(kTrainCand) ||
        std::find(std::begin(kEvalCand), std::end(kEvalCand), eval_persistent) == std::end(kEvalCand))
        return fail(c, GPDF_E_INVALID_ARG, "set_tuning: train_threads 256/512/1024, eval_persistent 0/1/2/4");
    c->tune.train_threads = train_threads;
    c->tune.eval_persistent = eval_persistent;
    return GPDF_OK;
}

extern "C" gpdf_status gpdf_get_tuning(const gpdf_ctx *c, int32_t *train_threads, int32_t *eval_persistent) {
    if (!c) return GPDF_E_INVALID_ARG;
    if (train_threads) *train_threads = c->tune.train_threads;
    if (eval_persistent) *eval_persistent = c->tune.eval_persistent;
    return GPDF_OK;
}

extern "C" gpdf_status gpdf_autotune(gpdf_ctx *c, const float *d_xyz, int64_t n, const float *d_q, int64_t m,
                                     const float *h_origin, float *h_ms) {
    if (!c) return GPDF_E_INVALID_ARG;
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "join");
    if (n < 1 || !d_xyz || m < 1 || !d_q) return fail(c, GPDF_E_INVALID_ARG, "autotune: empty or null input");
    if (m > c->p.max_queries) return fail(c, GPDF_E_CAPACITY, "autotune: m exceeds max_queries");
    float ms[7] = {};
    try {
        int best_t = c->tune.train_threads;
        float best = 0.f;
        for (int i = 0; i < 3; ++i) {
            c->tune.train_threads = kTrainCand[i];
            gpdf_status st = time_median(c, [&] {
                // the timed region covers the large-cluster trainer too
                const gpdf_status ts = train(c, d_xyz, n);
                (void)join_train(c);
                return ts;
            }, &ms[i]);
            if (st != GPDF_OK) return st;
            if (i == 0 || ms[i] < best) { best = ms[i]; best_t = kTrainCand[i]; }
        }
        c->tune.train_threads = best_t;
        gpdf_status st = train(c, d_xyz, n);
        if (st != GPDF_OK) return st;
        int best_p = c->tune.eval_persistent;
        for (int i = 0; i < 4; ++i) {
            c->tune.eval_persistent = kEvalCand[i];
            st = time_median(c, [&] {
                return query(c, d_q, m, h_origin, c->d_tmp_dist, c->d_tmp_grad, c->d_tmp_var, c->d_tmp_valid,
                             nullptr, 0);
            }, &ms[3 + i]);
            if (st != GPDF_OK) return st;
            if (i == 0 || ms[3 + i] < best) { best = ms[3 + i]; best_p = kEvalCand[i]; }
        }
        c->tune.eval_persistent = best_p;
        c->tune.tuned = 1;
    } catch (...) {
        return fail(c, GPDF_E_OOM, "autotune: host allocation failed");
    }
    if (h_ms) std::copy(ms, ms + 7, h_ms);
    return GPDF_OK;
}
