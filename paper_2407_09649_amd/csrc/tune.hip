// tune.hip -- launch shapes of the batched paths, picked by measurement and
// cached by workload shape.
//
// Three shapes are tuned on the caller's own workload:
//   train_threads    workgroup of the trainer of the clusters above 256 points
//                    (256, 512, 1024 threads).
//   eval_persistent  the FP32/FP64 evaluation either launches one wavefront
//                    per 64-query chunk (0) or keeps 1, 2 or 4 persistent
//                    wavefronts per SIMD taking chunks from a counter.
//   mfma_min_n       the size bucket boundary of the FP32 evaluation: the
//                    clusters of at least mfma_min_n (17, 33, 65 or 129) up
//                    to 248 points take the variance product W k on FP32
//                    MFMA, the smaller ones the VALU path; 0 keeps every
//                    cluster on the VALU path.
// Each candidate runs three times after one warm-up run; the median of the
// HIP-event times on the context stream decides.
//
// The result is kept in a process-wide cache keyed by the workload shape: the
// precision, selection, kernel and clustering mode, the histogram of cluster
// sizes over the buckets 1-8, 9-16, 17-32, 33-64, 65-128, 129-256 and above
// (each count rounded to the nearest power of two), and the query count
// (rounded likewise).  An autotune call whose shape is cached takes the
// cached shapes without timing; the cache can be written to and read from a
// text file.
#include "gpdf_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

using namespace gpdf;

namespace {

const int kTrainCand[] = {256, 512, 1024};
const int kEvalCand[] = {0, 1, 2, 4};
const int kMfmaCand[] = {17, 33, 65, 129};
constexpr int kTuneTimes = 11;   // 3 trainer + 4 evaluation + 4 MFMA boundaries

std::mutex g_cache_mu;
std::map<std::string, gpdf_tune> g_cache;

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

int64_t round_pow2(int64_t v) {
    if (v <= 0) return 0;
    const double l = std::round(std::log2(double(v)));
    return int64_t(1) << int64_t(l);
}

// the cache key of the trained workload and m queries (reads the cluster
// offsets back; the model must be trained eagerly)
gpdf_status shape_key(gpdf_ctx *c, int64_t m, std::string *key) {
    const Model &M = c->model;
    std::vector<int32_t> off(size_t(M.nclusters) + 1, 0);
    hipError_t e;
    if (M.nclusters > 0 &&
        ((e = hipMemcpyAsync(off.data(), c->d_coff, sizeof(int32_t) * off.size(), hipMemcpyDeviceToHost,
                             c->stream)) != hipSuccess ||
         (e = hipStreamSynchronize(c->stream)) != hipSuccess))
        return hip_fail(c, e, "autotune: read cluster offsets");
    int64_t h[7] = {};
    for (int64_t i = 0; i < M.nclusters; ++i) {
        const int n = off[size_t(i) + 1] - off[size_t(i)];
        const int b = n <= 8 ? 0 : n <= 16 ? 1 : n <= 32 ? 2 : n <= 64 ? 3 : n <= 128 ? 4 : n <= 256 ? 5 : 6;
        ++h[b];
    }
    char buf[256];
    std::snprintf(buf, sizeof buf, "p%d s%d k%d v%d h%lld,%lld,%lld,%lld,%lld,%lld,%lld q%lld", c->p.precision,
                  c->p.selection, c->p.kernel, c->p.voxel_size > 0.0 ? 1 : 0, (long long)round_pow2(h[0]),
                  (long long)round_pow2(h[1]), (long long)round_pow2(h[2]), (long long)round_pow2(h[3]),
                  (long long)round_pow2(h[4]), (long long)round_pow2(h[5]), (long long)round_pow2(h[6]),
                  (long long)round_pow2(m));
    *key = buf;
    return GPDF_OK;
}

bool valid_shape(int train_threads, int eval_persistent, int mfma_min_n) {
    return std::find(std::begin(kTrainCand), std::end(kTrainCand), train_threads) != std::end(kTrainCand) &&
           std::find(std::begin(kEvalCand), std::end(kEvalCand), eval_persistent) != std::end(kEvalCand) &&
           (mfma_min_n == 0 ||
            std::find(std::begin(kMfmaCand), std::end(kMfmaCand), mfma_min_n) != std::end(kMfmaCand));
}

}  // namespace

extern "C" gpdf_status gpdf_set_tuning(gpdf_ctx *c, int32_t train_threads, int32_t eval_persistent,
                                       int32_t mfma_min_n) {
    if (!c) return GPDF_E_INVALID_ARG;
    if (!valid_shape(train_threads, eval_persistent, mfma_min_n))
        return fail(c, GPDF_E_INVALID_ARG,
                    "set_tuning: train_threads 256/512/1024, eval_persistent 0/1/2/4, mfma_min_n 0/17/33/65/129");
    c->tune.train_threads = train_threads;
    c->tune.eval_persistent = eval_persistent;
    c->tune.mfma_min_n = mfma_min_n;
    return GPDF_OK;
}

extern "C" gpdf_status gpdf_get_tuning(const gpdf_ctx *c, int32_t *train_threads, int32_t *eval_persistent,
                                       int32_t *mfma_min_n) {
    if (!c) return GPDF_E_INVALID_ARG;
    if (train_threads) *train_threads = c->tune.train_threads;
    if (eval_persistent) *eval_persistent = c->tune.eval_persistent;
    if (mfma_min_n) *mfma_min_n = c->tune.mfma_min_n;
    return GPDF_OK;
}

extern "C" gpdf_status gpdf_autotune(gpdf_ctx *c, const float *d_xyz, int64_t n, const float *d_q, int64_t m,
                                     const float *h_origin, float *h_ms, int32_t *h_cached) {
    if (!c) return GPDF_E_INVALID_ARG;
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "join");
    if (n < 1 || !d_xyz || m < 1 || !d_q) return fail(c, GPDF_E_INVALID_ARG, "autotune: empty or null input");
    if (m > c->p.max_queries) return fail(c, GPDF_E_CAPACITY, "autotune: m exceeds max_queries");
    float ms[kTuneTimes];
    std::fill(ms, ms + kTuneTimes, -1.f);
    if (h_cached) *h_cached = 0;
    try {
        // the shape of this workload: train once to know its cluster sizes
        gpdf_status st = train(c, d_xyz, n);
        if (st != GPDF_OK) return st;
        std::string key;
        if ((st = shape_key(c, m, &key)) != GPDF_OK) return st;
        {
            std::lock_guard<std::mutex> lock(g_cache_mu);
            const auto it = g_cache.find(key);
            if (it != g_cache.end()) {
                c->tune = it->second;
                c->tune.tuned = 1;
                if (h_cached) *h_cached = 1;
                if (h_ms) std::copy(ms, ms + kTuneTimes, h_ms);
                return GPDF_OK;
            }
        }
        int best_t = c->tune.train_threads;
        float best = 0.f;
        for (int i = 0; i < 3; ++i) {
            c->tune.train_threads = kTrainCand[i];
            st = time_median(c, [&] {
                // the timed region covers the large-cluster trainer too
                const gpdf_status ts = train(c, d_xyz, n);
                (void)join_train(c);
                return ts;
            }, &ms[i]);
            if (st != GPDF_OK) return st;
            if (i == 0 || ms[i] < best) { best = ms[i]; best_t = kTrainCand[i]; }
        }
        c->tune.train_threads = best_t;
        st = train(c, d_xyz, n);
        if (st != GPDF_OK) return st;
        auto run_query = [&] {
            return query(c, d_q, m, h_origin, c->d_tmp_dist, c->d_tmp_grad, c->d_tmp_var, c->d_tmp_valid, nullptr,
                         0);
        };
        // evaluation: the VALU launch shapes, then the MFMA size boundaries
        // (FP32 and NEIGHBOR27 only; the persistent shape does not apply to
        // the MFMA kernel)
        int best_p = c->tune.eval_persistent, best_m = 0;
        c->tune.mfma_min_n = 0;
        for (int i = 0; i < 4; ++i) {
            c->tune.eval_persistent = kEvalCand[i];
            st = time_median(c, run_query, &ms[3 + i]);
            if (st != GPDF_OK) return st;
            if (i == 0 || ms[3 + i] < best) { best = ms[3 + i]; best_p = kEvalCand[i]; }
        }
        const bool mfma_ok = (c->p.precision == GPDF_PREC_FP32 || c->p.precision == GPDF_PREC_FP32_MFMA) &&
                             c->p.selection == GPDF_SEL_NEIGHBOR27;
        if (mfma_ok) {
            c->tune.eval_persistent = 0;
            for (int i = 0; i < 4; ++i) {
                c->tune.mfma_min_n = kMfmaCand[i];
                st = time_median(c, run_query, &ms[7 + i]);
                if (st != GPDF_OK) return st;
                if (ms[7 + i] < best) { best = ms[7 + i]; best_m = kMfmaCand[i]; }
            }
        }
        c->tune.eval_persistent = best_m ? 0 : best_p;
        c->tune.mfma_min_n = best_m;
        c->tune.tuned = 1;
        std::lock_guard<std::mutex> lock(g_cache_mu);
        g_cache[key] = c->tune;
    } catch (...) {
        return fail(c, GPDF_E_OOM, "autotune: host allocation failed");
    }
    if (h_ms) std::copy(ms, ms + kTuneTimes, h_ms);
    return GPDF_OK;
}

extern "C" gpdf_status gpdf_tuning_cache_save(const char *path) {
    if (!path) return GPDF_E_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_cache_mu);
    FILE *f = std::fopen(path, "w");
    if (!f) return GPDF_E_INVALID_ARG;
    bool ok = std::fprintf(f, "gpdf-tuning 1\n") > 0;
    for (const auto &kv : g_cache)
        ok = ok && std::fprintf(f, "%s|%d %d %d\n", kv.first.c_str(), kv.second.train_threads,
                                kv.second.eval_persistent, kv.second.mfma_min_n) > 0;
    ok = (std::fclose(f) == 0) && ok;
    return ok ? GPDF_OK : GPDF_E_INVALID_ARG;
}

extern "C" gpdf_status gpdf_tuning_cache_load(const char *path) {
    if (!path) return GPDF_E_INVALID_ARG;
    FILE *f = std::fopen(path, "r");
    if (!f) return GPDF_E_INVALID_ARG;
    char line[512];
    std::map<std::string, gpdf_tune> add;
    bool ok = std::fgets(line, sizeof line, f) && std::string(line) == "gpdf-tuning 1\n";
    while (ok && std::fgets(line, sizeof line, f)) {
        std::string s(line);
        const size_t bar = s.find('|');
        gpdf_tune t;
        if (bar == std::string::npos ||
            std::sscanf(s.c_str() + bar + 1, "%d %d %d", &t.train_threads, &t.eval_persistent, &t.mfma_min_n) != 3 ||
            !valid_shape(t.train_threads, t.eval_persistent, t.mfma_min_n)) {
            ok = false;
            break;
        }
        t.tuned = 1;
        add[s.substr(0, bar)] = t;
    }
    std::fclose(f);
    if (!ok) return GPDF_E_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_cache_mu);
    for (const auto &kv : add) g_cache[kv.first] = kv.second;
    return GPDF_OK;
}

extern "C" gpdf_status gpdf_tuning_cache_clear(void) {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    g_cache.clear();
    return GPDF_OK;
}
