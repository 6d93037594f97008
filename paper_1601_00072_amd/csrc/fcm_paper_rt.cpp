// Host loop of the paper-design baseline (Sec. 4 and its block diagram): the
// host initialises U (or computes it from given centroids), the device
// updates the centroids and the memberships cluster by cluster, and after
// every iteration the host copies U back and evaluates the stopping test.
// Defuzzification also runs on the host, from the final centroids.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

#include "fcm.h"
#include "fcm_host.h"
#include "fcm_paper.h"

namespace {

using fcm::PaperBuffers;

// draw k of the SplitMix64 stream `seed`, top 24 bits + 1, scaled to (0, 1]
float draw24(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (float)((uint32_t)(z >> 40) + 1u) * (1.0f / 16777216.0f);
}

struct Work {
    PaperBuffers b{};
    float* hU[2] = {nullptr, nullptr};  // pinned host copies of U (previous, current)
    std::vector<uint8_t> hx;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    ~Work() {
        for (void* p : {(void*)b.U, (void*)b.num, (void*)b.den, (void*)b.bnum, (void*)b.bden, (void*)b.v,
                        (void*)b.v32})
            if (p) (void)hipFree(p);
        for (float* p : hU)
            if (p) (void)hipHostFree(p);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

extern "C" int fcm_paper_solve(const uint8_t* d_x, int64_t n, const fcm_params* p, void* stream, fcm_result* out,
                               double* v_hist, double* delta_hist, uint8_t* labels, fcm_paper_stats* stats) {
    using namespace fcm;
    if (!d_x || n < 1 || !p || !out) return FCM_EINVAL;
    const int C = p->n_clusters;
    if (C < 2 || C > FCM_MAX_CLUSTERS || !std::isfinite(p->m) || !(p->m > 1.0) || !std::isfinite(p->eps) ||
        !(p->eps > 0.0) || p->max_iter < 1 || p->max_iter > (1 << 24))
        return FCM_EINVAL;
    if (p->init != FCM_INIT_RANDOM_U && p->init != FCM_INIT_LINSPACE && p->init != FCM_INIT_GIVEN) return FCM_EINVAL;
    if (p->init == FCM_INIT_GIVEN) {
        if (!p->init_centroids) return FCM_EINVAL;
        for (int k = 0; k < C; ++k)
            if (!std::isfinite(p->init_centroids[k])) return FCM_EINVAL;
    }
    if ((uint64_t)n > (uint64_t)std::numeric_limits<int64_t>::max() / (uint64_t)(C * sizeof(float)))
        return FCM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const float m = (float)p->m;
    Work w;
    PaperBuffers& b = w.b;
    b.x = d_x;
    b.n = n;
    const size_t ubytes = sizeof(float) * (size_t)C * (size_t)n;
    const int64_t parts = paper_parts(n);
    if (hipMalloc(&b.U, ubytes) != hipSuccess || hipMalloc(&b.num, sizeof(float) * n) != hipSuccess ||
        hipMalloc(&b.den, sizeof(float) * n) != hipSuccess || hipMalloc(&b.bnum, sizeof(float) * parts) != hipSuccess ||
        hipMalloc(&b.bden, sizeof(float) * parts) != hipSuccess || hipMalloc(&b.v, sizeof(double) * C) != hipSuccess ||
        hipMalloc(&b.v32, sizeof(float) * C) != hipSuccess)
        return FCM_ENOMEM;
    for (float*& h : w.hU)
        if (hipHostMalloc(&h, ubytes, hipHostMallocDefault) != hipSuccess) return FCM_ENOMEM;
    for (hipEvent_t& e : w.ev) FCM_HIP(hipEventCreate(&e));
    try {
        w.hx.resize((size_t)n);
    } catch (...) {
        return FCM_ENOMEM;
    }
    // the image on the host (the design keeps it there too) and its range
    FCM_HIP(hipMemcpyAsync(w.hx.data(), d_x, (size_t)n, hipMemcpyDeviceToHost, s));
    FCM_HIP(hipStreamSynchronize(s));
    const auto mm = std::minmax_element(w.hx.begin(), w.hx.end());
    const int lo = *mm.first, hi = *mm.second;

    // start: U^0 on the host (random), or from v^0 on the device
    double v[FCM_MAX_CLUSTERS];
    const double nan = std::numeric_limits<double>::quiet_NaN();
    if (p->init == FCM_INIT_RANDOM_U) {
        float* U0 = w.hU[0];
        for (int64_t i = 0; i < n; ++i) {
            float r[FCM_MAX_CLUSTERS], sum = 0.f;
            for (int j = 0; j < C; ++j) {
                r[j] = draw24(p->seed, (uint64_t)i * C + j);
                sum += r[j];
            }
            for (int j = 0; j < C; ++j) U0[(int64_t)j * n + i] = r[j] / sum;
        }
        for (int j = 0; j < C; ++j) v[j] = nan;
        FCM_HIP(hipMemcpyAsync(b.U, U0, ubytes, hipMemcpyHostToDevice, s));
        FCM_HIP(hipMemcpyAsync(b.v, v, sizeof(double) * C, hipMemcpyHostToDevice, s));
    } else {
        float v32[FCM_MAX_CLUSTERS];
        for (int j = 0; j < C; ++j) {
            const double vj = p->init == FCM_INIT_GIVEN ? p->init_centroids[j]
                                                        : (double)lo + (double)(j * (hi - lo)) / (double)(C - 1);
            v32[j] = (float)vj;
            v[j] = (double)v32[j];
        }
        FCM_HIP(hipMemcpyAsync(b.v, v, sizeof(double) * C, hipMemcpyHostToDevice, s));
        FCM_HIP(hipMemcpyAsync(b.v32, v32, sizeof(float) * C, hipMemcpyHostToDevice, s));
        FCM_HIP(paper_memberships(b, C, m, s));
        FCM_HIP(hipMemcpyAsync(w.hU[0], b.U, ubytes, hipMemcpyDeviceToHost, s));
    }
    FCM_HIP(hipStreamSynchronize(s));
    if (v_hist)
        for (int j = 0; j < C; ++j) v_hist[j] = v[j];
    if (delta_hist) delta_hist[0] = nan;

    fcm_paper_stats st{};
    const auto t_loop = std::chrono::steady_clock::now();
    int T = p->max_iter, status = FCM_NOT_CONVERGED;
    double delta = nan;
    int prev = 0;
    for (int t = 1; t <= p->max_iter; ++t) {
        FCM_HIP(hipEventRecord(w.ev[0], s));
        FCM_HIP(paper_centroids(b, C, m, s));
        FCM_HIP(paper_memberships(b, C, m, s));
        FCM_HIP(hipEventRecord(w.ev[1], s));
        FCM_HIP(hipMemcpyAsync(w.hU[prev ^ 1], b.U, ubytes, hipMemcpyDeviceToHost, s));
        FCM_HIP(hipMemcpyAsync(v, b.v, sizeof(double) * C, hipMemcpyDeviceToHost, s));
        FCM_HIP(hipEventRecord(w.ev[2], s));
        FCM_HIP(hipStreamSynchronize(s));
        float k_ms = 0.f, c_ms = 0.f;
        FCM_HIP(hipEventElapsedTime(&k_ms, w.ev[0], w.ev[1]));
        FCM_HIP(hipEventElapsedTime(&c_ms, w.ev[1], w.ev[2]));
        st.kernels_ms += k_ms;
        st.copy_ms += c_ms;
        st.launches += 5LL * C;
        // the stopping test on the host: max_ij |u_ij^t - u_ij^(t-1)|
        const auto t_host = std::chrono::steady_clock::now();
        const float* a = w.hU[prev];
        const float* c = w.hU[prev ^ 1];
        float dmax = 0.f;
        for (int64_t i = 0; i < (int64_t)C * n; ++i) dmax = std::max(dmax, std::fabs(c[i] - a[i]));
        st.host_ms += ms_since(t_host);
        delta = (double)dmax;
        prev ^= 1;
        if (v_hist)
            for (int j = 0; j < C; ++j) v_hist[(int64_t)t * C + j] = v[j];
        if (delta_hist) delta_hist[t] = delta;
        if (delta < p->eps) {
            T = t;
            status = FCM_OK;
            break;
        }
    }
    st.total_ms = ms_since(t_loop);
    // defuzzification on the host: nearest centroid (ties to the lowest index)
    if (labels) {
        for (int64_t i = 0; i < n; ++i) {
            int best = 0;
            double bd = std::fabs((double)w.hx[i] - v[0]);
            for (int j = 1; j < C; ++j) {
                const double d = std::fabs((double)w.hx[i] - v[j]);
                if (d < bd) {
                    bd = d;
                    best = j;
                }
            }
            labels[i] = (uint8_t)best;
        }
    }
    std::memset(out, 0, sizeof(*out));
    out->iters = T;
    out->passes = T;
    out->status = status;
    out->n_clusters = C;
    out->delta = delta;
    out->J = nan;
    for (int j = 0; j < C; ++j) out->centroids[j] = v[j];
    out->kernel_ms = st.kernels_ms;
    out->lo = lo;
    out->hi = hi;
    if (stats) *stats = st;
    return status;
}
