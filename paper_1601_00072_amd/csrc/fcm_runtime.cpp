// Host runtime and C ABI of the gfx950 Fuzzy C-Means library (declared in include/fcm.h).
//
// The paper's host side (Sec. 4.1-4.3) allocates 1-D device arrays, loops on
// the host, copies the whole membership matrix back every iteration to test
// convergence, and defuzzifies on the host.  Here the host only validates,
// owns the workspace and launches passes in batches; the stopping test, the
// centroid update and the defuzzification table run on the device, and the
// host reads back a ~200-byte state record once per batch.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fcm.h"
#include "fcm_internal.h"

using namespace fcm;

namespace {

thread_local std::string g_last_error;

int dev_err(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return FCM_EDEVICE;
}

#define FCM_HIP(call)                                         \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return dev_err(e_, #call);      \
    } while (0)

constexpr uint32_t kKnownFlags = FCM_F_KAHAN_ONLY | FCM_F_TIMING;
constexpr int kMaxGraphK = 64;

int validate_params(const fcm_params* p) {
    if (!p) return FCM_EINVAL;
    if (p->n_clusters < 2 || p->n_clusters > FCM_MAX_CLUSTERS) return FCM_EINVAL;
    if (!std::isfinite(p->m) || !(p->m > 1.0)) return FCM_EINVAL;
    if (!std::isfinite(p->eps) || !(p->eps > 0.0)) return FCM_EINVAL;
    if (p->max_iter < 1 || p->max_iter > (1 << 24)) return FCM_EINVAL;
    if (p->init != FCM_INIT_LINSPACE && p->init != FCM_INIT_GIVEN) return FCM_EINVAL;
    if (p->init == FCM_INIT_GIVEN) {
        if (!p->init_centroids) return FCM_EINVAL;
        for (int k = 0; k < p->n_clusters; ++k)
            if (!std::isfinite(p->init_centroids[k]) || std::fabs(p->init_centroids[k]) > 3.0e38)
                return FCM_EINVAL;
    }
    if (p->flags & ~kKnownFlags) return FCM_EINVAL;
    return FCM_OK;
}

int validate_tuning(const fcm_tuning* t) {
    if (!t) return FCM_EINVAL;
    if (t->block != kBlock) return FCM_EINVAL;
    if (t->grid < 0 || t->grid > kMaxGrid) return FCM_EINVAL;
    if (t->unroll != 1 && t->unroll != 2) return FCM_EINVAL;
    if (t->driver != FCM_DRIVER_LOOP && t->driver != FCM_DRIVER_GRAPH) return FCM_EINVAL;
    if (t->graph_k < 1 || t->graph_k > kMaxGraphK) return FCM_EINVAL;
    return FCM_OK;
}

}  // namespace

struct fcm_handle {
    const uint8_t* d_x = nullptr;
    int64_t n = 0, head = 0, nbody = 0;
    fcm_params p{};
    double given[kMaxC] = {};
    hipStream_t stream = nullptr;
    int device = 0;
    int ncu = 256;
    int mclass = kM2;
    float alpha = 1.f, mexp = 2.f;

    DevState* d_state = nullptr;
    float* d_partials = nullptr;
    double* d_hist = nullptr;   // v: (max_iter + 2) * C, then delta, then J: (max_iter + 2) each
    DevState* h_state = nullptr;

    fcm_tuning tun{};
    int grid = 1;               // resolved pass grid

    hipStream_t cap = nullptr;  // capture-only stream for the graph driver
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int graph_k = 0;            // passes in the built graph
    int graph_grid = 0, graph_unroll = 0;

    std::vector<hipEvent_t> ev;
    double kernel_ms = 0.0;
    bool state_valid = false;

    double* hist_v() const { return d_hist; }
    double* hist_d() const { return d_hist + (int64_t)(p.max_iter + 2) * p.n_clusters; }
    double* hist_J() const { return hist_d() + (p.max_iter + 2); }
};

namespace {

int resolve_grid(const fcm_handle* h) {
    if (h->tun.grid > 0) return h->tun.grid;
    // one 16-voxel chunk per thread at least, at most 4 blocks per CU
    int64_t want = (h->nbody + kBlock - 1) / kBlock;
    int64_t cap = 4LL * h->ncu;
    return (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(want, cap), kMaxGrid));
}

PassArgs pass_args(const fcm_handle* h) {
    PassArgs a{};
    a.x = h->d_x;
    a.n = h->n;
    a.head = h->head;
    a.nbody = h->nbody;
    a.st = h->d_state;
    a.partials = h->d_partials;
    a.hist_v = h->hist_v();
    a.hist_d = h->hist_d();
    a.hist_J = h->hist_J();
    a.eps = h->p.eps;
    a.alpha = h->alpha;
    a.mexp = h->mexp;
    a.max_iter = h->p.max_iter;
    a.kahan_only = (h->p.flags & FCM_F_KAHAN_ONLY) ? 1 : 0;
    return a;
}

void drop_graph(fcm_handle* h) {
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->gexec = nullptr;
    h->graph = nullptr;
    h->graph_k = 0;
}

int build_graph(fcm_handle* h) {
    drop_graph(h);
    if (!h->cap) FCM_HIP(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    const PassArgs a = pass_args(h);
    FCM_HIP(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < h->tun.graph_k; ++i) {
        hipError_t e = launch_pass(a, h->p.n_clusters, h->mclass, h->tun.unroll, h->grid, h->cap);
        if (e != hipSuccess) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(h->cap, &g);
            if (g) (void)hipGraphDestroy(g);
            return dev_err(e, "launch_pass (capture)");
        }
    }
    FCM_HIP(hipStreamEndCapture(h->cap, &h->graph));
    FCM_HIP(hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
    h->graph_k = h->tun.graph_k;
    h->graph_grid = h->grid;
    h->graph_unroll = h->tun.unroll;
    return FCM_OK;
}

int read_state(fcm_handle* h) {
    FCM_HIP(hipMemcpyAsync(h->h_state, h->d_state, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
    FCM_HIP(hipStreamSynchronize(h->stream));
    h->state_valid = true;
    return FCM_OK;
}

void fill_result(const fcm_handle* h, fcm_result* out) {
    const DevState& s = *h->h_state;
    std::memset(out, 0, sizeof(*out));
    out->iters = s.iters < 0 ? 0 : s.iters;
    out->passes = s.passes;
    out->status = s.status;
    out->n_clusters = h->p.n_clusters;
    out->delta = s.delta;
    out->J = s.J;
    for (int k = 0; k < h->p.n_clusters; ++k) out->centroids[k] = s.vres[k];
    out->kernel_ms = h->kernel_ms;
    out->lo = s.lo;
    out->hi = s.hi;
}

// Launch up to `batch` passes and read the state back once.
int run_batch(fcm_handle* h, int batch) {
    const bool timing = (h->p.flags & FCM_F_TIMING) != 0;
    const int before = h->h_state->passes;
    if (!timing && h->tun.driver == FCM_DRIVER_GRAPH && batch == h->tun.graph_k) {
        if (!h->gexec || h->graph_k != h->tun.graph_k || h->graph_grid != h->grid ||
            h->graph_unroll != h->tun.unroll) {
            int rc = build_graph(h);
            if (rc != FCM_OK) return rc;
        }
        FCM_HIP(hipGraphLaunch(h->gexec, h->stream));
        return read_state(h);
    }
    const PassArgs a = pass_args(h);
    if (timing) {
        while ((int)h->ev.size() < 2 * batch) {
            hipEvent_t e;
            FCM_HIP(hipEventCreate(&e));
            h->ev.push_back(e);
        }
    }
    for (int i = 0; i < batch; ++i) {
        if (timing) FCM_HIP(hipEventRecord(h->ev[2 * i], h->stream));
        hipError_t e = launch_pass(a, h->p.n_clusters, h->mclass, h->tun.unroll, h->grid, h->stream);
        if (e != hipSuccess) return dev_err(e, "launch_pass");
        if (timing) FCM_HIP(hipEventRecord(h->ev[2 * i + 1], h->stream));
    }
    int rc = read_state(h);
    if (rc != FCM_OK) return rc;
    if (timing) {
        const int ran = std::min(batch, h->h_state->passes - before);
        for (int i = 0; i < ran; ++i) {
            float ms = 0.f;
            FCM_HIP(hipEventElapsedTime(&ms, h->ev[2 * i], h->ev[2 * i + 1]));
            h->kernel_ms += ms;
        }
    }
    return FCM_OK;
}

int enqueue_start(fcm_handle* h) {
    FCM_HIP(hipMemsetAsync(h->d_state, 0, sizeof(DevState), h->stream));
    InitArgs ia{};
    ia.x = h->d_x;
    ia.n = h->n;
    ia.head = h->head;
    ia.nbody = h->nbody;
    ia.st = h->d_state;
    ia.partials = reinterpret_cast<uint32_t*>(h->d_partials);
    ia.hist_v = h->hist_v();
    ia.C = h->p.n_clusters;
    ia.given = h->p.init == FCM_INIT_GIVEN ? 1 : 0;
    for (int k = 0; k < h->p.n_clusters; ++k) ia.v0[k] = h->given[k];
    const int igrid = (int)std::max<int64_t>(1, std::min<int64_t>((h->nbody + kBlock - 1) / kBlock,
                                                                    std::min<int64_t>(4LL * h->ncu, kMaxGrid)));
    hipError_t e = launch_init(ia, igrid, h->stream);
    if (e != hipSuccess) return dev_err(e, "launch_init");
    std::memset(h->h_state, 0, sizeof(DevState));
    h->h_state->iters = -1;
    h->h_state->status = FCM_RUNNING;
    h->kernel_ms = 0.0;
    return FCM_OK;
}

void release(fcm_handle* h) {
    if (!h) return;
    drop_graph(h);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    if (h->d_state) (void)hipFree(h->d_state);
    if (h->d_partials) (void)hipFree(h->d_partials);
    if (h->d_hist) (void)hipFree(h->d_hist);
    if (h->h_state) (void)hipHostFree(h->h_state);
    delete h;
}

}  // namespace

extern "C" {

int fcm_version(void) { return 1 * 10000 + 0 * 100 + 0; }

const char* fcm_strerror(int status) {
    switch (status) {
        case FCM_OK: return "converged";
        case FCM_NOT_CONVERGED: return "max_iter reached before convergence";
        case FCM_RUNNING: return "iterations remain";
        case FCM_EINVAL: return "invalid argument";
        case FCM_ENOMEM: return "out of memory";
        case FCM_EDEVICE: return "HIP error";
        case FCM_ESTATE: return "call out of order";
        case FCM_ENUMERIC: return "non-finite centroid or objective";
        case FCM_EUNSUPPORTED: return "configuration not supported";
        default: return "unknown status";
    }
}

const char* fcm_last_error(void) { return g_last_error.c_str(); }

int fcm_init(fcm_handle** out, const uint8_t* d_x, int64_t n, const fcm_params* p, void* stream) {
    if (!out || !d_x || n < 1) return FCM_EINVAL;
    int rc = validate_params(p);
    if (rc != FCM_OK) return rc;
    fcm_handle* h = new (std::nothrow) fcm_handle();
    if (!h) return FCM_ENOMEM;
    h->d_x = d_x;
    h->n = n;
    h->p = *p;
    if (p->init == FCM_INIT_GIVEN)
        for (int k = 0; k < p->n_clusters; ++k) h->given[k] = p->init_centroids[k];
    h->p.init_centroids = nullptr;
    h->stream = (hipStream_t)stream;
    const int C = p->n_clusters;
    h->mclass = (p->m == 2.0) ? kM2 : (p->m == 1.5 ? kM15 : kMGeneric);
    h->alpha = (float)(1.0 / (p->m - 1.0));
    h->mexp = (float)p->m;
    const uintptr_t addr = (uintptr_t)d_x;
    h->head = std::min<int64_t>(n, (int64_t)((16 - (addr & 15)) & 15));
    h->nbody = (n - h->head) / 16;

    auto fail = [&](int code) {
        release(h);
        return code;
    };
    hipError_t e;
    if ((e = hipGetDevice(&h->device)) != hipSuccess) return fail(dev_err(e, "hipGetDevice"));
    if ((e = hipDeviceGetAttribute(&h->ncu, hipDeviceAttributeMultiprocessorCount, h->device)) != hipSuccess)
        return fail(dev_err(e, "hipDeviceGetAttribute"));
    h->tun.block = kBlock;
    h->tun.grid = 0;
    h->tun.unroll = 1;
    h->tun.driver = FCM_DRIVER_GRAPH;
    h->tun.graph_k = 8;
    h->grid = resolve_grid(h);

    if (hipMalloc(&h->d_state, sizeof(DevState)) != hipSuccess) return fail(FCM_ENOMEM);
    if (hipMalloc(&h->d_partials, sizeof(float) * partial_rows(kMaxC) * kMaxGrid) != hipSuccess)
        return fail(FCM_ENOMEM);
    const size_t hist_doubles = (size_t)(p->max_iter + 2) * (C + 2);
    if (hipMalloc(&h->d_hist, sizeof(double) * hist_doubles) != hipSuccess) return fail(FCM_ENOMEM);
    if (hipHostMalloc(&h->h_state, sizeof(DevState), hipHostMallocDefault) != hipSuccess) return fail(FCM_ENOMEM);
    rc = enqueue_start(h);
    if (rc != FCM_OK) return fail(rc);
    *out = h;
    return FCM_OK;
}

int fcm_reset(fcm_handle* h) {
    if (!h) return FCM_EINVAL;
    return enqueue_start(h);
}

int fcm_set_tuning(fcm_handle* h, const fcm_tuning* t) {
    if (!h) return FCM_EINVAL;
    int rc = validate_tuning(t);
    if (rc != FCM_OK) return rc;
    if (!pass_supported(h->p.n_clusters, h->mclass, t->unroll)) return FCM_EUNSUPPORTED;
    h->tun = *t;
    h->grid = resolve_grid(h);
    return FCM_OK;
}

int fcm_get_tuning(const fcm_handle* h, fcm_tuning* t) {
    if (!h || !t) return FCM_EINVAL;
    *t = h->tun;
    t->grid = h->grid;
    return FCM_OK;
}

int fcm_iterate(fcm_handle* h, int32_t k, fcm_result* out) {
    if (!h || !out || k < 0) return FCM_EINVAL;
    int rc = read_state(h);
    if (rc != FCM_OK) return rc;
    int remaining = k;
    while (remaining > 0 && !h->h_state->done) {
        const int batch = std::min(remaining, h->tun.graph_k);
        rc = run_batch(h, batch);
        if (rc != FCM_OK) return rc;
        remaining -= batch;
    }
    fill_result(h, out);
    return out->status;
}

int fcm_solve(fcm_handle* h, fcm_result* out) {
    if (!h || !out) return FCM_EINVAL;
    int rc = read_state(h);
    if (rc != FCM_OK) return rc;
    // every pass either finishes the solve or advances the pass index, so
    // max_iter + 1 passes always suffice; the bound guards the host loop
    int64_t budget = (int64_t)h->p.max_iter + 1 + h->tun.graph_k;
    while (!h->h_state->done && budget > 0) {
        rc = run_batch(h, h->tun.graph_k);
        if (rc != FCM_OK) return rc;
        budget -= h->tun.graph_k;
    }
    fill_result(h, out);
    return out->status;
}

int fcm_labels(fcm_handle* h, uint8_t* d_labels) {
    if (!h || !d_labels) return FCM_EINVAL;
    LabelArgs a{};
    a.x = h->d_x;
    a.labels = d_labels;
    a.n = h->n;
    a.head = h->head;
    a.nbody = h->nbody;
    a.st = h->d_state;
    a.hist_v = h->hist_v();
    a.C = h->p.n_clusters;
    a.bytewise = (((uintptr_t)h->d_x ^ (uintptr_t)d_labels) & 15) ? 1 : 0;
    int64_t work = a.bytewise ? (h->n + 15) / 16 : h->nbody;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((work + kBlock - 1) / kBlock,
                                                                  std::min<int64_t>(4LL * h->ncu, kMaxGrid)));
    hipError_t e = launch_labels(a, grid, h->stream);
    if (e != hipSuccess) return dev_err(e, "launch_labels");
    return FCM_OK;
}

int fcm_centroids(fcm_handle* h, double* out) {
    if (!h || !out) return FCM_EINVAL;
    int rc = read_state(h);
    if (rc != FCM_OK) return rc;
    for (int k = 0; k < h->p.n_clusters; ++k) out[k] = h->h_state->vres[k];
    return FCM_OK;
}

int fcm_trajectory(fcm_handle* h, int32_t t, double* v_out, double* delta, double* J) {
    if (!h) return FCM_EINVAL;
    int rc = read_state(h);
    if (rc != FCM_OK) return rc;
    if (t < 0 || t > h->h_state->iters) return FCM_EINVAL;
    const int C = h->p.n_clusters;
    double row[kMaxC + 2];
    FCM_HIP(hipMemcpyAsync(row, h->hist_v() + (int64_t)t * C, sizeof(double) * C, hipMemcpyDeviceToHost,
                           h->stream));
    FCM_HIP(hipMemcpyAsync(row + C, h->hist_d() + t, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    FCM_HIP(hipMemcpyAsync(row + C + 1, h->hist_J() + t, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    FCM_HIP(hipStreamSynchronize(h->stream));
    if (v_out) std::memcpy(v_out, row, sizeof(double) * C);
    if (delta) *delta = row[C];
    if (J) *J = row[C + 1];
    return FCM_OK;
}

void fcm_destroy(fcm_handle* h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    release(h);
}

}  // extern "C"
