// Host runtime and C ABI of the gfx950 Fuzzy C-Means library (declared in include/fcm.h).
//
// The paper's host side (Sec. 4.1-4.3) allocates 1-D device arrays, loops on
// the host, copies the whole membership matrix back every iteration to test
// convergence, and defuzzifies on the host.  Here the host only validates,
// owns the workspace and launches work; the stopping test, the centroid
// update and the defuzzification table run on the device, and the host reads
// back a ~250-byte state record once per batch of passes (once per solve with
// the persistent driver).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstddef>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fcm.h"
#include "fcm_host.h"
#include "fcm_random.h"
#include "fcm_internal.h"
#include "fcm_learn.h"

using namespace fcm;

namespace fcm {

std::string& last_error() {
    thread_local std::string text;
    return text;
}

int dev_err(hipError_t e, const char* what) {
    last_error() = std::string(what) + ": " + hipGetErrorString(e);
    return FCM_EDEVICE;
}

}  // namespace fcm

namespace {

constexpr uint32_t kKnownFlags = FCM_F_KAHAN_ONLY | FCM_F_TIMING;
constexpr int kMaxGraphK = 64;
constexpr double kBarrierLimitSeconds = 5.0;
constexpr int64_t kAllGatherBytes = 6LL << 20;

int validate_params(const fcm_params* p) {
    if (!p) return FCM_EINVAL;
    if (p->n_clusters < 2 || p->n_clusters > FCM_MAX_CLUSTERS) return FCM_EINVAL;
    if (!std::isfinite(p->m) || !(p->m > 1.0)) return FCM_EINVAL;
    if (!std::isfinite(p->eps) || !(p->eps > 0.0)) return FCM_EINVAL;
    if (p->max_iter < 1 || p->max_iter > (1 << 24)) return FCM_EINVAL;
    if (p->init != FCM_INIT_LINSPACE && p->init != FCM_INIT_GIVEN && p->init != FCM_INIT_DEVICE &&
        p->init != FCM_INIT_RANDOM_U)
        return FCM_EINVAL;
    if (p->init == FCM_INIT_DEVICE && !p->init_centroids) return FCM_EINVAL;
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
    if (t->driver != FCM_DRIVER_LOOP && t->driver != FCM_DRIVER_GRAPH && t->driver != FCM_DRIVER_PERSISTENT &&
        t->driver != FCM_DRIVER_HISTOGRAM)
        return FCM_EINVAL;
    if (t->graph_k < 1 || t->graph_k > kMaxGraphK) return FCM_EINVAL;
    if (t->exchange < FCM_EXCHANGE_AUTO || t->exchange > FCM_EXCHANGE_XCD) return FCM_EINVAL;
    if (t->launch != FCM_LAUNCH_COOPERATIVE && t->launch != FCM_LAUNCH_RESIDENT) return FCM_EINVAL;
    return FCM_OK;
}

}  // namespace

struct fcm_handle {
    const uint8_t* d_x = nullptr;
    int64_t n = 0, head = 0, nbody = 0;
    fcm_params p{};
    double given[kMaxC] = {};
    const double* dv0 = nullptr;   // device start centroids (FCM_INIT_DEVICE)
    hipStream_t stream = nullptr;
    int device = 0;
    int ncu = 256;
    int coop = 0;               // cooperative launches supported
    uint64_t spin_ticks = 0;    // barrier wait limit in wall-clock ticks
    uint64_t default_ticks = 0; // the default limit (kBarrierLimitSeconds)
    uint64_t clock_khz = 100000;
    bool coop_retry = false;    // the running solve is the cooperative retry of a resident launch
    int32_t recoveries = 0;     // resident solves that gave up and were solved again cooperatively
    int mclass = kM2;
    float alpha = 1.f, mexp = 2.f;

    DevState* d_state = nullptr;
    float* d_partials = nullptr;   // [rows][grid] partial rows of the per-pass launches
    uint32_t* d_minmax = nullptr;  // [2][grid]
    uint64_t* d_rows = nullptr;    // [2][kMaxPersistGrid][rows] tagged partial rows (cooperative driver)
    uint64_t* d_mmrows = nullptr;  // [2][kMaxPersistGrid][2] tagged grey-level ranges (cooperative driver)
    bool aborted = false;          // a cooperative wait timed out; the next reset clears everything
    double* d_hist = nullptr;      // v: (max_iter + 2) * C, then delta, then J: (max_iter + 2) each
    DevState* h_state = nullptr;

    fcm_tuning tun{};
    int grid = 1;               // resolved grid of the current driver
    bool pending_init = true;   // the data-range pass has not run since init/reset

    hipStream_t cap = nullptr;  // capture-only stream for the graph driver
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int graph_k = 0;            // passes in the built graph
    int graph_grid = 0, graph_unroll = 0;

    std::vector<hipEvent_t> ev;
    double kernel_ms = 0.0;
    int async_timed = 0;        // timed fcm_solve_async launches since the last fcm_solve_wait (event pairs)
    double async_ms = 0.0;      // kernel time of host-driven solves run by fcm_solve_async

    // warm start workspace (first fcm_solve_warm)
    int64_t* d_woff = nullptr;     // {0, n}
    uint32_t* d_wcounts = nullptr; // [kHistCopies][256] histogram workspace (copy 0: totals)
    float* d_whist = nullptr;      // [256]
    float* d_wy = nullptr;         // [kMaxC] network output
    double* d_wv0 = nullptr;       // [kMaxC] learned start
    uint32_t* d_ghist = nullptr;   // [2][kHistCopies][256] counters of the in-kernel histogram; a learned
                                   // launch uses buffer ghist_sel and zeroes the other one
    uint32_t ghist_sel = 0;
    const uint16_t* mlp_w = nullptr;  // BF16 network of the running fused warm solve

    double* hist_v() const { return d_hist; }
    double* hist_d() const { return d_hist + (int64_t)(p.max_iter + 2) * p.n_clusters; }
    double* hist_J() const { return hist_d() + (p.max_iter + 2); }
};

namespace {

int64_t chunk_blocks(const fcm_handle* h) { return (h->nbody + kBlock - 1) / kBlock; }

// Internal start mode of a warm solve on the persistent driver: histogram and
// network inference inside the solve kernel.
constexpr int32_t kInitLearnedFused = 0x100;

int start_mode(int init) {
    return init == FCM_INIT_GIVEN ? 1 : (init == FCM_INIT_DEVICE ? 2 : (init == kInitLearnedFused ? 3 : 0));
}

int resolve_grid(fcm_handle* h, int* out) {
    int64_t want = h->tun.grid > 0 ? h->tun.grid : std::min<int64_t>(chunk_blocks(h), 4LL * h->ncu);
    if (h->tun.driver == FCM_DRIVER_PERSISTENT) {
        int cap = 0;
        FCM_HIP(persist_max_grid(h->p.n_clusters, h->mclass, h->tun.unroll, h->ncu, &cap));
        want = std::min<int64_t>(want, std::min(cap, kMaxPersistGrid));
    }
    *out = (int)std::max<int64_t>(1, std::min<int64_t>(want, kMaxGrid));
    return FCM_OK;
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
    a.rows = h->d_rows;
    a.mm_rows = h->d_mmrows;
    // all-gather while the rows every block reads stay small (grid^2 rows)
    a.allgather = (int64_t)h->grid * h->grid * (2 * h->p.n_clusters + 2) * 8 <= kAllGatherBytes ? 1 : 0;
    if (h->tun.exchange == FCM_EXCHANGE_LEADER) a.allgather = 0;
    if (h->tun.exchange == FCM_EXCHANGE_ALLGATHER) a.allgather = 1;
    a.xcd = h->tun.exchange == FCM_EXCHANGE_XCD ? 1 : 0;
    if (a.xcd) a.allgather = 0;  // the data-range round and any fallback use the leader
    a.do_init = h->pending_init ? 1 : 0;
    a.given = start_mode(h->p.init);
    for (int k = 0; k < kMaxC; ++k) a.v0[k] = h->given[k];
    a.dv0 = h->dv0;
    a.mlp_w = h->mlp_w;
    a.ghist = h->d_ghist ? h->d_ghist + (size_t)(h->ghist_sel & 1) * 256 * kHistCopies : nullptr;
    a.ghist_next = h->d_ghist ? h->d_ghist + (size_t)((h->ghist_sel + 1) & 1) * 256 * kHistCopies : nullptr;
    a.max_passes = 0;
    // the cooperative retry guarantees co-residency: it waits at least the default limit
    a.spin_ticks = h->coop_retry ? std::max(h->spin_ticks, h->default_ticks) : h->spin_ticks;
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
    if (h->h_state->sync.abort) {
        h->aborted = true;
        last_error() = "a cross-block wait exceeded its time limit; the solve was aborted (reset the handle)";
        return FCM_EDEVICE;
    }
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

int ensure_events(fcm_handle* h, int count) {
    while ((int)h->ev.size() < count) {
        hipEvent_t e;
        FCM_HIP(hipEventCreate(&e));
        h->ev.push_back(e);
    }
    return FCM_OK;
}

// The data-range pass as its own launch (loop and graph drivers, and any call
// that needs v^0 before a pass has run).
int flush_init(fcm_handle* h) {
    if (!h->pending_init) return FCM_OK;
    InitArgs ia{};
    ia.x = h->d_x;
    ia.n = h->n;
    ia.head = h->head;
    ia.nbody = h->nbody;
    ia.st = h->d_state;
    ia.partials = h->d_minmax;
    ia.hist_v = h->hist_v();
    ia.C = h->p.n_clusters;
    ia.given = start_mode(h->p.init);
    for (int k = 0; k < h->p.n_clusters; ++k) ia.v0[k] = h->given[k];
    ia.dv0 = h->dv0;
    const int igrid = (int)std::max<int64_t>(1, std::min<int64_t>(chunk_blocks(h), std::min<int64_t>(4LL * h->ncu,
                                                                                                      kMaxGrid)));
    hipError_t e = launch_init(ia, igrid, h->stream);
    if (e != hipSuccess) return dev_err(e, "launch_init");
    h->pending_init = false;
    return FCM_OK;
}

int ensure_level_ws(fcm_handle* h);

// Random-membership start: the data-range pass (for lo, hi), then those of
// passes 0 and 1 that are still due, from the budget `batch`, launched back
// to back (each kernel checks the pass counter) with one read-back.
int run_random_start(fcm_handle* h, int& batch) {
    int rc = flush_init(h);
    if (rc != FCM_OK) return rc;
    const int first = h->h_state->passes;
    if (first >= 2 || h->h_state->done || batch < 1) return FCM_OK;
    const int last = std::min(2, first + batch);
    const bool timing = (h->p.flags & FCM_F_TIMING) != 0;
    if (timing) {
        if ((rc = ensure_events(h, 2)) != FCM_OK) return rc;
        FCM_HIP(hipEventRecord(h->ev[0], h->stream));
    }
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(chunk_blocks(h), std::min<int64_t>(4LL * h->ncu,
                                                                                                     kMaxGrid)));
    const PassArgs a = pass_args(h);
    for (int phase = first; phase < last; ++phase) {
        hipError_t e = launch_random_pass(a, h->p.n_clusters, phase, h->p.seed, grid, h->stream);
        if (e != hipSuccess) return dev_err(e, "launch_random_pass");
    }
    if (timing) FCM_HIP(hipEventRecord(h->ev[1], h->stream));
    if ((rc = read_state(h)) != FCM_OK) return rc;
    if (timing) {
        float ms = 0.f;
        FCM_HIP(hipEventElapsedTime(&ms, h->ev[0], h->ev[1]));
        h->kernel_ms += ms;
    }
    batch -= last - first;
    return FCM_OK;
}

// Kernel time of the timed asynchronous solves still pending, folded into
// async_ms (waits for their last event), so that their event pairs can be reused.
int fold_async(fcm_handle* h) {
    if (h->async_timed == 0) return FCM_OK;
    FCM_HIP(hipEventSynchronize(h->ev[2 * h->async_timed - 1]));
    for (int i = 0; i < h->async_timed; ++i) {
        float t = 0.f;
        FCM_HIP(hipEventElapsedTime(&t, h->ev[2 * i], h->ev[2 * i + 1]));
        h->async_ms += t;
    }
    h->async_timed = 0;
    return FCM_OK;
}

// Run up to `batch` passes and read the state back once.
int run_batch(fcm_handle* h, int batch) {
    const bool timing = (h->p.flags & FCM_F_TIMING) != 0;
    if (timing && h->async_timed) {
        int rc = fold_async(h);
        if (rc != FCM_OK) return rc;
    }
    if (h->p.init == FCM_INIT_RANDOM_U && h->tun.driver != FCM_DRIVER_HISTOGRAM) {
        int rc = run_random_start(h, batch);
        if (rc != FCM_OK) return rc;
        if (batch < 1 || h->h_state->done) return FCM_OK;
    }
    if (h->tun.driver == FCM_DRIVER_HISTOGRAM) {
        int rc = ensure_level_ws(h);
        if (rc != FCM_OK) return rc;
        LevelArgs la{};
        la.counts = h->d_wcounts;  // copy 0: the totals
        la.st = h->d_state;
        la.hist_v = h->hist_v();
        la.hist_d = h->hist_d();
        la.hist_J = h->hist_J();
        la.eps = h->p.eps;
        la.m = h->p.m;
        la.max_iter = h->p.max_iter;
        la.do_init = h->pending_init ? 1 : 0;
        la.given = start_mode(h->p.init);
        for (int k = 0; k < kMaxC; ++k) la.v0[k] = h->given[k];
        la.dv0 = h->dv0;
        la.max_passes = batch;
        if (timing) {
            if ((rc = ensure_events(h, 2)) != FCM_OK) return rc;
            FCM_HIP(hipEventRecord(h->ev[0], h->stream));
        }
        if (h->pending_init)
            FCM_HIP(launch_histogram(h->d_x, h->d_woff, 1, h->n, h->d_wcounts, h->d_whist, h->stream));
        FCM_HIP(launch_levels(la, h->p.n_clusters, h->stream));
        h->pending_init = false;
        if (timing) FCM_HIP(hipEventRecord(h->ev[1], h->stream));
        if ((rc = read_state(h)) != FCM_OK) return rc;
        if (timing) {
            float ms = 0.f;
            FCM_HIP(hipEventElapsedTime(&ms, h->ev[0], h->ev[1]));
            h->kernel_ms += ms;
        }
        return FCM_OK;
    }
    if (h->tun.driver == FCM_DRIVER_PERSISTENT) {
        PassArgs a = pass_args(h);
        a.max_passes = batch;
        if (timing) {
            int rc = ensure_events(h, 2);
            if (rc != FCM_OK) return rc;
            FCM_HIP(hipEventRecord(h->ev[0], h->stream));
        }
        hipError_t e = launch_persist(a, h->p.n_clusters, h->mclass, h->tun.unroll, h->grid,
                                      h->tun.launch == FCM_LAUNCH_COOPERATIVE || h->coop_retry, h->stream);
        if (e != hipSuccess) return dev_err(e, "persistent launch");
        h->pending_init = false;
        if (timing) FCM_HIP(hipEventRecord(h->ev[1], h->stream));
        int rc = read_state(h);
        if (rc != FCM_OK) return rc;
        if (timing) {
            float ms = 0.f;
            FCM_HIP(hipEventElapsedTime(&ms, h->ev[0], h->ev[1]));
            h->kernel_ms += ms;
        }
        return FCM_OK;
    }
    int rc = flush_init(h);
    if (rc != FCM_OK) return rc;
    if (!timing && h->tun.driver == FCM_DRIVER_GRAPH && batch == h->tun.graph_k) {
        if (!h->gexec || h->graph_k != h->tun.graph_k || h->graph_grid != h->grid ||
            h->graph_unroll != h->tun.unroll) {
            rc = build_graph(h);
            if (rc != FCM_OK) return rc;
        }
        FCM_HIP(hipGraphLaunch(h->gexec, h->stream));
        return read_state(h);
    }
    const int before = h->h_state->passes;
    const PassArgs a = pass_args(h);
    if (timing) {
        rc = ensure_events(h, 2 * batch);
        if (rc != FCM_OK) return rc;
    }
    for (int i = 0; i < batch; ++i) {
        if (timing) FCM_HIP(hipEventRecord(h->ev[2 * i], h->stream));
        hipError_t e = launch_pass(a, h->p.n_clusters, h->mclass, h->tun.unroll, h->grid, h->stream);
        if (e != hipSuccess) return dev_err(e, "launch_pass");
        if (timing) FCM_HIP(hipEventRecord(h->ev[2 * i + 1], h->stream));
    }
    rc = read_state(h);
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

// Grey-level workspace of a handle (histogram, network output, learned
// start), allocated on first use by the warm start or the histogram driver.
int ensure_level_ws(fcm_handle* h) {
    if (h->d_woff) return FCM_OK;
    if (!h->d_wcounts && hipMalloc(&h->d_wcounts, sizeof(uint32_t) * 256 * histogram_copies(1)) != hipSuccess)
        return FCM_ENOMEM;
    if (!h->d_whist && hipMalloc(&h->d_whist, sizeof(float) * 256) != hipSuccess) return FCM_ENOMEM;
    if (!h->d_wy && hipMalloc(&h->d_wy, sizeof(float) * kMaxC) != hipSuccess) return FCM_ENOMEM;
    if (!h->d_wv0 && hipMalloc(&h->d_wv0, sizeof(double) * kMaxC) != hipSuccess) return FCM_ENOMEM;
    int64_t* off = nullptr;
    if (hipMalloc(&off, sizeof(int64_t) * 2) != hipSuccess) return FCM_ENOMEM;
    const int64_t range[2] = {0, h->n};
    hipError_t e = hipMemcpyAsync(off, range, sizeof(range), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        (void)hipFree(off);
        return dev_err(e, "hipMemcpyAsync");
    }
    h->d_woff = off;
    return FCM_OK;
}

// Clear the device state and mark the data-range pass as pending.  The
// cooperative exchange state is kept (its round count only grows) unless a
// wait was aborted, which clears it together with the tagged row buffers.
int enqueue_start(fcm_handle* h) {
    if (h->aborted) {
        FCM_HIP(hipMemsetAsync(h->d_state, 0, sizeof(DevState), h->stream));
        FCM_HIP(hipMemsetAsync(h->d_rows, 0, sizeof(uint64_t) * 2 * kMaxPersistGrid * kTaggedStrideMax, h->stream));
        FCM_HIP(hipMemsetAsync(h->d_mmrows, 0, sizeof(uint64_t) * 4 * kMaxPersistGrid, h->stream));
        if (h->d_ghist) FCM_HIP(hipMemsetAsync(h->d_ghist, 0, sizeof(uint32_t) * 2 * 256 * kHistCopies, h->stream));
        h->aborted = false;
    } else {
        FCM_HIP(hipMemsetAsync(h->d_state, 0, offsetof(DevState, sync), h->stream));
    }
    std::memset(h->h_state, 0, sizeof(DevState));
    h->h_state->iters = -1;
    h->h_state->status = FCM_RUNNING;
    h->kernel_ms = 0.0;
    h->pending_init = true;
    return FCM_OK;
}

// State as of the last completed work, running the data-range pass first if needed.
int sync_state(fcm_handle* h) {
    int rc = flush_init(h);
    if (rc != FCM_OK) return rc;
    return read_state(h);
}

void release(fcm_handle* h) {
    if (!h) return;
    drop_graph(h);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    if (h->d_state) (void)hipFree(h->d_state);
    if (h->d_partials) (void)hipFree(h->d_partials);
    if (h->d_minmax) (void)hipFree(h->d_minmax);
    if (h->d_rows) (void)hipFree(h->d_rows);
    if (h->d_mmrows) (void)hipFree(h->d_mmrows);
    if (h->d_hist) (void)hipFree(h->d_hist);
    for (void* p : {(void*)h->d_woff, (void*)h->d_wcounts, (void*)h->d_whist, (void*)h->d_wy, (void*)h->d_wv0,
                    (void*)h->d_ghist})
        if (p) (void)hipFree(p);
    if (h->h_state) (void)hipHostFree(h->h_state);
    delete h;
}

}  // namespace

extern "C" {

int fcm_version(void) { return 1 * 10000 + 1 * 100 + 0; }

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
        case FCM_EIO: return "file could not be read or written, or has the wrong layout";
        default: return "unknown status";
    }
}

const char* fcm_last_error(void) { return last_error().c_str(); }

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
    if (p->init == FCM_INIT_DEVICE) h->dv0 = p->init_centroids;
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
    if (hipDeviceGetAttribute(&h->coop, hipDeviceAttributeCooperativeLaunch, h->device) != hipSuccess) h->coop = 0;
    int clock_khz = 0;
    if (hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, h->device) != hipSuccess || clock_khz <= 0)
        clock_khz = 100000;
    h->clock_khz = (uint64_t)clock_khz;
    h->spin_ticks = h->default_ticks = (uint64_t)(kBarrierLimitSeconds * 1000.0 * clock_khz);
    h->tun.block = kBlock;
    h->tun.grid = 0;
    h->tun.unroll = 1;
    h->tun.driver = h->coop ? FCM_DRIVER_PERSISTENT : FCM_DRIVER_GRAPH;
    h->tun.graph_k = 8;
    h->tun.exchange = FCM_EXCHANGE_AUTO;
    h->tun.launch = FCM_LAUNCH_RESIDENT;
    if ((rc = resolve_grid(h, &h->grid)) != FCM_OK) return fail(rc);

    if (hipMalloc(&h->d_state, sizeof(DevState)) != hipSuccess) return fail(FCM_ENOMEM);
    if (hipMalloc(&h->d_partials, sizeof(float) * partial_rows(kMaxC) * kMaxGrid) != hipSuccess)
        return fail(FCM_ENOMEM);
    if (hipMalloc(&h->d_minmax, sizeof(uint32_t) * 2 * kMaxGrid) != hipSuccess) return fail(FCM_ENOMEM);
    if (hipMalloc(&h->d_rows, sizeof(uint64_t) * 2 * kMaxPersistGrid * kTaggedStrideMax) != hipSuccess)
        return fail(FCM_ENOMEM);
    if (hipMalloc(&h->d_mmrows, sizeof(uint64_t) * 4 * kMaxPersistGrid) != hipSuccess) return fail(FCM_ENOMEM);
    const size_t hist_doubles = (size_t)(p->max_iter + 2) * (C + 2);
    if (hipMalloc(&h->d_hist, sizeof(double) * hist_doubles) != hipSuccess) return fail(FCM_ENOMEM);
    if (hipHostMalloc(&h->h_state, sizeof(DevState), hipHostMallocDefault) != hipSuccess) return fail(FCM_ENOMEM);
    h->aborted = true;  // first start clears the handshake and the flags too
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
    if (t->driver == FCM_DRIVER_PERSISTENT && !h->coop) return FCM_EUNSUPPORTED;
    if (t->driver == FCM_DRIVER_HISTOGRAM && h->p.init == FCM_INIT_RANDOM_U) return FCM_EINVAL;
    if (t->exchange == FCM_EXCHANGE_XCD && (h->p.flags & FCM_F_KAHAN_ONLY)) return FCM_EUNSUPPORTED;
    const fcm_tuning old = h->tun;
    h->tun = *t;
    int grid = 1;
    rc = resolve_grid(h, &grid);
    if (rc != FCM_OK) {
        h->tun = old;
        return rc;
    }
    h->grid = grid;
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
    int rc = h->pending_init ? FCM_OK : read_state(h);
    if (rc != FCM_OK) return rc;
    int remaining = k;
    while (remaining > 0 && (h->pending_init || !h->h_state->done)) {
        const int batch = (h->tun.driver == FCM_DRIVER_PERSISTENT || h->tun.driver == FCM_DRIVER_HISTOGRAM)
                              ? remaining
                              : std::min(remaining, h->tun.graph_k);
        rc = run_batch(h, batch);
        if (rc != FCM_OK) return rc;
        remaining -= batch;
    }
    if (h->pending_init) {
        rc = sync_state(h);
        if (rc != FCM_OK) return rc;
    }
    fill_result(h, out);
    return out->status;
}

int fcm_solve(fcm_handle* h, fcm_result* out) {
    if (!h || !out) return FCM_EINVAL;
    int rc = h->pending_init ? FCM_OK : read_state(h);
    if (rc != FCM_OK) return rc;
    // A resident launch assumes that its whole grid is on the device at once;
    // another kernel holding CUs can keep some blocks waiting until a wait
    // gives up.  A solve that began from its start then runs once more from
    // the start in a cooperative launch, whose grid the runtime makes
    // co-resident (same iteration, same result).
    const bool fresh = h->pending_init;
    bool retried = false;
    // every pass either finishes the solve or advances the pass index, so
    // max_iter + 1 passes always suffice; the bound guards the host loop
    const int64_t total = (int64_t)h->p.max_iter + 1;
    int64_t budget = total + h->tun.graph_k;
    while ((h->pending_init || !h->h_state->done) && budget > 0) {
        const int batch = (h->tun.driver == FCM_DRIVER_PERSISTENT || h->tun.driver == FCM_DRIVER_HISTOGRAM)
                              ? (int)total
                              : h->tun.graph_k;
        rc = run_batch(h, batch);
        if (rc == FCM_EDEVICE && h->aborted && fresh && !retried && h->coop &&
            h->tun.driver == FCM_DRIVER_PERSISTENT && h->tun.launch == FCM_LAUNCH_RESIDENT) {
            retried = true;
            if ((rc = enqueue_start(h)) != FCM_OK) return rc;
            h->coop_retry = true;
            budget = total + h->tun.graph_k;
            continue;
        }
        if (rc != FCM_OK) {
            h->coop_retry = false;
            return rc;
        }
        budget -= batch;
    }
    if (h->coop_retry) {
        h->coop_retry = false;
        ++h->recoveries;
        last_error() = "a resident launch gave up waiting; the solve was run again in a cooperative launch";
    }
    fill_result(h, out);
    return out->status;
}

int fcm_solve_async(fcm_handle* h, uint8_t* d_labels) {
    if (!h) return FCM_EINVAL;
    if (h->tun.driver != FCM_DRIVER_PERSISTENT || h->p.init == FCM_INIT_RANDOM_U) {
        // host-driven solves: the synchronous path
        fcm_result r;
        int rc = fold_async(h);
        if (rc != FCM_OK) return rc;
        rc = enqueue_start(h);
        if (rc != FCM_OK) return rc;
        rc = fcm_solve(h, &r);
        if (rc < 0 && rc != FCM_ENUMERIC) return rc;
        h->async_ms += r.kernel_ms;
        return d_labels ? fcm_labels(h, d_labels) : FCM_OK;
    }
    // A fresh persistent launch writes every result field of the state itself
    // (the data-range pass commits the start) and reads none, so the clear
    // of a reset is skipped unless an abort left the exchange words unknown.
    if (h->aborted) {
        int rc = enqueue_start(h);
        if (rc != FCM_OK) return rc;
    } else {
        std::memset(h->h_state, 0, sizeof(DevState));
        h->h_state->iters = -1;
        h->h_state->status = FCM_RUNNING;
        h->kernel_ms = 0.0;
        h->pending_init = true;
    }
    PassArgs a = pass_args(h);
    a.max_passes = h->p.max_iter + 1;  // always enough: the launch ends the solve
    a.labels = d_labels;
    a.labels_bytewise = (((uintptr_t)h->d_x ^ (uintptr_t)d_labels) & 15) ? 1 : 0;
    const bool timing = (h->p.flags & FCM_F_TIMING) != 0;
    if (timing) {
        int rc = ensure_events(h, 2 * (h->async_timed + 1));
        if (rc != FCM_OK) return rc;
        FCM_HIP(hipEventRecord(h->ev[2 * h->async_timed], h->stream));
    }
    hipError_t e = launch_persist(a, h->p.n_clusters, h->mclass, h->tun.unroll, h->grid,
                                  h->tun.launch == FCM_LAUNCH_COOPERATIVE, h->stream);
    if (e != hipSuccess) return dev_err(e, "persistent launch");
    h->pending_init = false;
    if (timing) {
        FCM_HIP(hipEventRecord(h->ev[2 * h->async_timed + 1], h->stream));
        ++h->async_timed;
    }
    return FCM_OK;
}

int fcm_solve_wait(fcm_handle* h, fcm_result* out, int64_t* total_passes) {
    if (!h || !out) return FCM_EINVAL;
    int rc = h->pending_init ? sync_state(h) : read_state(h);
    if (rc != FCM_OK) return rc;
    if ((rc = fold_async(h)) != FCM_OK) return rc;
    const double ms = h->async_ms;
    h->async_ms = 0.0;
    fill_result(h, out);
    out->kernel_ms = ms > 0.0 ? ms : h->kernel_ms;
    if (total_passes) *total_passes = (int64_t)h->h_state->sync.passes_total;
    return out->status;
}

int fcm_solve_warm(fcm_handle* h, fcm_mlp* net, int32_t check, fcm_result* out, fcm_result* plain, int32_t* used) {
    if (!h || !net || !out) return FCM_EINVAL;
    if (mlp_clusters(net) != h->p.n_clusters) return FCM_EINVAL;
    int rc = ensure_level_ws(h);
    if (rc != FCM_OK) return rc;
    fcm_result rp{}, rw{};
    if (check) {  // the plain solve from the handle's own start
        if ((rc = enqueue_start(h)) != FCM_OK) return rc;
        if ((rc = fcm_solve(h, &rp)) < 0) return rc;
    }
    // learned start: histogram -> network (BF16) -> start centroids, then
    // Algorithm 1.  The persistent driver does all of it in its one launch
    // (the data-range pass counts the grey levels, block 0 runs the network);
    // the other drivers launch the histogram and network kernels first.  Both
    // ways run the same device code and give the same start.
    const int32_t own_init = h->p.init;
    const double* own_dv0 = h->dv0;
    if (h->tun.driver == FCM_DRIVER_PERSISTENT) {
        if (!h->d_ghist) {
            if (hipMalloc(&h->d_ghist, sizeof(uint32_t) * 2 * 256 * kHistCopies) != hipSuccess) return FCM_ENOMEM;
            FCM_HIP(hipMemsetAsync(h->d_ghist, 0, sizeof(uint32_t) * 2 * 256 * kHistCopies, h->stream));
        }
        h->mlp_w = mlp_bf16_weights(net, h->stream, &rc);
        if (rc != FCM_OK) return rc;
        h->p.init = kInitLearnedFused;
    } else {
        FCM_HIP(launch_histogram(h->d_x, h->d_woff, 1, h->n, h->d_wcounts, h->d_whist, h->stream));
        if ((rc = mlp_warm(net, h->d_whist, 1, h->d_wy, h->d_wv0, h->stream)) != FCM_OK) return rc;
        h->p.init = FCM_INIT_DEVICE;
        h->dv0 = h->d_wv0;
    }
    rc = enqueue_start(h);
    if (rc == FCM_OK) rc = fcm_solve(h, &rw);
    // a launch that ran to its end (converged, out of iterations or non-finite)
    // zeroed the other counter buffer: the next learned launch uses that one
    if (h->p.init == kInitLearnedFused && (rc >= 0 || rc == FCM_ENUMERIC)) h->ghist_sel ^= 1u;
    h->p.init = own_init;
    h->dv0 = own_dv0;
    h->mlp_w = nullptr;
    if (rc < 0) return rc;
    int use = 1;
    if (check) {
        use = rw.status != FCM_ENUMERIC && rw.J <= rp.J * (1.0 + 1e-6);
        if (plain) *plain = rp;
        if (!use) {  // fall back: run the plain solve again so that the handle holds it
            if ((rc = enqueue_start(h)) != FCM_OK) return rc;
            if ((rc = fcm_solve(h, &rw)) < 0) return rc;
        }
    }
    *out = rw;
    if (used) *used = use;
    return out->status;
}

int fcm_set_wait_limit(fcm_handle* h, double seconds, int32_t* recoveries) {
    if (!h) return FCM_EINVAL;
    if (seconds != 0.0 && !(std::isfinite(seconds) && seconds > 0.0 && seconds <= 60.0)) return FCM_EINVAL;
    if (seconds > 0.0) h->spin_ticks = std::max<uint64_t>(1, (uint64_t)(seconds * 1000.0 * (double)h->clock_khz));
    if (recoveries) *recoveries = h->recoveries;
    return FCM_OK;
}

int fcm_labels(fcm_handle* h, uint8_t* d_labels) {
    if (!h || !d_labels) return FCM_EINVAL;
    int rc = flush_init(h);
    if (rc != FCM_OK) return rc;
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
    int rc = sync_state(h);
    if (rc != FCM_OK) return rc;
    for (int k = 0; k < h->p.n_clusters; ++k) out[k] = h->h_state->vres[k];
    return FCM_OK;
}

int fcm_trajectory(fcm_handle* h, int32_t t, double* v_out, double* delta, double* J) {
    if (!h) return FCM_EINVAL;
    int rc = sync_state(h);
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

// ---------------------------------------------------------------------------
// batched solver
// ---------------------------------------------------------------------------

struct fcm_batch {
    const uint8_t* d_x = nullptr;
    int32_t count = 0;
    std::vector<int64_t> offsets;
    std::vector<fcm_params> p;
    std::vector<double> given;  // count * kMaxC
    std::vector<const double*> own_dv0;  // FCM_INIT_DEVICE start arrays of the caller
    hipStream_t stream = nullptr;
    int device = 0, ncu = 256, max_grid = 1, grid = 1, grid_req = 0;
    int block = kBatchBlock;       // threads per block of the batched kernel (128, 256 or 512)
    int chunks_per_thread = kBatchChunks;
    int fine_from = kBatchFineFrom;   // passes from this one on use the fine tiles
    int fine_chunks = kBatchFineChunks;  // chunks per thread of a fine tile
    int64_t coarse_tiles = 0;         // tiles of the coarse set (the first in the table)
    uint64_t spin_ticks = 0;
    double clock_mhz = 100.0;  // wall clock of the device
    uint32_t round = 0;        // largest tag used so far (tags of later solves start above it)
    bool solved = false;

    std::vector<BatchInst> h_inst;
    std::vector<BatchTile> h_tiles;
    int64_t hist_total = 0;

    BatchInst* d_inst = nullptr;
    int32_t* d_ntiles = nullptr;
    BatchTile* d_tiles = nullptr;
    BatchRec* d_recs = nullptr;
    double* d_hist = nullptr;
    uint64_t* d_rows = nullptr;
    uint64_t* d_dec = nullptr;
    uint64_t* d_ctl = nullptr;
    BatchSync* d_sync = nullptr;
    int64_t tiles_cap = 0;     // capacity of d_tiles / d_rows
    BatchRec* h_recs = nullptr;
    BatchSync* h_sync = nullptr;
    uint64_t* h_ctl = nullptr;

    // learned starts (first fcm_batch_set_start with a network)
    int64_t* d_off = nullptr;      // offsets [count + 1]
    uint32_t* d_counts = nullptr;  // [count][256]
    float* d_whist = nullptr;      // [count][256]
    float* d_wy = nullptr;         // [count][kMaxC]
    double* d_wv0 = nullptr;       // [count][kMaxC]
};

namespace {

void batch_free_tiles(fcm_batch* b) {
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_rows) (void)hipFree(b->d_rows);
    b->d_tiles = nullptr;
    b->d_rows = nullptr;
    b->tiles_cap = 0;
}

void batch_release(fcm_batch* b) {
    if (!b) return;
    batch_free_tiles(b);
    for (void* p : {(void*)b->d_inst, (void*)b->d_ntiles, (void*)b->d_recs, (void*)b->d_hist, (void*)b->d_dec,
                    (void*)b->d_ctl, (void*)b->d_sync, (void*)b->d_off, (void*)b->d_counts, (void*)b->d_whist,
                    (void*)b->d_wy, (void*)b->d_wv0})
        if (p) (void)hipFree(p);
    if (b->h_recs) (void)hipHostFree(b->h_recs);
    if (b->h_sync) (void)hipHostFree(b->h_sync);
    if (b->h_ctl) (void)hipHostFree(b->h_ctl);
    delete b;
}

// Cut every instance into two tile sets -- coarse tiles of 256 *
// chunks_per_thread chunks (phase 0 and the early passes), then fine tiles of
// 256 * fine_chunks chunks (the later passes); more chunks per tile where an
// instance would need more than kBatchMaxTiles tiles -- and upload the
// instance and tile tables (the coarse tiles of every instance first).  The
// tile-indexed buffers grow as needed and are cleared, so no stale tag can
// match.
int batch_build_tiles(fcm_batch* b) {
    b->h_tiles.clear();
    std::vector<int32_t> nt_of((size_t)b->count * 2);
    for (int set = 0; set < 2; ++set) {
        const int cpt = set ? b->fine_chunks : b->chunks_per_thread;
        for (int32_t i = 0; i < b->count; ++i) {
            BatchInst& in = b->h_inst[i];
            const int64_t tile_chunks =
                std::max<int64_t>((int64_t)b->block * cpt, (in.nbody + kBatchMaxTiles - 1) / kBatchMaxTiles);
            const int32_t first = (int32_t)b->h_tiles.size();
            int64_t c0 = 0;
            do {
                BatchTile t{};
                t.c0 = c0;
                t.c1 = std::min<int64_t>(in.nbody, c0 + tile_chunks);
                t.inst = i;
                t.ragged = c0 == 0 ? 1 : 0;
                b->h_tiles.push_back(t);
                c0 = t.c1;
            } while (c0 < in.nbody);
            const int32_t count = (int32_t)b->h_tiles.size() - first;
            (set ? in.tile0f : in.tile0) = first;
            (set ? in.ntilesf : in.ntiles) = count;
            nt_of[(size_t)i * 2 + set] = count;
        }
        if (!set) b->coarse_tiles = (int64_t)b->h_tiles.size();
    }
    const int64_t nt = (int64_t)b->h_tiles.size();
    if (nt > (int64_t)INT32_MAX) return FCM_EINVAL;
    if (nt > b->tiles_cap) {
        batch_free_tiles(b);
        if (hipMalloc(&b->d_tiles, sizeof(BatchTile) * nt) != hipSuccess) return FCM_ENOMEM;
        if (hipMalloc(&b->d_rows, sizeof(uint64_t) * kBatchRowWords * nt) != hipSuccess) return FCM_ENOMEM;
        b->tiles_cap = nt;
    }
    FCM_HIP(hipMemsetAsync(b->d_rows, 0, sizeof(uint64_t) * kBatchRowWords * b->tiles_cap, b->stream));
    FCM_HIP(hipMemsetAsync(b->d_dec, 0, sizeof(uint64_t) * kBatchDecWords * b->count, b->stream));
    FCM_HIP(hipMemcpyAsync(b->d_tiles, b->h_tiles.data(), sizeof(BatchTile) * nt, hipMemcpyHostToDevice, b->stream));
    FCM_HIP(hipMemcpyAsync(b->d_inst, b->h_inst.data(), sizeof(BatchInst) * b->count, hipMemcpyHostToDevice,
                           b->stream));
    FCM_HIP(hipMemcpyAsync(b->d_ntiles, nt_of.data(), sizeof(int32_t) * 2 * b->count, hipMemcpyHostToDevice,
                           b->stream));
    FCM_HIP(hipStreamSynchronize(b->stream));  // the host tables may change after return
    int64_t most = 0;
    for (const BatchInst& in : b->h_inst) most += std::max(in.ntiles, in.ntilesf);
    const int64_t want = b->grid_req > 0 ? b->grid_req : b->max_grid;
    b->grid = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(want, b->max_grid), most));
    b->round = 0;  // buffers were cleared: tags restart
    return FCM_OK;
}

}  // namespace

extern "C" {

int fcm_batch_init(fcm_batch** out, const uint8_t* d_x, const int64_t* offsets, int32_t count,
                   const fcm_params* params, void* stream) {
    if (!out || !d_x || !offsets || !params || count < 1) return FCM_EINVAL;
    if (offsets[0] != 0) return FCM_EINVAL;
    for (int32_t i = 0; i < count; ++i) {
        if (offsets[i + 1] <= offsets[i]) return FCM_EINVAL;
        int rc = validate_params(params + i);
        if (rc != FCM_OK) return rc;
        if (params[i].init == FCM_INIT_RANDOM_U) return FCM_EINVAL;  // single handles only
    }
    fcm_batch* b = new (std::nothrow) fcm_batch();
    if (!b) return FCM_ENOMEM;
    auto fail = [&](int code) {
        batch_release(b);
        return code;
    };
    b->d_x = d_x;
    b->count = count;
    b->offsets.assign(offsets, offsets + count + 1);
    b->p.assign(params, params + count);
    b->given.assign((size_t)count * kMaxC, 0.0);
    b->own_dv0.assign((size_t)count, nullptr);
    b->stream = (hipStream_t)stream;
    b->h_inst.resize(count);
    int64_t hist = 0;
    for (int32_t i = 0; i < count; ++i) {
        const fcm_params& q = params[i];
        if (q.init == FCM_INIT_GIVEN)
            for (int k = 0; k < q.n_clusters; ++k) b->given[(size_t)i * kMaxC + k] = q.init_centroids[k];
        b->p[i].init_centroids = nullptr;
        BatchInst& in = b->h_inst[i];
        std::memset(&in, 0, sizeof(in));
        in.base = offsets[i];
        in.n = offsets[i + 1] - offsets[i];
        const uintptr_t addr = (uintptr_t)(d_x + in.base);
        in.head = std::min<int64_t>(in.n, (int64_t)((16 - (addr & 15)) & 15));
        in.nbody = (in.n - in.head) / 16;
        in.hist = hist;
        hist += (int64_t)(q.max_iter + 2) * (q.n_clusters + 3);  // v, delta, J, commit times
        in.C = q.n_clusters;
        in.mclass = (q.m == 2.0) ? kM2 : (q.m == 1.5 ? kM15 : kMGeneric);
        in.max_iter = q.max_iter;
        in.kahan_only = (q.flags & FCM_F_KAHAN_ONLY) ? 1 : 0;
        in.given = start_mode(q.init);
        in.dv0 = q.init == FCM_INIT_DEVICE ? q.init_centroids : nullptr;
        b->own_dv0[(size_t)i] = in.dv0;
        in.alpha = (float)(1.0 / (q.m - 1.0));
        in.mexp = (float)q.m;
        in.eps = q.eps;
        for (int k = 0; k < kMaxC; ++k) in.v0[k] = b->given[(size_t)i * kMaxC + k];
    }
    b->hist_total = hist;
    hipError_t e;
    if ((e = hipGetDevice(&b->device)) != hipSuccess) return fail(dev_err(e, "hipGetDevice"));
    if ((e = hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, b->device)) != hipSuccess)
        return fail(dev_err(e, "hipDeviceGetAttribute"));
    int clock_khz = 0;
    if (hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, b->device) != hipSuccess || clock_khz <= 0)
        clock_khz = 100000;
    b->clock_mhz = clock_khz / 1000.0;
    b->spin_ticks = (uint64_t)(kBarrierLimitSeconds * 1000.0 * clock_khz);
    if ((e = batch_max_grid(b->block, b->ncu, &b->max_grid)) != hipSuccess) return fail(dev_err(e, "occupancy"));
    b->max_grid = std::max(1, std::min(b->max_grid, kMaxPersistGrid));

    if (hipMalloc(&b->d_inst, sizeof(BatchInst) * count) != hipSuccess) return fail(FCM_ENOMEM);
    if (hipMalloc(&b->d_ntiles, sizeof(int32_t) * 2 * count) != hipSuccess) return fail(FCM_ENOMEM);
    if (hipMalloc(&b->d_recs, sizeof(BatchRec) * count) != hipSuccess) return fail(FCM_ENOMEM);
    if (hipMalloc(&b->d_hist, sizeof(double) * hist) != hipSuccess) return fail(FCM_ENOMEM);
    if (hipMalloc(&b->d_dec, sizeof(uint64_t) * kBatchDecWords * count) != hipSuccess) return fail(FCM_ENOMEM);
    if (hipMalloc(&b->d_ctl, sizeof(uint64_t) * count) != hipSuccess) return fail(FCM_ENOMEM);
    if (hipMalloc(&b->d_sync, sizeof(BatchSync)) != hipSuccess) return fail(FCM_ENOMEM);
    if (hipHostMalloc(&b->h_recs, sizeof(BatchRec) * count, hipHostMallocDefault) != hipSuccess)
        return fail(FCM_ENOMEM);
    if (hipHostMalloc(&b->h_sync, sizeof(BatchSync), hipHostMallocDefault) != hipSuccess) return fail(FCM_ENOMEM);
    if (hipHostMalloc(&b->h_ctl, sizeof(uint64_t) * count, hipHostMallocDefault) != hipSuccess)
        return fail(FCM_ENOMEM);
    if ((e = hipMemsetAsync(b->d_recs, 0, sizeof(BatchRec) * count, b->stream)) != hipSuccess)
        return fail(dev_err(e, "hipMemsetAsync"));
    int rc = batch_build_tiles(b);
    if (rc != FCM_OK) return fail(rc);
    *out = b;
    return FCM_OK;
}

int fcm_batch_set_tiling(fcm_batch* b, int32_t chunks_per_thread, int32_t grid) {
    if (!b || chunks_per_thread < 1 || chunks_per_thread > 64 || grid < 0 || grid > kMaxPersistGrid)
        return FCM_EINVAL;
    b->chunks_per_thread = chunks_per_thread;
    b->grid_req = grid;
    b->solved = false;
    return batch_build_tiles(b);
}

int fcm_batch_set_block(fcm_batch* b, int32_t threads) {
    if (!b || (threads != 128 && threads != 256 && threads != 512)) return FCM_EINVAL;
    int max_grid = 0;
    hipError_t e = batch_max_grid(threads, b->ncu, &max_grid);
    if (e != hipSuccess) return dev_err(e, "occupancy");
    b->block = threads;
    b->max_grid = std::max(1, std::min(max_grid, kMaxPersistGrid));
    b->solved = false;
    return batch_build_tiles(b);
}

int fcm_batch_set_tail_tiling(fcm_batch* b, int32_t from_pass, int32_t chunks_per_thread) {
    if (!b || from_pass < 0 || chunks_per_thread < 1 || chunks_per_thread > 64) return FCM_EINVAL;
    b->fine_from = from_pass;
    b->fine_chunks = chunks_per_thread;
    b->solved = false;
    return batch_build_tiles(b);
}

int fcm_batch_set_start(fcm_batch* b, fcm_mlp* net, const uint8_t* use_learned) {
    if (!b) return FCM_EINVAL;
    const int C = net ? mlp_clusters(net) : 0;
    if (net) {
        const size_t cnt = (size_t)b->count;
        if (!b->d_off) {
            if (hipMalloc(&b->d_counts, sizeof(uint32_t) * 256 * cnt * histogram_copies(b->count)) != hipSuccess)
                return FCM_ENOMEM;
            if (hipMalloc(&b->d_whist, sizeof(float) * 256 * cnt) != hipSuccess) return FCM_ENOMEM;
            if (hipMalloc(&b->d_wy, sizeof(float) * kMaxC * cnt) != hipSuccess) return FCM_ENOMEM;
            if (hipMalloc(&b->d_wv0, sizeof(double) * kMaxC * cnt) != hipSuccess) return FCM_ENOMEM;
            int64_t* off = nullptr;
            if (hipMalloc(&off, sizeof(int64_t) * (cnt + 1)) != hipSuccess) return FCM_ENOMEM;
            FCM_HIP(hipMemcpyAsync(off, b->offsets.data(), sizeof(int64_t) * (cnt + 1), hipMemcpyHostToDevice,
                                   b->stream));
            FCM_HIP(hipStreamSynchronize(b->stream));
            b->d_off = off;
        }
        int64_t max_n = 1;
        for (int32_t i = 0; i < b->count; ++i) max_n = std::max<int64_t>(max_n, b->h_inst[i].n);
        FCM_HIP(launch_histogram(b->d_x, b->d_off, b->count, max_n, b->d_counts, b->d_whist, b->stream));
        int rc = mlp_warm(net, b->d_whist, b->count, b->d_wy, b->d_wv0, b->stream);
        if (rc != FCM_OK) return rc;
    }
    for (int32_t i = 0; i < b->count; ++i) {
        BatchInst& in = b->h_inst[i];
        if (net && in.C == C && (!use_learned || use_learned[i])) {
            in.given = 2;
            in.dv0 = b->d_wv0 + (int64_t)i * C;
        } else {
            in.given = start_mode(b->p[i].init);
            in.dv0 = b->own_dv0[(size_t)i];
        }
    }
    FCM_HIP(hipMemcpyAsync(b->d_inst, b->h_inst.data(), sizeof(BatchInst) * b->count, hipMemcpyHostToDevice,
                           b->stream));
    FCM_HIP(hipStreamSynchronize(b->stream));  // the host table may change after return
    return FCM_OK;
}

int fcm_batch_solve(fcm_batch* b, fcm_result* out) {
    if (!b || !out) return FCM_EINVAL;
    int max_iter = 1;
    for (const fcm_params& q : b->p) max_iter = std::max(max_iter, q.max_iter);
    // tags of this launch: round0 + 1 + phase, phases 0 .. max_iter + 1, and
    // the finished mark one above; restart (clearing every tagged word) before
    // they could wrap
    if ((uint64_t)b->round + (uint64_t)max_iter + 4 >= 0xFFFF0000ull) {
        int rc = batch_build_tiles(b);
        if (rc != FCM_OK) return rc;
    }
    const uint32_t round0 = b->round;
    for (int32_t i = 0; i < b->count; ++i) b->h_ctl[i] = (uint64_t)(round0 + 1u) << 32;
    int64_t tiles = 0;
    for (const BatchInst& in : b->h_inst) tiles += std::max(in.ntiles, in.ntilesf);
    b->h_sync->abort = 0;
    b->h_sync->active = (uint32_t)b->count;
    b->h_sync->tiles_left = (uint32_t)tiles;
    b->h_sync->epoch = 0;
    b->h_sync->t_start = 0;
    FCM_HIP(hipMemcpyAsync(b->d_ctl, b->h_ctl, sizeof(uint64_t) * b->count, hipMemcpyHostToDevice, b->stream));
    FCM_HIP(hipMemcpyAsync(b->d_sync, b->h_sync, sizeof(BatchSync), hipMemcpyHostToDevice, b->stream));
    BatchArgs a{};
    a.x = b->d_x;
    a.inst = b->d_inst;
    a.ntiles = b->d_ntiles;
    a.tiles = b->d_tiles;
    a.recs = b->d_recs;
    a.hist = b->d_hist;
    a.rows = b->d_rows;
    a.dec = b->d_dec;
    a.ctl = b->d_ctl;
    a.sync = b->d_sync;
    a.I = b->count;
    a.fine_from = b->fine_from;
    a.round0 = round0;
    a.spin_ticks = b->spin_ticks;
    hipError_t e = launch_batch(a, b->block, b->grid, b->stream);
    if (e != hipSuccess) return dev_err(e, "launch (batch)");
    FCM_HIP(hipMemcpyAsync(b->h_recs, b->d_recs, sizeof(BatchRec) * b->count, hipMemcpyDeviceToHost, b->stream));
    FCM_HIP(hipMemcpyAsync(b->h_sync, b->d_sync, sizeof(BatchSync), hipMemcpyDeviceToHost, b->stream));
    FCM_HIP(hipStreamSynchronize(b->stream));
    if (b->h_sync->abort || b->h_sync->active != 0u) {
        last_error() = "a wait of the batched solve exceeded its time limit";
        // clear every tagged buffer so that the next solve starts clean
        int rc = batch_build_tiles(b);
        return rc != FCM_OK ? rc : FCM_EDEVICE;
    }
    b->round = round0 + (uint32_t)max_iter + 3u;
    b->solved = true;
    int worst = FCM_OK;
    for (int32_t i = 0; i < b->count; ++i) {
        const BatchRec& r = b->h_recs[i];
        fcm_result& o = out[i];
        std::memset(&o, 0, sizeof(o));
        o.iters = r.iters < 0 ? 0 : r.iters;
        o.passes = r.passes;
        o.status = r.status;
        o.n_clusters = b->p[i].n_clusters;
        o.delta = r.delta;
        o.J = r.J;
        for (int k = 0; k < o.n_clusters; ++k) o.centroids[k] = r.vres[k];
        o.lo = r.lo;
        o.hi = r.hi;
        if (r.status == FCM_ENUMERIC) worst = FCM_ENUMERIC;
        else if (r.status != FCM_OK && worst == FCM_OK) worst = r.status;
    }
    return worst;
}

int fcm_batch_timeline(fcm_batch* b, int32_t inst, double* us, int32_t cap, int32_t* count) {
    if (!b || inst < 0 || inst >= b->count || (cap > 0 && !us) || cap < 0) return FCM_EINVAL;
    if (!b->solved) return FCM_ESTATE;
    const BatchInst& in = b->h_inst[inst];
    const int32_t nphase = b->h_recs[inst].passes + 1;
    if (count) *count = nphase;
    const int32_t m = std::min(cap, nphase);
    if (m <= 0) return FCM_OK;
    std::vector<uint64_t> ticks((size_t)m);
    const double* base = b->d_hist + in.hist + (int64_t)(in.max_iter + 2) * (in.C + 2);
    FCM_HIP(hipMemcpyAsync(ticks.data(), base, sizeof(uint64_t) * m, hipMemcpyDeviceToHost, b->stream));
    FCM_HIP(hipStreamSynchronize(b->stream));
    const uint64_t t0 = b->h_sync->t_start;
    for (int32_t q = 0; q < m; ++q) us[q] = (double)(int64_t)(ticks[(size_t)q] - t0) / b->clock_mhz;
    return FCM_OK;
}

int fcm_batch_solve_warm(fcm_batch* b, fcm_mlp* net, int32_t check, fcm_result* out, fcm_result* plain,
                         uint8_t* used) {
    if (!b || !net || !out) return FCM_EINVAL;
    const int C = mlp_clusters(net);
    const size_t cnt = (size_t)b->count;
    std::vector<fcm_result> rp;
    std::vector<uint8_t> learned(cnt);
    for (size_t i = 0; i < cnt; ++i) learned[i] = b->p[i].n_clusters == C ? 1 : 0;
    int rc;
    if (check) {  // the plain results: Algorithm 1 from each instance's own start
        rp.resize(cnt);
        if ((rc = fcm_batch_set_start(b, nullptr, nullptr)) != FCM_OK) return rc;
        if ((rc = fcm_batch_solve(b, rp.data())) < 0 && rc != FCM_ENUMERIC) return rc;
    }
    if ((rc = fcm_batch_set_start(b, net, learned.data())) != FCM_OK) return rc;
    if ((rc = fcm_batch_solve(b, out)) < 0 && rc != FCM_ENUMERIC) return rc;
    if (check) {
        bool differ = false;
        std::vector<uint8_t> keep(cnt);
        for (size_t i = 0; i < cnt; ++i) {
            keep[i] = learned[i] && out[i].status != FCM_ENUMERIC && out[i].J <= rp[i].J * (1.0 + 1e-6);
            differ |= keep[i] != learned[i];
        }
        if (differ) {  // fall back: one more launch so that the batch holds the returned results
            if ((rc = fcm_batch_set_start(b, net, keep.data())) != FCM_OK) return rc;
            if ((rc = fcm_batch_solve(b, out)) < 0 && rc != FCM_ENUMERIC) return rc;
        }
        learned.swap(keep);
        if (plain) std::memcpy(plain, rp.data(), sizeof(fcm_result) * cnt);
    }
    if (used) std::memcpy(used, learned.data(), cnt);
    return rc;
}

int fcm_batch_targets(fcm_batch* b, int32_t C, float* d_target) {
    if (!b || !d_target || C < 2 || C > FCM_MAX_CLUSTERS) return FCM_EINVAL;
    for (const fcm_params& q : b->p)
        if (q.n_clusters != C) return FCM_EINVAL;
    if (!b->solved) return FCM_ESTATE;
    hipError_t e = launch_batch_targets(b->d_recs, b->count, C, d_target, b->stream);
    if (e != hipSuccess) return dev_err(e, "launch_batch_targets");
    return FCM_OK;
}

int fcm_batch_labels(fcm_batch* b, uint8_t* d_labels) {
    if (!b || !d_labels) return FCM_EINVAL;
    if (!b->solved) return FCM_ESTATE;
    BatchLabelArgs a{};
    a.x = b->d_x;
    a.labels = d_labels;
    a.inst = b->d_inst;
    a.tiles = b->d_tiles;
    a.recs = b->d_recs;
    a.hist = b->d_hist;
    a.ntiles = (int32_t)b->coarse_tiles;  // the coarse set covers every voxel once
    a.bytewise = (((uintptr_t)b->d_x ^ (uintptr_t)d_labels) & 15) ? 1 : 0;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(a.ntiles, 4LL * b->ncu));
    hipError_t e = launch_batch_labels(a, grid, b->stream);
    if (e != hipSuccess) return dev_err(e, "launch_batch_labels");
    return FCM_OK;
}

int fcm_batch_trajectory(fcm_batch* b, int32_t inst, int32_t t, double* v_out, double* delta, double* J) {
    if (!b || inst < 0 || inst >= b->count) return FCM_EINVAL;
    if (!b->solved) return FCM_ESTATE;
    const BatchRec& r = b->h_recs[inst];
    if (t < 0 || t > r.iters) return FCM_EINVAL;
    const BatchInst& in = b->h_inst[inst];
    const int C = in.C;
    const double* hv = b->d_hist + in.hist;
    const double* hd = hv + (int64_t)(in.max_iter + 2) * C;
    const double* hJ = hd + (in.max_iter + 2);
    double row[kMaxC + 2];
    FCM_HIP(hipMemcpyAsync(row, hv + (int64_t)t * C, sizeof(double) * C, hipMemcpyDeviceToHost, b->stream));
    FCM_HIP(hipMemcpyAsync(row + C, hd + t, sizeof(double), hipMemcpyDeviceToHost, b->stream));
    FCM_HIP(hipMemcpyAsync(row + C + 1, hJ + t, sizeof(double), hipMemcpyDeviceToHost, b->stream));
    FCM_HIP(hipStreamSynchronize(b->stream));
    if (v_out) std::memcpy(v_out, row, sizeof(double) * C);
    if (delta) *delta = row[C];
    if (J) *J = row[C + 1];
    return FCM_OK;
}

void fcm_batch_destroy(fcm_batch* b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    batch_release(b);
}

}  // extern "C"

namespace fcm {

int handle_shape(const fcm_handle* h, HandleShape* s) {
    if (!h || !s) return FCM_EINVAL;
    s->n = h->n;
    s->nbody = h->nbody;
    s->C = h->p.n_clusters;
    s->mclass = h->mclass;
    s->kahan = (h->p.flags & FCM_F_KAHAN_ONLY) ? 1 : 0;
    s->device = h->device;
    s->ncu = h->ncu;
    s->coop = h->coop;
    return FCM_OK;
}

int batch_shape(const fcm_batch* b, BatchShape* s) {
    if (!b || !s) return FCM_EINVAL;
    s->voxels = b->offsets.back();
    s->count = b->count;
    s->max_C = 0;
    for (const fcm_params& q : b->p) s->max_C = std::max(s->max_C, (int)q.n_clusters);
    s->device = b->device;
    s->max_grid = b->max_grid;
    s->chunks_per_thread = b->chunks_per_thread;
    s->grid = b->grid_req;
    s->block = b->block;
    return FCM_OK;
}

}  // namespace fcm
