// Host runtime of the learned warm start: the histogram -> centroid network,
// its training loop and its inference (C ABI declared in include/fcm.h).
//
// Everything numeric runs in the kernels of fcm_learn.hip; the host owns the
// buffers, draws the initial weights and the sample order from a counter
// generator, and sequences the launches of one training step:
//   gather the minibatch -> three forward GEMMs (bias and ReLU fused) ->
//   loss and dL/dy -> backward GEMMs (ReLU masks fused) and bias column sums
//   -> Adam over the flat parameter vector.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fcm.h"
#include "fcm_host.h"
#include "fcm_internal.h"
#include "fcm_learn.h"

using namespace fcm;

namespace {

constexpr int kIn = 256, kH1 = 128, kH2 = 64;
constexpr int kMaxBatch = 4096;

// offsets of the parameter blocks in the flat vector
struct Layout {
    int64_t W1, b1, W2, b2, W3, b3, total;
    explicit Layout(int C) {
        W1 = 0;
        b1 = W1 + (int64_t)kIn * kH1;
        W2 = b1 + kH1;
        b2 = W2 + (int64_t)kH1 * kH2;
        W3 = b2 + kH2;
        b3 = W3 + (int64_t)kH2 * C;
        total = b3 + C;
    }
};

// SplitMix64 finaliser over a counter: the generator behind the weight
// initialisation and the shuffles (Steele, Lea and Flood, OOPSLA 2014).
uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// uniform in (0, 1) from stream `key`, element i
double uniform(uint64_t key, uint64_t i) {
    return ((double)(splitmix64(key * 0xD1B54A32D192ED03ull + i) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

// standard normal by Box-Muller from the pair (2i, 2i + 1)
double normal(uint64_t key, uint64_t i) {
    const double u1 = uniform(key, 2 * i), u2 = uniform(key, 2 * i + 1);
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

}  // namespace

struct fcm_mlp {
    int C = 4;
    int64_t P = 0;
    hipStream_t stream = nullptr;
    float* theta = nullptr;
    float* grad = nullptr;
    float* am = nullptr;  // Adam first moment
    float* av = nullptr;  // Adam second moment
    uint16_t* wb = nullptr;  // BF16 copy of theta for inference
    bool wb_stale = true;
    int step = 0;         // Adam steps taken
    uint64_t seed = 0;    // creation seed (or the seed of the file loaded)

    // training workspace, `cap` rows
    int cap = 0;
    float *Xb = nullptr, *Tb = nullptr, *h1 = nullptr, *h2 = nullptr, *y = nullptr, *dy = nullptr,
          *dz2 = nullptr, *dz1 = nullptr;
    float* losses = nullptr;  // per-step losses of one epoch
    int64_t loss_cap = 0;
    int32_t* idx = nullptr;   // sample order of one epoch
    int64_t idx_cap = 0;
    float* ybuf = nullptr;    // inference output scratch (fcm_warm_centroids)
    int64_t ybuf_cap = 0;
};

namespace {

void free_ptr(void* p) {
    if (p) (void)hipFree(p);
}

void mlp_release(fcm_mlp* n) {
    if (!n) return;
    for (void* p : {(void*)n->theta, (void*)n->grad, (void*)n->am, (void*)n->av, (void*)n->wb, (void*)n->Xb,
                    (void*)n->Tb, (void*)n->h1, (void*)n->h2, (void*)n->y, (void*)n->dy, (void*)n->dz2,
                    (void*)n->dz1, (void*)n->losses, (void*)n->idx, (void*)n->ybuf})
        free_ptr(p);
    delete n;
}

template <typename T>
int grow(T*& p, int64_t& cap, int64_t want, hipStream_t s) {
    if (want <= cap) return FCM_OK;
    FCM_HIP(hipStreamSynchronize(s));
    free_ptr(p);
    p = nullptr;
    cap = 0;
    if (hipMalloc(&p, sizeof(T) * (size_t)want) != hipSuccess) return FCM_ENOMEM;
    cap = want;
    return FCM_OK;
}

int ensure_rows(fcm_mlp* n, int rows) {
    if (rows <= n->cap) return FCM_OK;
    FCM_HIP(hipStreamSynchronize(n->stream));
    for (float** p : {&n->Xb, &n->Tb, &n->h1, &n->h2, &n->y, &n->dy, &n->dz2, &n->dz1}) {
        free_ptr(*p);
        *p = nullptr;
    }
    n->cap = 0;
    const size_t r = (size_t)rows;
    if (hipMalloc(&n->Xb, sizeof(float) * r * kIn) != hipSuccess) return FCM_ENOMEM;
    if (hipMalloc(&n->Tb, sizeof(float) * r * n->C) != hipSuccess) return FCM_ENOMEM;
    if (hipMalloc(&n->h1, sizeof(float) * r * kH1) != hipSuccess) return FCM_ENOMEM;
    if (hipMalloc(&n->h2, sizeof(float) * r * kH2) != hipSuccess) return FCM_ENOMEM;
    if (hipMalloc(&n->y, sizeof(float) * r * n->C) != hipSuccess) return FCM_ENOMEM;
    if (hipMalloc(&n->dy, sizeof(float) * r * n->C) != hipSuccess) return FCM_ENOMEM;
    if (hipMalloc(&n->dz2, sizeof(float) * r * kH2) != hipSuccess) return FCM_ENOMEM;
    if (hipMalloc(&n->dz1, sizeof(float) * r * kH1) != hipSuccess) return FCM_ENOMEM;
    n->cap = rows;
    return FCM_OK;
}

// FP32 forward of `rows` samples already in Xb: h1, h2, y.
int forward_f32(fcm_mlp* n, int rows) {
    const Layout L(n->C);
    const float* th = n->theta;
    hipStream_t s = n->stream;
    FCM_HIP(launch_gemm(false, false, n->Xb, th + L.W1, n->h1, rows, kH1, kIn, th + L.b1, 1, nullptr, s));
    FCM_HIP(launch_gemm(false, false, n->h1, th + L.W2, n->h2, rows, kH2, kH1, th + L.b2, 1, nullptr, s));
    FCM_HIP(launch_gemm(false, false, n->h2, th + L.W3, n->y, rows, n->C, kH2, th + L.b3, 0, nullptr, s));
    return FCM_OK;
}

// Loss slot and dL/dy from y and Tb, then the gradient into n->grad.  The
// ReLU derivative is taken from the stored activations (h > 0 exactly where
// the pre-activation is > 0).
int backward(fcm_mlp* n, int rows, float* loss_slot) {
    const Layout L(n->C);
    const int C = n->C;
    const float* th = n->theta;
    float* g = n->grad;
    hipStream_t s = n->stream;
    FCM_HIP(launch_mse(n->y, n->Tb, rows * C, 1.0f / (float)(rows * C), n->dy, loss_slot, s));
    FCM_HIP(launch_gemm(true, false, n->h2, n->dy, g + L.W3, kH2, C, rows, nullptr, 0, nullptr, s));
    FCM_HIP(launch_colsum(n->dy, rows, C, g + L.b3, s));
    FCM_HIP(launch_gemm(false, true, n->dy, th + L.W3, n->dz2, rows, kH2, C, nullptr, 0, n->h2, s));
    FCM_HIP(launch_gemm(true, false, n->h1, n->dz2, g + L.W2, kH1, kH2, rows, nullptr, 0, nullptr, s));
    FCM_HIP(launch_colsum(n->dz2, rows, kH2, g + L.b2, s));
    FCM_HIP(launch_gemm(false, true, n->dz2, th + L.W2, n->dz1, rows, kH1, kH2, nullptr, 0, n->h1, s));
    FCM_HIP(launch_gemm(true, false, n->Xb, n->dz1, g + L.W1, kIn, kH1, rows, nullptr, 0, nullptr, s));
    FCM_HIP(launch_colsum(n->dz1, rows, kH1, g + L.b1, s));
    return FCM_OK;
}

int refresh_bf16(fcm_mlp* n, hipStream_t s) {
    if (!n->wb_stale) return FCM_OK;
    if (s != n->stream) FCM_HIP(hipStreamSynchronize(n->stream));
    FCM_HIP(launch_to_bf16(n->theta, n->wb, n->C, s));
    if (s != n->stream) FCM_HIP(hipStreamSynchronize(s));
    n->wb_stale = false;
    return FCM_OK;
}

// ---- network files ----

constexpr char kMagic[8] = {'F', 'C', 'M', 'M', 'L', 'P', '0', '1'};
constexpr uint32_t kFileVersion = 1;
constexpr uint32_t kDtypeF32 = 0;

struct FileHeader {
    char magic[8];
    uint32_t version, dtype;
    int32_t n_in, h1, h2, C;
    int64_t n_params;
    uint64_t seed, layout, checksum;
};
static_assert(sizeof(FileHeader) == 64, "network file header is 64 bytes");

// FNV-1a, 64-bit (Fowler, Noll and Vo): offset basis and prime as published
uint64_t fnv1a(const void* data, size_t len, uint64_t h = 0xCBF29CE484222325ull) {
    const unsigned char* p = static_cast<const unsigned char*>(data);
    for (size_t i = 0; i < len; ++i) {
        h ^= p[i];
        h *= 0x100000001B3ull;
    }
    return h;
}

uint64_t layout_hash(const FileHeader& f) {
    const uint32_t w[8] = {f.version, f.dtype, (uint32_t)f.n_in, (uint32_t)f.h1, (uint32_t)f.h2, (uint32_t)f.C,
                           (uint32_t)((uint64_t)f.n_params & 0xFFFFFFFFu), (uint32_t)((uint64_t)f.n_params >> 32)};
    return fnv1a(w, sizeof(w));
}

}  // namespace

namespace fcm {

int mlp_clusters(const fcm_mlp* net) { return net ? net->C : 0; }

const uint16_t* mlp_bf16_weights(fcm_mlp* net, hipStream_t s, int* rc) {
    *rc = refresh_bf16(net, s);
    return net->wb;
}

int mlp_warm(fcm_mlp* net, const float* d_hist, int count, float* d_y, double* d_v0, hipStream_t s) {
    int rc = refresh_bf16(net, s);
    if (rc != FCM_OK) return rc;
    FCM_HIP(launch_mlp_infer(net->wb, true, d_hist, count, net->C, d_y, s));
    FCM_HIP(launch_warm_post(d_y, d_hist, count, net->C, d_v0, s));
    return FCM_OK;
}

}  // namespace fcm

extern "C" {

int32_t fcm_mlp_param_count(int32_t C) {
    if (C < 2 || C > FCM_MAX_CLUSTERS) return FCM_EINVAL;
    return (int32_t)Layout(C).total;
}

int fcm_mlp_create(fcm_mlp** out, int32_t C, uint64_t seed, void* stream) {
    if (!out || C < 2 || C > FCM_MAX_CLUSTERS) return FCM_EINVAL;
    fcm_mlp* n = new (std::nothrow) fcm_mlp();
    if (!n) return FCM_ENOMEM;
    auto fail = [&](int code) {
        mlp_release(n);
        return code;
    };
    n->C = C;
    n->seed = seed;
    const Layout L(C);
    n->P = L.total;
    n->stream = (hipStream_t)stream;
    const size_t bytes = sizeof(float) * (size_t)n->P;
    if (hipMalloc(&n->theta, bytes) != hipSuccess) return fail(FCM_ENOMEM);
    if (hipMalloc(&n->grad, bytes) != hipSuccess) return fail(FCM_ENOMEM);
    if (hipMalloc(&n->am, bytes) != hipSuccess) return fail(FCM_ENOMEM);
    if (hipMalloc(&n->av, bytes) != hipSuccess) return fail(FCM_ENOMEM);
    if (hipMalloc(&n->wb, sizeof(uint16_t) * (size_t)n->P) != hipSuccess) return fail(FCM_ENOMEM);
    // He initialisation: W ~ N(0, 2 / fan_in), b = 0
    std::vector<float> h((size_t)n->P, 0.0f);
    const struct { int64_t off, rows, cols; } blocks[3] = {{L.W1, kIn, kH1}, {L.W2, kH1, kH2}, {L.W3, kH2, C}};
    for (const auto& b : blocks) {
        const double sd = std::sqrt(2.0 / (double)b.rows);
        for (int64_t i = 0; i < b.rows * b.cols; ++i)
            h[(size_t)(b.off + i)] = (float)(sd * normal(seed, (uint64_t)(b.off + i)));
    }
    hipError_t e;
    if ((e = hipMemcpyAsync(n->theta, h.data(), bytes, hipMemcpyHostToDevice, n->stream)) != hipSuccess)
        return fail(dev_err(e, "hipMemcpyAsync"));
    if ((e = hipMemsetAsync(n->am, 0, bytes, n->stream)) != hipSuccess) return fail(dev_err(e, "hipMemsetAsync"));
    if ((e = hipMemsetAsync(n->av, 0, bytes, n->stream)) != hipSuccess) return fail(dev_err(e, "hipMemsetAsync"));
    if ((e = hipStreamSynchronize(n->stream)) != hipSuccess) return fail(dev_err(e, "hipStreamSynchronize"));
    *out = n;
    return FCM_OK;
}

int fcm_mlp_get_params(fcm_mlp* n, float* out) {
    if (!n || !out) return FCM_EINVAL;
    FCM_HIP(hipMemcpyAsync(out, n->theta, sizeof(float) * (size_t)n->P, hipMemcpyDeviceToHost, n->stream));
    FCM_HIP(hipStreamSynchronize(n->stream));
    return FCM_OK;
}

int fcm_mlp_set_params(fcm_mlp* n, const float* in) {
    if (!n || !in) return FCM_EINVAL;
    const size_t bytes = sizeof(float) * (size_t)n->P;
    FCM_HIP(hipMemcpyAsync(n->theta, in, bytes, hipMemcpyHostToDevice, n->stream));
    FCM_HIP(hipMemsetAsync(n->am, 0, bytes, n->stream));
    FCM_HIP(hipMemsetAsync(n->av, 0, bytes, n->stream));
    FCM_HIP(hipStreamSynchronize(n->stream));
    n->step = 0;
    n->wb_stale = true;
    return FCM_OK;
}

int fcm_mlp_save(fcm_mlp* n, const char* path) {
    if (!n || !path || !*path) return FCM_EINVAL;
    std::vector<float> theta((size_t)n->P);
    int rc = fcm_mlp_get_params(n, theta.data());
    if (rc != FCM_OK) return rc;
    FileHeader f{};
    std::memcpy(f.magic, kMagic, sizeof(kMagic));
    f.version = kFileVersion;
    f.dtype = kDtypeF32;
    f.n_in = kIn;
    f.h1 = kH1;
    f.h2 = kH2;
    f.C = n->C;
    f.n_params = n->P;
    f.seed = n->seed;
    f.layout = layout_hash(f);
    f.checksum = fnv1a(theta.data(), sizeof(float) * theta.size());
    const std::string tmp = std::string(path) + ".tmp";
    FILE* fp = std::fopen(tmp.c_str(), "wb");
    if (!fp) return FCM_EIO;
    bool ok = std::fwrite(&f, sizeof(f), 1, fp) == 1 &&
              std::fwrite(theta.data(), sizeof(float), theta.size(), fp) == theta.size();
    ok = (std::fclose(fp) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return FCM_EIO;
    }
    return FCM_OK;
}

int fcm_mlp_load(fcm_mlp* n, const char* path) {
    if (!n || !path || !*path) return FCM_EINVAL;
    FILE* fp = std::fopen(path, "rb");
    if (!fp) return FCM_EIO;
    FileHeader f{};
    std::vector<float> theta;
    int rc = FCM_OK;
    if (std::fread(&f, sizeof(f), 1, fp) != 1 || std::memcmp(f.magic, kMagic, sizeof(kMagic)) != 0 ||
        f.version != kFileVersion || f.dtype != kDtypeF32 || f.n_in != kIn || f.h1 != kH1 || f.h2 != kH2 ||
        f.C < 2 || f.C > FCM_MAX_CLUSTERS || f.n_params != Layout(f.C).total || f.layout != layout_hash(f)) {
        rc = FCM_EIO;
    } else if (f.C != n->C) {
        rc = FCM_EINVAL;
    } else {
        theta.resize((size_t)f.n_params);
        char extra;
        if (std::fread(theta.data(), sizeof(float), theta.size(), fp) != theta.size() ||
            std::fread(&extra, 1, 1, fp) != 0 || fnv1a(theta.data(), sizeof(float) * theta.size()) != f.checksum)
            rc = FCM_EIO;
    }
    std::fclose(fp);
    if (rc != FCM_OK) return rc;
    if ((rc = fcm_mlp_set_params(n, theta.data())) != FCM_OK) return rc;
    n->seed = f.seed;
    return FCM_OK;
}

int fcm_mlp_forward(fcm_mlp* n, const float* d_hist, int32_t count, float* d_out, int32_t precision) {
    if (!n || !d_hist || !d_out || count < 1) return FCM_EINVAL;
    if (precision != FCM_MLP_FP32 && precision != FCM_MLP_BF16) return FCM_EINVAL;
    if (precision == FCM_MLP_BF16) {
        int rc = refresh_bf16(n, n->stream);
        if (rc != FCM_OK) return rc;
        FCM_HIP(launch_mlp_infer(n->wb, true, d_hist, count, n->C, d_out, n->stream));
    } else {
        FCM_HIP(launch_mlp_infer(n->theta, false, d_hist, count, n->C, d_out, n->stream));
    }
    return FCM_OK;
}

int fcm_mlp_loss_grad(fcm_mlp* n, const float* d_hist, const float* d_target, int32_t count, double* loss,
                      float* grad) {
    if (!n || !d_hist || !d_target || count < 1 || count > (1 << 20)) return FCM_EINVAL;
    int rc = ensure_rows(n, count);
    if (rc != FCM_OK) return rc;
    if ((rc = grow(n->losses, n->loss_cap, 1, n->stream)) != FCM_OK) return rc;
    FCM_HIP(hipMemcpyAsync(n->Xb, d_hist, sizeof(float) * (size_t)count * kIn, hipMemcpyDeviceToDevice, n->stream));
    FCM_HIP(hipMemcpyAsync(n->Tb, d_target, sizeof(float) * (size_t)count * n->C, hipMemcpyDeviceToDevice,
                           n->stream));
    if ((rc = forward_f32(n, count)) != FCM_OK) return rc;
    if ((rc = backward(n, count, n->losses)) != FCM_OK) return rc;
    float l = 0.f;
    FCM_HIP(hipMemcpyAsync(&l, n->losses, sizeof(float), hipMemcpyDeviceToHost, n->stream));
    if (grad) FCM_HIP(hipMemcpyAsync(grad, n->grad, sizeof(float) * (size_t)n->P, hipMemcpyDeviceToHost, n->stream));
    FCM_HIP(hipStreamSynchronize(n->stream));
    if (loss) *loss = (double)l;
    return FCM_OK;
}

int fcm_mlp_train(fcm_mlp* n, const float* d_hist, const float* d_target, int32_t count, const fcm_train_cfg* cfg,
                  double* epoch_loss) {
    if (!n || !d_hist || !d_target || !cfg || count < 1) return FCM_EINVAL;
    if (cfg->epochs < 1 || cfg->batch < 1 || cfg->batch > kMaxBatch) return FCM_EINVAL;
    if (!std::isfinite(cfg->lr) || !(cfg->lr > 0.f)) return FCM_EINVAL;
    const int B = std::min<int>(cfg->batch, count);
    const int64_t nb = ((int64_t)count + B - 1) / B;
    int rc = ensure_rows(n, B);
    if (rc != FCM_OK) return rc;
    if ((rc = grow(n->losses, n->loss_cap, nb, n->stream)) != FCM_OK) return rc;
    if ((rc = grow(n->idx, n->idx_cap, count, n->stream)) != FCM_OK) return rc;
    std::vector<int32_t> order((size_t)count);
    std::vector<float> losses((size_t)nb);
    for (int ep = 0; ep < cfg->epochs; ++ep) {
        // Fisher-Yates shuffle drawn from (seed, epoch)
        for (int32_t i = 0; i < count; ++i) order[(size_t)i] = i;
        const uint64_t key = splitmix64(cfg->seed ^ (0xA5A5A5A5ull + (uint64_t)ep * 0x100000001B3ull));
        for (int32_t i = count - 1; i > 0; --i) {
            const int32_t j = (int32_t)std::min<double>(i, std::floor(uniform(key, (uint64_t)i) * (double)(i + 1)));
            std::swap(order[(size_t)i], order[(size_t)j]);
        }
        FCM_HIP(hipMemcpyAsync(n->idx, order.data(), sizeof(int32_t) * (size_t)count, hipMemcpyHostToDevice,
                               n->stream));
        for (int64_t b = 0; b < nb; ++b) {
            const int rows = (int)std::min<int64_t>(B, (int64_t)count - b * B);
            const int32_t* ib = n->idx + b * B;
            FCM_HIP(launch_gather(d_hist, ib, rows, kIn, n->Xb, n->stream));
            FCM_HIP(launch_gather(d_target, ib, rows, n->C, n->Tb, n->stream));
            if ((rc = forward_f32(n, rows)) != FCM_OK) return rc;
            if ((rc = backward(n, rows, n->losses + b)) != FCM_OK) return rc;
            FCM_HIP(launch_adam(n->theta, n->grad, n->am, n->av, n->P, cfg->lr, ++n->step, n->stream));
        }
        FCM_HIP(hipMemcpyAsync(losses.data(), n->losses, sizeof(float) * (size_t)nb, hipMemcpyDeviceToHost,
                               n->stream));
        FCM_HIP(hipStreamSynchronize(n->stream));
        if (epoch_loss) {
            double sum = 0.0;
            for (int64_t b = 0; b < nb; ++b)
                sum += (double)losses[(size_t)b] * (double)std::min<int64_t>(B, (int64_t)count - b * B);
            epoch_loss[ep] = sum / (double)count;
        }
    }
    n->wb_stale = true;
    return FCM_OK;
}

void fcm_mlp_destroy(fcm_mlp* n) {
    if (!n) return;
    (void)hipStreamSynchronize(n->stream);
    mlp_release(n);
}

int fcm_histogram(const uint8_t* d_x, const int64_t* offsets, int32_t count, float* d_hist, void* stream) {
    if (!d_x || !offsets || !d_hist || count < 1 || offsets[0] != 0) return FCM_EINVAL;
    int64_t max_n = 0;
    for (int32_t i = 0; i < count; ++i) {
        if (offsets[i + 1] <= offsets[i]) return FCM_EINVAL;
        max_n = std::max<int64_t>(max_n, offsets[i + 1] - offsets[i]);
    }
    if (max_n > (int64_t)UINT32_MAX) return FCM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int64_t* d_off = nullptr;
    uint32_t* d_counts = nullptr;
    if (hipMalloc(&d_off, sizeof(int64_t) * ((size_t)count + 1)) != hipSuccess) return FCM_ENOMEM;
    if (hipMalloc(&d_counts, sizeof(uint32_t) * 256 * (size_t)count * histogram_copies(count)) != hipSuccess) {
        (void)hipFree(d_off);
        return FCM_ENOMEM;
    }
    int rc = FCM_OK;
    hipError_t e = hipMemcpyAsync(d_off, offsets, sizeof(int64_t) * ((size_t)count + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_histogram(d_x, d_off, count, max_n, d_counts, d_hist, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = dev_err(e, "fcm_histogram");
    (void)hipFree(d_off);
    (void)hipFree(d_counts);
    return rc;
}

int fcm_warm_centroids(fcm_mlp* n, const float* d_hist, int32_t count, double* d_v0, void* stream) {
    if (!n || !d_hist || !d_v0 || count < 1) return FCM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int rc = grow(n->ybuf, n->ybuf_cap, (int64_t)count * n->C, s);
    if (rc != FCM_OK) return rc;
    return mlp_warm(n, d_hist, count, n->ybuf, d_v0, s);
}

}  // extern "C"
