// Learned warm start: grey-level histograms, and the histogram -> centroid
// network (256 -> 128 ReLU -> 64 ReLU -> C) trained and run by these kernels.
//
// Parameters live in one flat FP32 vector: W1 [256][128], b1, W2 [128][64], b2,
// W3 [64][C], b3 (row-major [in][out]).  Training: FP32 forward/backward on
// minibatches, mean squared error on the centroids divided by 255, Adam.
// Inference: BF16 weights and activations (round to nearest even), FP32
// accumulation, one block per histogram.  All reductions run in a fixed order
// (no floating-point atomics), so training is reproducible run to run.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "fcm.h"
#include "fcm_host.h"
#include "fcm_internal.h"
#include "fcm_learn.h"
#include "fcm_learn_dev.h"

namespace fcm {

constexpr int kWaveTables = kBlock / 64;

// ---------------------------------------------------------------------------
// histogram of each instance (integer counts, then normalised to sum 1)
// ---------------------------------------------------------------------------

// counts layout: [count][copies][256]; block x of instance y adds into copy
// x % copies (spreads the atomics of one busy level over `copies` addresses)
__global__ __launch_bounds__(kBlock) void hist_count_kernel(const uint8_t* x, const int64_t* offsets,
                                                            uint32_t* counts, int copies) {
    __shared__ uint32_t bins[kWaveTables][256];
    const int inst = blockIdx.y;
    const int tid = threadIdx.x;
    uint32_t* mine = bins[tid >> 6];  // one table per wave: fewer same-address conflicts
    for (int w = 0; w < kWaveTables; ++w) bins[w][tid] = 0u;
    __syncthreads();
    const int64_t b0 = offsets[inst], n = offsets[inst + 1] - b0;
    const uint8_t* xi = x + b0;
    const int64_t lead = (int64_t)((16 - ((uintptr_t)xi & 15)) & 15);
    const int64_t head = n < lead ? n : lead;
    const int64_t nbody = (n - head) / 16;
    const uint4* body = reinterpret_cast<const uint4*>(xi + head);
    for (int64_t c = (int64_t)blockIdx.x * kBlock + tid; c < nbody; c += (int64_t)gridDim.x * kBlock) {
        const uint4 w = body[c];
        const uint32_t words[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
            for (int b = 0; b < 4; ++b) atomicAdd(&mine[(words[q] >> (8 * b)) & 0xFFu], 1u);
        }
    }
    if (blockIdx.x == 0) {
        const int64_t tail0 = head + 16 * nbody;
        const int64_t nr = head + (n - tail0);
        for (int64_t r = tid; r < nr; r += kBlock) {
            const int64_t i = r < head ? r : tail0 + (r - head);
            atomicAdd(&mine[xi[i]], 1u);
        }
    }
    __syncthreads();
    uint32_t c = 0u;
    for (int w = 0; w < kWaveTables; ++w) c += bins[w][tid];
    if (c) atomicAdd(counts + ((int64_t)inst * copies + blockIdx.x % copies) * 256 + tid, c);
}

// totals of the copies -> copy 0 (integer counts) and count / n (FP64, stored FP32)
__global__ __launch_bounds__(kBlock) void hist_norm_kernel(uint32_t* counts, const int64_t* offsets, float* hist,
                                                           int copies) {
    const int inst = blockIdx.x;
    uint32_t* ci = counts + (int64_t)inst * copies * 256;
    uint32_t total = 0u;
    for (int c = 0; c < copies; ++c) total += ci[c * 256 + threadIdx.x];
    ci[threadIdx.x] = total;
    hist[(int64_t)inst * 256 + threadIdx.x] = hist_norm(total, offsets[inst + 1] - offsets[inst]);
}

int histogram_copies(int count) { return count == 1 ? kHistCopies : 1; }

// counting and normalisation on counters that are already zero
hipError_t launch_histogram_counts(const uint8_t* x, const int64_t* d_offsets, int count, int64_t max_n,
                                   uint32_t* counts, float* hist, hipStream_t s) {
    const int copies = histogram_copies(count);
    hipError_t e;
    const int64_t chunks = (max_n + 15) / 16;
    const int64_t cap = count == 1 ? 1024 : 64;  // a single instance may use the whole device
    int64_t gx64 = (chunks + kBlock * 16 - 1) / (kBlock * 16);
    gx64 = gx64 < 1 ? 1 : (gx64 > cap ? cap : gx64);
    const int gx = (int)gx64;
    constexpr int kMaxY = 65535;  // grid y limit: instances per launch
    for (int c0 = 0; c0 < count; c0 += kMaxY) {
        const int cnt = count - c0 < kMaxY ? count - c0 : kMaxY;
        hipLaunchKernelGGL(hist_count_kernel, dim3(gx, cnt), dim3(kBlock), 0, s, x, d_offsets + c0,
                           counts + (int64_t)c0 * copies * 256, copies);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(hist_norm_kernel, dim3(count), dim3(256), 0, s, counts, d_offsets, hist, copies);
    return hipGetLastError();
}

hipError_t launch_histogram(const uint8_t* x, const int64_t* d_offsets, int count, int64_t max_n, uint32_t* counts,
                            float* hist, hipStream_t s) {
    const int copies = histogram_copies(count);
    hipError_t e = hipMemsetAsync(counts, 0, sizeof(uint32_t) * 256 * (size_t)count * copies, s);
    if (e != hipSuccess) return e;
    return launch_histogram_counts(x, d_offsets, count, max_n, counts, hist, s);
}

// ---------------------------------------------------------------------------
// FP32 GEMM for training: Cm[M][N] = op(A) op(B) (+ bias[N]) (ReLU) (* mask>0)
// op(A) is A [M][K] or, transposed, A [K][M]; op(B) is B [K][N] or B [N][K].
// The training shapes are small (K and M up to 256 rows of a minibatch), so
// the output is cut into 16 x 16 tiles, one output per thread (enough blocks
// to spread over the chip), K in steps of 16 through LDS.  Each output is a
// sum over k in increasing order.
// ---------------------------------------------------------------------------

constexpr int kT = 16;  // 16 x 16 outputs per block, one per thread; K in steps of 16

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_kernel(const float* A, const float* B, float* Cm, int M, int N, int K,
                                                   const float* bias, int relu, const float* mask) {
    __shared__ float As[kT][kT + 1];  // [m][k]
    __shared__ float Bs[kT][kT + 1];  // [k][n]
    const int tx = threadIdx.x % kT, ty = threadIdx.x / kT;
    const int row0 = blockIdx.y * kT, col0 = blockIdx.x * kT;
    float acc = 0.f;
    for (int k0 = 0; k0 < K; k0 += kT) {
        // one element of each tile per thread; consecutive threads take
        // consecutive addresses of the stored layout (transposed operands
        // walk the tile the other way round)
        const int e = threadIdx.x;
        {
            const int r = TA ? e % kT : e / kT, c = TA ? e / kT : e % kT;
            const int gm = row0 + r, gk = k0 + c;
            float va = 0.f;
            if (gm < M && gk < K) va = TA ? A[(int64_t)gk * M + gm] : A[(int64_t)gm * K + gk];
            As[r][c] = va;
        }
        {
            const int rb = TB ? e % kT : e / kT, cb = TB ? e / kT : e % kT;
            const int gk = k0 + rb, gn = col0 + cb;
            float vb = 0.f;
            if (gk < K && gn < N) vb = TB ? B[(int64_t)gn * K + gk] : B[(int64_t)gk * N + gn];
            Bs[rb][cb] = vb;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kT; ++kk) acc = fmaf(As[ty][kk], Bs[kk][tx], acc);
        __syncthreads();
    }
    const int gm = row0 + ty, gn = col0 + tx;
    if (gm >= M || gn >= N) return;
    float v = acc;
    if (bias) v += bias[gn];
    if (relu) v = fmaxf(v, 0.f);
    if (mask && !(mask[(int64_t)gm * N + gn] > 0.f)) v = 0.f;
    Cm[(int64_t)gm * N + gn] = v;
}

hipError_t launch_gemm(bool ta, bool tb, const float* A, const float* B, float* Cm, int M, int N, int K,
                       const float* bias, int relu, const float* mask, hipStream_t s) {
    const dim3 grid((N + kT - 1) / kT, (M + kT - 1) / kT);
    if (!ta && !tb)
        hipLaunchKernelGGL((gemm_kernel<false, false>), grid, dim3(256), 0, s, A, B, Cm, M, N, K, bias, relu, mask);
    else if (ta && !tb)
        hipLaunchKernelGGL((gemm_kernel<true, false>), grid, dim3(256), 0, s, A, B, Cm, M, N, K, bias, relu, mask);
    else if (!ta && tb)
        hipLaunchKernelGGL((gemm_kernel<false, true>), grid, dim3(256), 0, s, A, B, Cm, M, N, K, bias, relu, mask);
    else
        hipLaunchKernelGGL((gemm_kernel<true, true>), grid, dim3(256), 0, s, A, B, Cm, M, N, K, bias, relu, mask);
    return hipGetLastError();
}

// column sums of G [M][N] into out[N]: a block takes 16 columns; its 16 row
// groups (thread (g, c) adds rows g, g + 16, ... of column c) run in
// parallel, then the groups are added in order g = 0..15 -- a fixed order, so
// the sums are reproducible run to run
constexpr int kColTile = 16, kRowGroups = 16;

__global__ __launch_bounds__(kColTile * kRowGroups) void colsum_kernel(const float* G, int M, int N, float* out) {
    __shared__ float part[kRowGroups][kColTile + 1];
    const int c = threadIdx.x % kColTile, g = threadIdx.x / kColTile;
    const int j = blockIdx.x * kColTile + c;
    float s = 0.f;
    if (j < N)
        for (int i = g; i < M; i += kRowGroups) s += G[(int64_t)i * N + j];
    part[g][c] = s;
    __syncthreads();
    if (g == 0 && j < N) {
        float t = part[0][c];
        for (int r = 1; r < kRowGroups; ++r) t += part[r][c];
        out[j] = t;
    }
}

hipError_t launch_colsum(const float* G, int M, int N, float* out, hipStream_t s) {
    hipLaunchKernelGGL(colsum_kernel, dim3((N + kColTile - 1) / kColTile), dim3(kColTile * kRowGroups), 0, s, G, M, N,
                       out);
    return hipGetLastError();
}

// dY = 2 (Y - T) / (B C); loss_out[slot] = sum (Y - T)^2 / (B C) (one block, fixed order)
__global__ __launch_bounds__(256) void mse_kernel(const float* Y, const float* T, int n, float scale, float* dY,
                                                  float* loss_out) {
    __shared__ double part[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const float d = Y[i] - T[i];
        dY[i] = 2.f * d * scale;
        s += (double)d * d;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss_out = (float)(part[0] * scale);
}

hipError_t launch_mse(const float* Y, const float* T, int n, float scale, float* dY, float* loss_out,
                      hipStream_t s) {
    hipLaunchKernelGGL(mse_kernel, dim3(1), dim3(256), 0, s, Y, T, n, scale, dY, loss_out);
    return hipGetLastError();
}

__global__ void adam_kernel(float* theta, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t launch_adam(float* theta, const float* g, float* m, float* v, int64_t n, float lr, int step,
                       hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, theta, g, m, v, n, lr, b1,
                       b2, 1e-8f, c1, c2);
    return hipGetLastError();
}

__global__ void gather_rows_kernel(const float* X, const int32_t* idx, int rows, int cols, float* out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * cols) return;
    const int r = (int)(e / cols), c = (int)(e % cols);
    out[e] = X[(int64_t)idx[r] * cols + c];
}

hipError_t launch_gather(const float* X, const int32_t* idx, int rows, int cols, float* out, hipStream_t s) {
    const int64_t n = (int64_t)rows * cols;
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, idx, rows, cols,
                       out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// BF16 inference
// ---------------------------------------------------------------------------

// BF16 inference copy (InferLayout) of the flat FP32 parameters, one thread
// per element of the copy.
__global__ void to_bf16_kernel(const float* theta, uint16_t* out, int C) {
    using L = InferLayout;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t fW1 = 0, fb1 = fW1 + 256 * 128, fW2 = fb1 + 128, fb2 = fW2 + 128 * 64, fW3 = fb2 + 64;
    const int64_t fb3 = fW3 + 64 * (int64_t)C;
    int64_t src;
    if (e < L::b1) src = fW1 + (e % 256) * 128 + e / 256;                      // W1t[o][i] = W1[i][o]
    else if (e < L::W2) src = fb1 + (e - L::b1);
    else if (e < L::b2) src = fW2 + ((e - L::W2) % 128) * 64 + (e - L::W2) / 128;
    else if (e < L::W3) src = fb2 + (e - L::b2);
    else if (e < L::b3(C)) src = fW3 + ((e - L::W3) % 64) * C + (e - L::W3) / 64;
    else if (e < L::b3(C) + C) src = fb3 + (e - L::b3(C));
    else return;
    out[e] = to_bf16(theta[src]);
}

hipError_t launch_to_bf16(const float* theta, uint16_t* out, int C, hipStream_t s) {
    const int64_t n = InferLayout::b3(C) + C;
    hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, theta, out, C);
    return hipGetLastError();
}

// One block (256 threads) per histogram (mlp_block_forward).
template <bool BF16>
__global__ __launch_bounds__(256) void mlp_infer_kernel(const void* w, const float* X, int C, float* Y) {
    __shared__ float a0[256];
    __shared__ float a1[128];
    __shared__ float a2[64];
    __shared__ float tmp[256];
    const int64_t s = blockIdx.x;
    mlp_block_forward<BF16>(w, X + s * 256, C, a0, a1, a2, tmp, Y + s * C);
}

hipError_t launch_mlp_infer(const void* w, bool bf16, const float* X, int count, int C, float* Y, hipStream_t s) {
    if (bf16)
        hipLaunchKernelGGL(mlp_infer_kernel<true>, dim3(count), dim3(256), 0, s, w, X, C, Y);
    else
        hipLaunchKernelGGL(mlp_infer_kernel<false>, dim3(count), dim3(256), 0, s, w, X, C, Y);
    return hipGetLastError();
}

// Network output -> start centroids, one thread per instance (warm_post_one).
__global__ void warm_post_kernel(const float* Y, const float* hist, int count, int C, double* v0) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    const float* h = hist + (int64_t)s * 256;
    int lo = 0, hi = 255;
    while (lo < 255 && !(h[lo] > 0.f)) ++lo;
    while (hi > 0 && !(h[hi] > 0.f)) --hi;
    warm_post_one(Y + (int64_t)s * C, lo, hi, C, v0 + (int64_t)s * C);
}

hipError_t launch_warm_post(const float* Y, const float* hist, int count, int C, double* v0, hipStream_t s) {
    hipLaunchKernelGGL(warm_post_kernel, dim3((count + 127) / 128), dim3(128), 0, s, Y, hist, count, C, v0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// histograms without allocation (fcm_histogram_noalloc)
// ---------------------------------------------------------------------------

// The workspace of fcm_histogram in a fixed device array: the instance
// offsets, then the counters ([count][copies][256]; one instance uses
// kHistCopies copies, more instances one copy each).  Each device holds its
// own copy of the array for the life of the process.
constexpr int kNoAllocMaxCount = 1024;
constexpr size_t kNoAllocOffBytes = (sizeof(int64_t) * (kNoAllocMaxCount + 1) + 255) / 256 * 256;
constexpr size_t kNoAllocCountWords = 256 * (size_t)kNoAllocMaxCount;
static_assert((size_t)kHistCopies <= (size_t)kNoAllocMaxCount, "one instance's copies fit");
static __device__ __align__(256) unsigned char scratch[kNoAllocOffBytes + sizeof(uint32_t) * kNoAllocCountWords];

__global__ __launch_bounds__(kBlock) void zero_words_kernel(uint32_t* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) p[i] = 0u;
}

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (in host code the array's
// name is not a device address); looked up once per device.
int scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return dev_err(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return FCM_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return dev_err(e == hipSuccess ? hipErrorInvalidSymbol : e, "hipGetSymbolAddress");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FCM_OK;
}

}  // namespace

}  // namespace fcm

extern "C" int fcm_histogram_noalloc(const uint8_t* d_x, const int64_t* offsets, int32_t count, float* d_hist,
                                     void* stream) {
    using namespace fcm;
    if (!d_x || !offsets || !d_hist || count < 1 || offsets[0] != 0) return FCM_EINVAL;
    int64_t max_n = 0;
    for (int32_t i = 0; i < count; ++i) {
        if (offsets[i + 1] <= offsets[i]) return FCM_EINVAL;
        max_n = offsets[i + 1] - offsets[i] > max_n ? offsets[i + 1] - offsets[i] : max_n;
    }
    if (max_n > (int64_t)UINT32_MAX) return FCM_EINVAL;
    if (count > kNoAllocMaxCount) {
        last_error() = "fcm_histogram_noalloc: more instances than its fixed workspace holds (1024)";
        return FCM_EINVAL;
    }
    void* base = nullptr;
    int rc = scratch_address(&base);
    if (rc != FCM_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    int64_t* d_off = reinterpret_cast<int64_t*>(base);
    uint32_t* d_counts = reinterpret_cast<uint32_t*>(static_cast<unsigned char*>(base) + kNoAllocOffBytes);
    const int64_t words = 256 * (int64_t)count * histogram_copies(count);
    FCM_HIP(hipMemcpyAsync(d_off, offsets, sizeof(int64_t) * ((size_t)count + 1), hipMemcpyHostToDevice, s));
    // the array keeps the previous call's counts: clear them (a kernel, no memset node)
    const int zgrid = (int)((words + kBlock - 1) / kBlock < 1024 ? (words + kBlock - 1) / kBlock : 1024);
    hipLaunchKernelGGL(zero_words_kernel, dim3(zgrid), dim3(kBlock), 0, s, d_counts, words);
    FCM_HIP(hipGetLastError());
    FCM_HIP(launch_histogram_counts(d_x, d_off, count, max_n, d_counts, d_hist, s));
    FCM_HIP(hipStreamSynchronize(s));
    return FCM_OK;
}
