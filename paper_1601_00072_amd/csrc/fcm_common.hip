// Non-template kernels: data range + v^0 (one launch) and defuzzification.
#include "fcm_device.h"

namespace fcm {

__global__ __launch_bounds__(kBlock) void fcm_init_kernel(InitArgs a) {
    uint32_t lo = 255u, hi = 0u;
    thread_minmax(a.x, a.n, a.head, a.nbody, lo, hi);
    const int G = gridDim.x;
    block_minmax(lo, hi);
    if (threadIdx.x == 0) {
        store_coherent(a.partials + blockIdx.x, lo);
        store_coherent(a.partials + G + blockIdx.x, hi);
    }
    if (!arrive_last(&a.st->ticket)) return;
    const uint32_t* part = a.partials;
    auto get = [&](int b, uint32_t& l, uint32_t& h) {
        l = part[b];
        h = part[G + b];
        return true;
    };
    reduce_minmax(get, G, lo, hi);
    if (threadIdx.x == 0) {
        double v[kMaxC];
        start_centroids(a.C, lo, hi, a.given, a.v0, a.dv0, v);
        commit_start(a.st, a.hist_v, a.C, lo, hi, v);
        a.st->ticket = 0;
    }
}

// ---------------------------------------------------------------------------
// defuzzification
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void fcm_labels_kernel(LabelArgs a) {
    __shared__ uint8_t lut[256];
    const int tid = threadIdx.x;
    {
        const int t = a.st->iters < 0 ? 0 : a.st->iters;
        const double* v = a.hist_v + (int64_t)t * a.C;
        for (int g = tid; g < 256; g += kBlock) {
            int best = 0;
            double bd = fabs((double)g - v[0]);
            for (int k = 1; k < a.C; ++k) {
                const double d = fabs((double)g - v[k]);
                if (d < bd) {
                    bd = d;
                    best = k;
                }
            }
            lut[g] = (uint8_t)best;
        }
    }
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t gt = (int64_t)blockIdx.x * kBlock + tid;
    if (a.bytewise) {
        for (int64_t i = gt; i < a.n; i += stride) a.labels[i] = lut[a.x[i]];
        return;
    }
    const uint4* in = reinterpret_cast<const uint4*>(a.x + a.head);
    uint4* out = reinterpret_cast<uint4*>(a.labels + a.head);
    for (int64_t c = gt; c < a.nbody; c += stride) {
        const uint4 w = in[c];
        uint32_t o[4];
        const uint32_t words[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t x = words[i];
            o[i] = (uint32_t)lut[x & 0xFFu] | ((uint32_t)lut[(x >> 8) & 0xFFu] << 8) |
                   ((uint32_t)lut[(x >> 16) & 0xFFu] << 16) | ((uint32_t)lut[x >> 24] << 24);
        }
        out[c] = make_uint4(o[0], o[1], o[2], o[3]);
    }
    if (blockIdx.x == 0) {
        const int64_t tail0 = a.head + 16 * a.nbody;
        const int64_t nr = a.head + (a.n - tail0);
        if (tid < nr) {
            const int64_t i = tid < a.head ? (int64_t)tid : tail0 + (tid - a.head);
            a.labels[i] = lut[a.x[i]];
        }
    }
}

hipError_t launch_init(const InitArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(fcm_init_kernel, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_labels(const LabelArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(fcm_labels_kernel, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace fcm
