// The paper's own GPU design (Sec. 4), rebuilt on gfx950 as a baseline: the
// membership matrix U lives in device memory, and every iteration runs, per
// cluster j, a per-pixel kernel for the Eq.3 numerator and denominator terms,
// two shared-memory tree reductions (Algorithm 2: blocks of 128 threads, two
// inputs per thread, n / (2 * 128) partial sums), and a one-thread kernel that
// adds the partial sums and divides; then, per cluster, a per-pixel kernel
// for Eq.4.  The host copies U back after every iteration and tests the
// change itself (fcm_paper_rt.cpp).  Written for measurement: it shows what
// the fused, device-resident design gains over this structure on the same
// chip.  Two readings: Algorithm 2 prints no barrier between tree levels (one
// is placed before each level here), and the one-thread sum accumulates in
// FP64 (the paper does not state its precision).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fcm_paper.h"

namespace fcm {

namespace {

// Eq.3 terms of cluster j for every pixel: a = u_ij^m, num_i = a x_i, den_i = a
__global__ __launch_bounds__(kPaperPixelBlock) void paper_terms_kernel(const float* U, const uint8_t* x, int64_t n,
                                                                       int j, float m, float* num, float* den) {
    const int64_t i = (int64_t)blockIdx.x * kPaperPixelBlock + threadIdx.x;
    if (i >= n) return;
    const float u = U[(int64_t)j * n + i];
    const float a = m == 2.0f ? u * u : powf(u, m);
    num[i] = a * (float)x[i];
    den[i] = a;
}

// The reduction structure of Algorithm 2 (Sec. 4.2): blocks of 128 threads,
// each thread first adds its two inputs -- elements t and t + 128 of the
// block's 256-element window, zero past n -- in a register, then the block
// halves its 128 sums in shared memory level by level (a barrier before
// every level) and stores one partial sum per block.
__global__ __launch_bounds__(kPaperReduceBlock) void paper_reduce_kernel(const float* A, int64_t n, float* Bout) {
    __shared__ float acc[kPaperReduceBlock];
    const int t = threadIdx.x;
    const int64_t window = (int64_t)blockIdx.x * (2 * kPaperReduceBlock);
    float s = 0.0f;
    for (int q = 0; q < 2; ++q) {
        const int64_t i = window + q * kPaperReduceBlock + t;
        if (i < n) s += A[i];
    }
    acc[t] = s;
    for (int width = kPaperReduceBlock / 2; width >= 1; width >>= 1) {
        __syncthreads();
        if (t < width) acc[t] += acc[t + width];
    }
    if (t == 0) Bout[blockIdx.x] = acc[0];
}

// one thread: the final sums of both reductions and the centroid of cluster j
__global__ void paper_centroid_kernel(const float* Bn, const float* Bd, int64_t parts, int j, double* v,
                                      float* v32) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double sn = 0.0, sd = 0.0;
    for (int64_t b = 0; b < parts; ++b) {
        sn += (double)Bn[b];
        sd += (double)Bd[b];
    }
    if (sd > 0.0) v[j] = sn / sd;  // an empty cluster keeps its centroid
    v32[j] = (float)v[j];
}

// Eq.4 as printed for cluster j: u_ij = 1 / sum_k (d_ij / d_ik)^(2/(m-1)),
// with the zero-distance rule (equal split over the clusters at distance 0)
__global__ __launch_bounds__(kPaperPixelBlock) void paper_memb_kernel(const uint8_t* x, int64_t n, const float* v32,
                                                                      int C, int j, float m, float* U) {
    const int64_t i = (int64_t)blockIdx.x * kPaperPixelBlock + threadIdx.x;
    if (i >= n) return;
    const float xi = (float)x[i];
    const float dj = fabsf(xi - v32[j]);
    const float e = 2.0f / (m - 1.0f);
    int zeros = 0;
    float s = 0.0f;
    for (int k = 0; k < C; ++k) {
        const float dk = fabsf(xi - v32[k]);
        zeros += dk == 0.0f;
        const float r = dj / dk;
        s += m == 2.0f ? r * r : powf(r, e);
    }
    U[(int64_t)j * n + i] = zeros ? (dj == 0.0f ? 1.0f / (float)zeros : 0.0f) : 1.0f / s;
}

}  // namespace

int64_t paper_parts(int64_t n) { return (n + 2 * kPaperReduceBlock - 1) / (2 * kPaperReduceBlock); }

hipError_t paper_centroids(const PaperBuffers& b, int C, float m, hipStream_t s) {
    const unsigned gp = (unsigned)((b.n + kPaperPixelBlock - 1) / kPaperPixelBlock);
    const unsigned gr = (unsigned)paper_parts(b.n);
    for (int j = 0; j < C; ++j) {
        hipLaunchKernelGGL(paper_terms_kernel, dim3(gp), dim3(kPaperPixelBlock), 0, s, b.U, b.x, b.n, j, m, b.num,
                           b.den);
        hipLaunchKernelGGL(paper_reduce_kernel, dim3(gr), dim3(kPaperReduceBlock), 0, s, b.num, b.n, b.bnum);
        hipLaunchKernelGGL(paper_reduce_kernel, dim3(gr), dim3(kPaperReduceBlock), 0, s, b.den, b.n, b.bden);
        hipLaunchKernelGGL(paper_centroid_kernel, dim3(1), dim3(1), 0, s, b.bnum, b.bden, (int64_t)gr, j, b.v,
                           b.v32);
    }
    return hipGetLastError();
}

hipError_t paper_memberships(const PaperBuffers& b, int C, float m, hipStream_t s) {
    const unsigned gp = (unsigned)((b.n + kPaperPixelBlock - 1) / kPaperPixelBlock);
    for (int j = 0; j < C; ++j)
        hipLaunchKernelGGL(paper_memb_kernel, dim3(gp), dim3(kPaperPixelBlock), 0, s, b.x, b.n, b.v32, C, j, m,
                           b.U);
    return hipGetLastError();
}

}  // namespace fcm
