// The paper's GPU design as a baseline (fcm_paper.hip kernels, host loop in
// fcm_paper_rt.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fcm {

constexpr int kPaperPixelBlock = 256;   // per-pixel kernels: one thread per pixel
constexpr int kPaperReduceBlock = 128;  // Algorithm 2: blockDim 128, two inputs per thread

struct PaperBuffers {
    const uint8_t* x;
    int64_t n;
    float* U;            // [C][n] memberships, cluster-major
    float* num;          // [n] Eq.3 numerator terms of one cluster
    float* den;          // [n] denominator terms
    float* bnum;         // [paper_parts(n)] partial sums
    float* bden;
    double* v;           // [C] centroids
    float* v32;          // [C] the same in FP32 (read by the membership kernel)
};

// Partial sums of one Algorithm 2 reduction over n inputs: n / (2 * 128), rounded up.
int64_t paper_parts(int64_t n);

// Per cluster: Eq.3 terms, the two reductions, the one-thread final sum.
hipError_t paper_centroids(const PaperBuffers& b, int C, float m, hipStream_t s);

// Per cluster: Eq.4 for every pixel into U.
hipError_t paper_memberships(const PaperBuffers& b, int C, float m, hipStream_t s);

}  // namespace fcm
