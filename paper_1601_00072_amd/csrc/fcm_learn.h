// Internal launchers of the learned warm start (fcm_learn.hip); not part of the ABI.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

struct fcm_mlp;

namespace fcm {

// Output width C of a network, and its warm start: BF16 inference of `count`
// normalised histograms into d_y (count x C) and the post-processing into
// start centroids d_v0 (count x C doubles; a row of NaN where no valid start
// exists).  Enqueued on s; returns an FCM_* status.
int mlp_clusters(const fcm_mlp* net);
int mlp_warm(fcm_mlp* net, const float* d_hist, int count, float* d_y, double* d_v0, hipStream_t s);

// The network's BF16 parameters, brought up to date on stream s (for the
// persistent solve's in-kernel inference); *rc receives an FCM_* status.
const uint16_t* mlp_bf16_weights(fcm_mlp* net, hipStream_t s, int* rc);

// Histograms of `count` instances: counts is a workspace of
// count * histogram_copies(count) * 256 words; on completion copy 0 of each
// instance's counts holds its integer totals and hist[count][256] the
// normalised histogram.
int histogram_copies(int count);
hipError_t launch_histogram(const uint8_t* x, const int64_t* d_offsets, int count, int64_t max_n, uint32_t* counts,
                            float* hist, hipStream_t s);
// the same on counters that are already zero (no memset)
hipError_t launch_histogram_counts(const uint8_t* x, const int64_t* d_offsets, int count, int64_t max_n,
                                   uint32_t* counts, float* hist, hipStream_t s);
hipError_t launch_gemm(bool ta, bool tb, const float* A, const float* B, float* Cm, int M, int N, int K,
                       const float* bias, int relu, const float* mask, hipStream_t s);
hipError_t launch_colsum(const float* G, int M, int N, float* out, hipStream_t s);
hipError_t launch_mse(const float* Y, const float* T, int n, float scale, float* dY, float* loss_out, hipStream_t s);
hipError_t launch_adam(float* theta, const float* g, float* m, float* v, int64_t n, float lr, int step,
                       hipStream_t s);
hipError_t launch_gather(const float* X, const int32_t* idx, int rows, int cols, float* out, hipStream_t s);
// BF16 inference copy (output-major rows; see fcm_learn_dev.h) of the flat parameters
hipError_t launch_to_bf16(const float* theta, uint16_t* out, int C, hipStream_t s);
hipError_t launch_mlp_infer(const void* w, bool bf16, const float* X, int count, int C, float* Y, hipStream_t s);
hipError_t launch_warm_post(const float* Y, const float* hist, int count, int C, double* v0, hipStream_t s);

}  // namespace fcm
