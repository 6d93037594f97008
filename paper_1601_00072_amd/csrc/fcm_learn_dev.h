// Device code of the learned start shared by the standalone kernels
// (fcm_learn.hip) and the persistent solve (fcm_device.h), so that both
// produce bit-identical start centroids from the same histogram.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

#include "fcm_internal.h"

namespace fcm {

// round to nearest even; NaN stays NaN
__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

template <bool BF16>
__device__ __forceinline__ float act(float v) {
    if constexpr (BF16)
        return from_bf16(to_bf16(v));
    else
        return v;
}

// BF16 inference copy of the parameters, output-major so that a thread's
// weights are contiguous: W1t [128][256], b1 [128], W2t [64][128], b2 [64],
// W3t [C][64], b3 [C] (W1t[o][i] = W1[i][o]); every row starts on a 16-byte
// boundary.
struct InferLayout {
    static constexpr int64_t W1 = 0, b1 = W1 + 128 * 256, W2 = b1 + 128, b2 = W2 + 64 * 128, W3 = b2 + 64;
    __host__ __device__ static constexpr int64_t b3(int C) { return W3 + 64 * (int64_t)C; }
};

// z + sum of a[i] w[i] over the 8 * N BF16 weights held in q (ascending i)
template <int N>
__device__ __forceinline__ float dot_bf16_regs(float z, const float* a, const uint4 (&q)[N]) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const uint32_t u[4] = {q[k].x, q[k].y, q[k].z, q[k].w};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            z = fmaf(a[8 * k + 2 * h], __builtin_bit_cast(float, u[h] << 16), z);
            z = fmaf(a[8 * k + 2 * h + 1], __builtin_bit_cast(float, u[h] & 0xFFFF0000u), z);
        }
    }
    return z;
}

template <int N>
__device__ __forceinline__ void load_bf16(const uint16_t* w, uint4 (&q)[N]) {
    const uint4* w4 = reinterpret_cast<const uint4*>(w);
#pragma unroll
    for (int k = 0; k < N; ++k) q[k] = w4[k];
}

// dot product z + sum_i a[i] w[i] over n BF16 weights (n a multiple of 64,
// w 16-byte aligned), in ascending i, 64 weights (8 loads) in flight
__device__ __forceinline__ float dot_bf16(float z, const float* a, const uint16_t* w, int n) {
    for (int c = 0; c < n; c += 64) {
        uint4 q[8];
        load_bf16<8>(w + c, q);
        z = dot_bf16_regs<8>(z, a + c, q);
    }
    return z;
}

// The network on one histogram x[256] (normalised), by the whole block
// (blockDim >= 256; every thread must call it: it synchronises).  The three
// layers sum in a fixed order (ascending input index) with FP32
// accumulation.  BF16: w is the inference copy (InferLayout), and the
// activations (the input included) are rounded to BF16 before every product.
// FP32: w is the flat parameter vector W1 [256][128], b1, W2 [128][64], b2,
// W3 [64][C], b3.  s_a0/s_a1/s_a2/s_tmp: shared scratch of 256/128/64/256 floats; y[C]
// (shared or global) receives the output, written by threads 0..C-1.
template <bool BF16>
__device__ __forceinline__ void mlp_block_forward(const void* w, const float* x, int C, float* s_a0, float* s_a1,
                                                  float* s_a2, float* s_tmp, float* y) {
    const int t = threadIdx.x;
    for (int i = t; i < 256; i += blockDim.x) s_a0[i] = act<BF16>(x[i]);
    __syncthreads();
    if constexpr (BF16) {
        using L = InferLayout;
        const uint16_t* wb = static_cast<const uint16_t*>(w);
        // layer 1 on 256 threads: output o = t % 128 sums inputs 0..127
        // (threads < 128, starting from the bias) and 128..255 (threads >= 128);
        // then (bias + first half) + second half
        // layer 2 and 3 weights are fetched before layer 1 runs (their
        // latency hides behind it)
        uint4 w2[16], w3[8];
        if (t < 64) load_bf16<16>(wb + L::W2 + t * 128, w2);
        if (t < C) load_bf16<8>(wb + L::W3 + t * 64, w3);
        if (t < 256) {
            const int o = t & 127, half = t >> 7;
            const float z0 = half ? 0.f : from_bf16(wb[L::b1 + o]);
            s_tmp[t] = dot_bf16(z0, s_a0 + 128 * half, wb + L::W1 + o * 256 + 128 * half, 128);
        }
        __syncthreads();
        if (t < 128) s_a1[t] = act<true>(fmaxf(s_tmp[t] + s_tmp[t + 128], 0.f));
        __syncthreads();
        if (t < 64) s_a2[t] = act<true>(fmaxf(dot_bf16_regs<16>(from_bf16(wb[L::b2 + t]), s_a1, w2), 0.f));
        __syncthreads();
        if (t < C) y[t] = dot_bf16_regs<8>(from_bf16(wb[L::b3(C) + t]), s_a2, w3);
    } else {
        const float* wf = static_cast<const float*>(w);
        constexpr int64_t oW1 = 0, ob1 = oW1 + 256 * 128, oW2 = ob1 + 128, ob2 = oW2 + 128 * 64, oW3 = ob2 + 64;
        const int64_t ob3 = oW3 + 64 * (int64_t)C;
        if (t < 128) {
            float z = wf[ob1 + t];
            for (int i = 0; i < 256; ++i) z = fmaf(s_a0[i], wf[oW1 + i * 128 + t], z);
            s_a1[t] = fmaxf(z, 0.f);
        }
        __syncthreads();
        if (t < 64) {
            float z = wf[ob2 + t];
            for (int i = 0; i < 128; ++i) z = fmaf(s_a1[i], wf[oW2 + i * 64 + t], z);
            s_a2[t] = fmaxf(z, 0.f);
        }
        __syncthreads();
        if (t < C) {
            float z = wf[ob3 + t];
            for (int i = 0; i < 64; ++i) z = fmaf(s_a2[i], wf[oW3 + i * C + t], z);
            y[t] = z;
        }
    }
}

// Network output -> start centroids (one thread): v = 255 y, sorted
// ascending, clamped to the data range [lo, hi] (the lowest and highest
// grey level present), consecutive gaps of at least 1; C doubles (FP32
// values), or NaN when no valid set exists (non-finite output, or
// hi - lo < C - 1), which the solver reads as "use the evenly spaced start".
__device__ __forceinline__ void warm_post_one(const float* y, int lo, int hi, int C, double* v0) {
    float v[kMaxC];
    bool ok = hi - lo >= C - 1;
    for (int k = 0; k < C; ++k) {
        v[k] = 255.f * y[k];
        if (!isfinite(v[k])) ok = false;
    }
    for (int k = 1; k < C; ++k) {  // insertion sort
        const float key = v[k];
        int j = k - 1;
        while (j >= 0 && v[j] > key) {
            v[j + 1] = v[j];
            --j;
        }
        v[j + 1] = key;
    }
    for (int k = 0; k < C; ++k) v[k] = fminf(fmaxf(v[k], (float)lo), (float)hi);
    for (int k = 1; k < C; ++k) v[k] = fmaxf(v[k], v[k - 1] + 1.f);
    if (v[C - 1] > (float)hi) {  // push back from the top
        v[C - 1] = (float)hi;
        for (int k = C - 2; k >= 0; --k) v[k] = fminf(v[k], v[k + 1] - 1.f);
        if (v[0] < (float)lo) ok = false;
    }
    for (int k = 0; k < C; ++k) v0[k] = ok ? (double)v[k] : __builtin_nan("");
}

// Normalised histogram value of a level: count / n in FP64, stored as FP32.
__device__ __forceinline__ float hist_norm(uint32_t count, int64_t n) {
    return (float)((double)count / (double)n);
}

}  // namespace fcm
