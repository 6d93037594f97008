// Random-membership start (Sec. 2.1, Algorithm 1 as printed): U^0 is drawn at
// random, so the first two passes of a solve differ from the centroid-first
// passes of the fused kernels:
//   pass 0: u^0_ij = r_ij / sum_k r_ik, a = (u^0)^m, Eq.3 sums -> v^1
//           (no centroids yet: v^0, J^0 and delta^0 are recorded as NaN);
//   pass 1: U^1 = Eq.4 at v^1, delta^1 = max |U^1 - U^0| with U^0 drawn again,
//           Eq.1 and Eq.3 sums -> J^1, v^2.
// From pass 2 on every driver continues unchanged (it recomputes U^(p-1) from
// v^(p-1), which for p = 2 is U^1).  U^0 is never stored: r_ij is draw
// number i C + j of the SplitMix64 stream `seed` (Steele, Lea and Flood,
// OOPSLA 2014: state seed + (k + 1) 0x9E3779B97F4A7C15, then the output mix),
// reduced to its top 24 bits, r = (bits + 1) 2^-24 in (0, 1], exact in FP32.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fcm.h"
#include "fcm_device.h"
#include "fcm_internal.h"
#include "fcm_random.h"

namespace fcm {

namespace {

__device__ __forceinline__ float draw24(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (float)((uint32_t)(z >> 40) + 1u) * 0x1p-24f;
}

// U^0 of voxel i (Eq.2: the row sums to 1)
template <int C>
__device__ __forceinline__ void random_row(uint64_t seed, int64_t i, float (&u)[C]) {
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < C; ++j) {
        u[j] = draw24(seed, (uint64_t)i * C + j);
        s += u[j];
    }
    const float r = 1.0f / s;
#pragma unroll
    for (int j = 0; j < C; ++j) u[j] *= r;
}

template <int C, int PHASE>
__device__ __forceinline__ void random_voxel(float x, int64_t i, uint64_t seed, const float (&v1)[C],
                                             const Consts& kc, Group<C>& g, float& dmax) {
    float u0[C], a[C], Jv = 0.f;
    random_row<C>(seed, i, u0);
    if constexpr (PHASE == 0) {
#pragma unroll
        for (int j = 0; j < C; ++j)
            a[j] = kc.mexp == 2.0f ? u0[j] * u0[j] : __builtin_amdgcn_exp2f(kc.mexp * __builtin_amdgcn_logf(u0[j]));
    } else {
        float u[C];
        memb<C, kNormLog, true>(x, v1, kc, u, a, Jv);
#pragma unroll
        for (int j = 0; j < C; ++j) dmax = fmaxf(dmax, fabsf(u[j] - u0[j]));
    }
#pragma unroll
    for (int j = 0; j < C; ++j) {
        g.n[j] = fmaf(a[j], x, g.n[j]);
        g.d[j] += a[j];
    }
    g.j += Jv;
}

template <int C, int PHASE>
__global__ __launch_bounds__(kBlock) void fcm_random_pass_kernel(PassArgs a, uint64_t seed) {
    DevState* st = a.st;
    if (st->done || st->pass != PHASE) return;
    const int tid = threadIdx.x;
    float v1[C];
#pragma unroll
    for (int k = 0; k < C; ++k) v1[k] = st->v32[1][k];
    const Consts kc{a.alpha, a.mexp};
    Acc<C> acc;
    acc.zero();
    const uint4* body = reinterpret_cast<const uint4*>(a.x + a.head);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + tid; c < a.nbody; c += stride) {
        const uint4 w = body[c];
        const uint32_t words[4] = {w.x, w.y, w.z, w.w};
        const int64_t i0 = a.head + 16 * c;
        Group<C> g;
        g.zero();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
            for (int b = 0; b < 4; ++b)
                random_voxel<C, PHASE>((float)((words[q] >> (8 * b)) & 0xFFu), i0 + 4 * q + b, seed, v1, kc, g,
                                       acc.dmax);
        }
        fold_group<C>(acc, g);
    }
    // unaligned head and tail (< 16 voxels each) go to block 0
    if (blockIdx.x == 0) {
        const int64_t tail0 = a.head + 16 * a.nbody;
        const int64_t nr = a.head + (a.n - tail0);
        if (tid < nr) {
            const int64_t i = tid < a.head ? (int64_t)tid : tail0 + (tid - a.head);
            Group<C> g;
            g.zero();
            random_voxel<C, PHASE>((float)a.x[i], i, seed, v1, kc, g, acc.dmax);
            fold_group<C>(acc, g);
        }
    }
    const int G = gridDim.x;
    const PlainRows rows{a.partials, G};
    write_partial_row<C>(acc, rows);
    if (!arrive_last(&st->ticket)) return;
    __shared__ Reduced<C> s_r;
    reduce_rows<C>(rows, G, a.kahan_only, s_r);
    if (tid == 0) {
        double vcur[C];
        Step<C> s;
        if constexpr (PHASE == 0) {
#pragma unroll
            for (int k = 0; k < C; ++k) {
                vcur[k] = __builtin_nan("");
                a.hist_v[k] = vcur[k];
            }
            decide<C>(s_r, 0, vcur, a.eps, a.max_iter, s);
            // no centroids before the first update: no objective, no change
            s.J = __builtin_nan("");
        } else {
#pragma unroll
            for (int k = 0; k < C; ++k) vcur[k] = a.hist_v[C + k];
            decide<C>(s_r, 1, vcur, a.eps, a.max_iter, s);
        }
        commit<C>(a, PHASE, vcur, s);
        st->ticket = 0;
    }
}

template <int C>
hipError_t launch_c(const PassArgs& a, int phase, uint64_t seed, int grid, hipStream_t s) {
    if (phase == 0)
        hipLaunchKernelGGL((fcm_random_pass_kernel<C, 0>), dim3(grid), dim3(kBlock), 0, s, a, seed);
    else
        hipLaunchKernelGGL((fcm_random_pass_kernel<C, 1>), dim3(grid), dim3(kBlock), 0, s, a, seed);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_random_pass(const PassArgs& a, int C, int phase, uint64_t seed, int grid, hipStream_t s) {
    if ((phase != 0 && phase != 1) || grid < 1 || grid > kMaxGrid) return hipErrorInvalidValue;
    switch (C) {
        case 2: return launch_c<2>(a, phase, seed, grid, s);
        case 3: return launch_c<3>(a, phase, seed, grid, s);
        case 4: return launch_c<4>(a, phase, seed, grid, s);
        case 5: return launch_c<5>(a, phase, seed, grid, s);
        case 6: return launch_c<6>(a, phase, seed, grid, s);
        case 7: return launch_c<7>(a, phase, seed, grid, s);
        case 8: return launch_c<8>(a, phase, seed, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fcm
