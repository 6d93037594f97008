// Segmentation quality (Sec. 5.2.2): confusion counts between a label image
// and a ground truth, and the Dice similarity coefficient of Eq.5 per class,
// DSC_k = 2 |PR_k and GT_k| / (|PR_k| + |GT_k|), where PR_k holds the voxels
// whose cluster is assigned to class k and GT_k the voxels of class k.
//
// The counting pass reads 2 bytes per voxel (HBM-bound): each thread takes
// 16-voxel chunks with one 16-byte load per image when the two images share
// their alignment (byte loads otherwise), counts in LDS, and each block adds
// its counts to the global 64-bit counters once.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fcm.h"
#include "fcm_host.h"
#include "fcm_internal.h"

namespace fcm {

namespace {

constexpr int kBins = 256;                    // n_pred * n_truth <= 16 * 16
constexpr int kTables = kBlock / 64;          // one table per wave
constexpr int64_t kPerBlockMax = 1LL << 31;   // voxels per block: LDS counters stay below 2^32
constexpr int kUnroll = 4;                    // 16-voxel chunks in flight per thread

__global__ __launch_bounds__(kBlock) void zero_counts_kernel(unsigned long long* c, int n) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) c[i] = 0ull;
}

// Counting tables.  Few class pairs (the usual case: C clusters against a
// handful of tissues): every thread owns a column of counters, bin-major
// [kSmallBins + 1][kBlock], so the 64 lanes of a wave touch 64 distinct
// words (no bank conflicts, no contended atomics) whatever the labels are.  More pairs:
// one shared table per wave, updated with LDS atomics.
constexpr int kSmallBins = 32;

template <bool SMALL>
struct Tables;

template <>
struct Tables<true> {
    uint32_t t[kSmallBins + 1][kBlock];
    __device__ __forceinline__ void clear(int tid) {
        for (int b = 0; b <= kSmallBins; ++b) t[b][tid] = 0u;
    }
    // LDS add without return: no read-after-write wait between voxels
    __device__ __forceinline__ void add(int tid, uint32_t bin) { atomicAdd(&t[bin][tid], 1u); }
    static constexpr uint32_t kOut = kSmallBins;
};

template <>
struct Tables<false> {
    uint32_t t[kTables][kBins + 1];
    __device__ __forceinline__ void clear(int tid) {
        for (int w = 0; w < kTables; ++w) {
            t[w][tid] = 0u;
            if (tid == 0) t[w][kBins] = 0u;
        }
    }
    __device__ __forceinline__ void add(int tid, uint32_t bin) { atomicAdd(&t[tid >> 6][bin], 1u); }
    static constexpr uint32_t kOut = kBins;
};

template <bool SMALL>
__device__ __forceinline__ void count_pair(Tables<SMALL>& tab, int tid, uint32_t p, uint32_t t, uint32_t np,
                                           uint32_t nt) {
    // labels are bytes and nt <= 16: the 24-bit multiply (full rate) is exact
    tab.add(tid, (p < np && t < nt) ? __umul24(p, nt) + t : Tables<SMALL>::kOut);
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <bool SMALL>
__global__ __launch_bounds__(kBlock) void confusion_kernel(const uint8_t* pred, const uint8_t* truth, int64_t n,
                                                           uint32_t np, uint32_t nt, int vector,
                                                           unsigned long long* counts) {
    __shared__ Tables<SMALL> tab;
    const int tid = threadIdx.x;
    tab.clear(tid);
    __syncthreads();
    // head (to 16-byte alignment of pred), 16-voxel body chunks, tail
    const int64_t lead = vector ? (int64_t)((16 - ((uintptr_t)pred & 15)) & 15) : 0;
    const int64_t head = n < lead ? n : lead;
    const int64_t nbody = vector ? (n - head) / 16 : 0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    if (vector) {
        const uint4* pb = reinterpret_cast<const uint4*>(pred + head);
        const uint4* tb = reinterpret_cast<const uint4*>(truth + head);
        // kUnroll chunks per thread and step, all loads issued before counting
        for (int64_t c0 = (int64_t)blockIdx.x * kBlock + tid; c0 < nbody; c0 += kUnroll * stride) {
            uint4 pw[kUnroll], tw[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int64_t c = c0 + u * stride;
                if (c < nbody) {
                    pw[u] = pb[c];
                    tw[u] = tb[c];
                }
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                if (c0 + u * stride >= nbody) break;
                const uint32_t pv[4] = {pw[u].x, pw[u].y, pw[u].z, pw[u].w};
                const uint32_t tv[4] = {tw[u].x, tw[u].y, tw[u].z, tw[u].w};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        count_pair(tab, tid, (pv[q] >> (8 * b)) & 0xFFu, (tv[q] >> (8 * b)) & 0xFFu, np, nt);
                }
            }
        }
    }
    // remaining voxels (all of them on the byte path), spread over the grid
    const int64_t tail0 = head + 16 * nbody;
    const int64_t rest = head + (n - tail0);
    for (int64_t r = (int64_t)blockIdx.x * kBlock + tid; r < rest; r += stride) {
        const int64_t i = r < head ? r : tail0 + (r - head);
        count_pair(tab, tid, pred[i], truth[i], np, nt);
    }
    __syncthreads();
    const int used = (int)(np * nt);
    if constexpr (SMALL) {
        // wave w folds bins w, w + 4, ...: four columns per lane, then the
        // wave; the totals go out as one atomic instruction per block (one
        // request per cache line of counters: the blocks' atomics on the same
        // few lines serialise, so their number is what costs)
        __shared__ uint32_t s_tot[kSmallBins + 1];
        const int lane = tid & 63, wid = tid >> 6;
        for (int b = wid; b <= used; b += kTables) {
            const int row = b == used ? kSmallBins : b;
            uint32_t v = tab.t[row][lane] + tab.t[row][lane + 64] + tab.t[row][lane + 128] + tab.t[row][lane + 192];
            v = wave_sum_u32(v);
            if (lane == 0) s_tot[b] = v;
        }
        __syncthreads();
        if (tid <= used && s_tot[tid]) atomicAdd(counts + tid, (unsigned long long)s_tot[tid]);
    } else {
        for (int b = tid; b <= kBins; b += kBlock) {
            if (b < used || b == kBins) {
                uint32_t v = 0u;
                for (int w = 0; w < kTables; ++w) v += tab.t[w][b];
                if (v) atomicAdd(counts + (b == kBins ? used : b), (unsigned long long)v);
            }
        }
    }
}

struct DiceArgs {
    const unsigned long long* counts;
    double* dsc;
    int np, nt;
    int class_of[16];
};

// one thread per class: Eq.5 from the exact integer counts, one rounding
__global__ void dice_kernel(DiceArgs a) {
    const int k = threadIdx.x;
    if (k >= a.nt) return;
    unsigned long long inter = 0ull, pr = 0ull, gt = 0ull;
    for (int j = 0; j < a.np; ++j) {
        const unsigned long long cjk = a.counts[j * a.nt + k];
        gt += cjk;
        if (a.class_of[j] == k) {
            inter += cjk;
            for (int t = 0; t < a.nt; ++t) pr += a.counts[j * a.nt + t];
        }
    }
    const unsigned long long den = pr + gt;
    a.dsc[k] = den ? (double)(2ull * inter) / (double)den : __builtin_nan("");
}

}  // namespace

}  // namespace fcm

extern "C" {

int fcm_confusion(const uint8_t* d_pred, const uint8_t* d_truth, int64_t n, int32_t n_pred, int32_t n_truth,
                  uint64_t* d_counts, void* stream) {
    using namespace fcm;
    if (!d_counts || n < 0 || (n > 0 && (!d_pred || !d_truth)) || n_pred < 1 || n_pred > 16 || n_truth < 1 ||
        n_truth > 16)
        return FCM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int slots = n_pred * n_truth + 1;
    auto* c = reinterpret_cast<unsigned long long*>(d_counts);
    hipLaunchKernelGGL(zero_counts_kernel, dim3((slots + kBlock - 1) / kBlock), dim3(kBlock), 0, s, c, slots);
    FCM_HIP(hipGetLastError());
    if (n == 0) return FCM_OK;
    const int vector = (((uintptr_t)d_pred ^ (uintptr_t)d_truth) & 15) == 0;
    // kUnroll 16-voxel chunks per thread and step, at most 1024 blocks, but
    // never more than 2^31 voxels per block
    const int64_t per_block = (int64_t)kBlock * 16 * kUnroll;
    int64_t grid = (n + per_block - 1) / per_block;
    if (grid > 1024) grid = 1024;
    const int64_t need = (n + kPerBlockMax - 1) / kPerBlockMax;
    if (grid < need) grid = need;
    if (grid > 0x7FFFFFFF) return FCM_EINVAL;
    if (n_pred * n_truth <= kSmallBins)
        hipLaunchKernelGGL(confusion_kernel<true>, dim3((unsigned)grid), dim3(kBlock), 0, s, d_pred, d_truth, n,
                           (uint32_t)n_pred, (uint32_t)n_truth, vector, c);
    else
        hipLaunchKernelGGL(confusion_kernel<false>, dim3((unsigned)grid), dim3(kBlock), 0, s, d_pred, d_truth, n,
                           (uint32_t)n_pred, (uint32_t)n_truth, vector, c);
    FCM_HIP(hipGetLastError());
    return FCM_OK;
}

int fcm_dice(const uint64_t* d_counts, int32_t n_pred, int32_t n_truth, const int32_t* class_of, double* d_dsc,
             void* stream) {
    using namespace fcm;
    if (!d_counts || !d_dsc || n_pred < 1 || n_pred > 16 || n_truth < 1 || n_truth > 16) return FCM_EINVAL;
    DiceArgs a{};
    a.counts = reinterpret_cast<const unsigned long long*>(d_counts);
    a.dsc = d_dsc;
    a.np = n_pred;
    a.nt = n_truth;
    for (int j = 0; j < n_pred; ++j) {
        const int k = class_of ? class_of[j] : (j < n_truth ? j : -1);
        if (k < -1 || k >= n_truth) return FCM_EINVAL;
        a.class_of[j] = k;
    }
    hipLaunchKernelGGL(dice_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, a);
    FCM_HIP(hipGetLastError());
    return FCM_OK;
}

}  // extern "C"
