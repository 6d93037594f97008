// Batched solver: many instances (slices and volumes of uneven size, each
// with its own C, m, eps and max_iter) converge in one cooperative launch.
//
// The input is a concatenation of instances; the host cuts every instance
// into tiles of 16-voxel chunks.  The launch runs lock-step sweeps; sweep s
// runs pass s of every unfinished instance:
//   tiles   every block takes tiles t = block, block + G, ...; for each it
//           reads the instance's decision of sweep s - 1 (skipping finished
//           instances), runs the fused pass over the tile's voxels and writes
//           the tile's partial row;
//   owners  block i mod G owns instance i: it reduces the instance's tile rows
//           in tile order (FP64, or compensated FP32), applies Eq.3 and the
//           stopping rule of Algorithm 1, records the history and publishes
//           the decision (centroids of the next pass, done flag).
// Tile work of sweep s needs only decisions of sweep s - 1, and owner work of
// sweep s needs only tile rows of sweep s, which every block writes before it
// starts owner work, so no wait can be circular.  Values travel as tagged
// 64-bit words (see fcm_device.h); every wait is bounded by a wall-clock limit
// and an abort word.  A finished instance's tiles are skipped from then on;
// the launch ends when no instance is left.

#include "fcm_device.h"

namespace fcm {

namespace {

// round counters compare as signed differences, so they may wrap
__device__ __forceinline__ bool reached(uint32_t v, uint32_t target) { return (int32_t)(v - target) >= 0; }

// Wait until the K words at src carry `round` (same scheme as poll_tagged:
// a few whole-group polls, then the last word with back-off).
template <int K>
__device__ __forceinline__ bool batch_poll(const uint64_t* src, uint32_t round, uint32_t (&out)[K], BatchSync* sy,
                                           uint64_t t0, uint64_t limit) {
    int spins = 0;
    while (true) {
        bool all = true;
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const uint64_t w = __hip_atomic_load(src + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            all = all && (uint32_t)(w >> 32) == round;
            out[r] = (uint32_t)w;
        }
        if (all) return true;
        if (poll_expired(sy, t0, limit, spins)) return false;
        if (spins < kFastPolls) continue;
        while (true) {
            const uint64_t w = __hip_atomic_load(src + K - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((uint32_t)(w >> 32) == round) break;
            if (poll_expired(sy, t0, limit, spins)) return false;
        }
    }
}

// Tile rows: tile b's row at W + b * kBatchRowWords, K = 2C + 2 tagged words
// (folded sums, then the max change).  Writers use `self` (the global tile).
template <int K>
struct BatchRows {
    uint64_t* W;
    uint32_t round;
    BatchSync* sy;
    uint64_t t0, limit;
    int64_t self;
    __device__ __forceinline__ void put_pair(int q, float s, float c) const {
        store_tagged(W + self * kBatchRowWords + q, round, __builtin_bit_cast(uint32_t, s - c));
    }
    __device__ __forceinline__ void put_max(int q, float m) const {
        store_tagged(W + self * kBatchRowWords + q, round, __builtin_bit_cast(uint32_t, m));
    }
    template <int R>
    __device__ __forceinline__ bool get(int b, float (&v)[R]) const {
        static_assert(R == 2 * (K - 1) + 1, "row format");
        uint32_t raw[K];
        if (!batch_poll<K>(W + (int64_t)b * kBatchRowWords, round, raw, sy, t0, limit)) return false;
#pragma unroll
        for (int q = 0; q < K - 1; ++q) {
            v[2 * q] = __builtin_bit_cast(float, raw[q]);
            v[2 * q + 1] = 0.f;
        }
        v[R - 1] = __builtin_bit_cast(float, raw[K - 1]);
        return true;
    }
};

// Decision of instance i for the round `round`, read by one thread.  Returns
// 1 when the instance is running (centroids in vn/vo, pass in p), 0 when it
// has finished, -1 when the wait was abandoned.  A finished flag counts only
// if it was written in this solve (tag >= base, the solve's first round).
__device__ __forceinline__ int read_decision(const uint64_t* dec, uint32_t round, uint32_t base, BatchSync* sy,
                                             uint64_t limit, float* vn, float* vo, int& p) {
    const uint64_t t0 = wall_clock64();
    int spins = 0;
    uint32_t raw[kBatchDecWords];
    const uint64_t* ctl = dec + 2 * kMaxC;
    while (true) {
        // a few whole-group polls (one round trip each), then the control
        // word (written last) with back-off
        bool all = true;
        uint32_t ctl_tag = 0;
#pragma unroll
        for (int r = 0; r < kBatchDecWords; ++r) {
            const uint64_t w = __hip_atomic_load(dec + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            all = all && (uint32_t)(w >> 32) == round;
            raw[r] = (uint32_t)w;
            ctl_tag = (uint32_t)(w >> 32);  // the last word is the control word
        }
        if ((raw[kBatchDecWords - 1] & 1u) && reached(ctl_tag, base) && reached(round, ctl_tag)) return 0;
        if (all) break;
        if (poll_expired(sy, t0, limit, spins)) return -1;
        if (spins < kFastPolls) continue;
        while (true) {
            const uint64_t w = __hip_atomic_load(ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t tag = (uint32_t)(w >> 32);
            if (((uint32_t)w & 1u) && reached(tag, base) && reached(round, tag)) return 0;  // finished earlier
            if (tag == round) break;
            if (poll_expired(sy, t0, limit, spins)) return -1;
        }
    }
    for (int k = 0; k < kMaxC; ++k) {
        vn[k] = __builtin_bit_cast(float, raw[k]);
        vo[k] = __builtin_bit_cast(float, raw[kMaxC + k]);
    }
    p = (int)(raw[2 * kMaxC] >> 1);
    return (raw[2 * kMaxC] & 1u) ? 0 : 1;
}

__device__ __forceinline__ void write_decision(uint64_t* dec, uint32_t round, const float* vn, const float* vo,
                                               int C, int p, int done) {
    for (int k = 0; k < kMaxC; ++k) {
        store_tagged(dec + k, round, __builtin_bit_cast(uint32_t, k < C ? vn[k] : 0.f));
        store_tagged(dec + kMaxC + k, round, __builtin_bit_cast(uint32_t, k < C ? vo[k] : 0.f));
    }
    store_tagged(dec + 2 * kMaxC, round, ((uint32_t)p << 1) | (uint32_t)(done != 0));
}

// Fused pass over one tile's voxels (thread-strided chunks, plus the
// instance's ragged voxels on its first tile).
template <int C, int FORM, bool OLD>
__device__ __forceinline__ void tile_body(const uint8_t* xi, const BatchInst& in, const BatchTile& tl,
                                          const float (&vn)[C], const float (&vo)[C], const Consts& kc, Acc<C>& acc) {
    const int tid = threadIdx.x;
    const uint4* body = reinterpret_cast<const uint4*>(xi + in.head);
    for (int64_t c = tl.c0 + tid; c < tl.c1; c += kBlock) chunk16<C, FORM, OLD>(body[c], vn, vo, kc, acc);
    if (tl.ragged) {
        const int64_t tail0 = in.head + 16 * in.nbody;
        const int64_t nr = in.head + (in.n - tail0);
        if (tid < nr) {
            const int64_t i = tid < in.head ? (int64_t)tid : tail0 + (tid - in.head);
            Group<C> g;
            g.zero();
            voxel<C, FORM, OLD>((float)xi[i], vn, vo, kc, g, acc.dmax);
            fold_group<C>(acc, g);
        }
    }
}

template <int C>
__device__ void tile_pass(const BatchArgs& a, int64_t t, const BatchInst& in, const BatchTile& tl, int p,
                          const float* svn, const float* svo, uint32_t round) {
    float vn[C], vo[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
        vn[k] = svn[k];
        vo[k] = svo[k];
    }
    const uint8_t* xi = a.x + in.base;
    const Consts kc{in.alpha, in.mexp};
    Acc<C> acc;
    acc.zero();
    const bool fast = separated<C>(vn) && (p == 0 || separated<C>(vo));
    if (fast && in.mclass == kM2) {
        if (p == 0)
            tile_body<C, kProdM2, false>(xi, in, tl, vn, vo, kc, acc);
        else
            tile_body<C, kProdM2, true>(xi, in, tl, vn, vo, kc, acc);
    } else if (fast) {
        if (p == 0)
            tile_body<C, kProdPow, false>(xi, in, tl, vn, vo, kc, acc);
        else
            tile_body<C, kProdPow, true>(xi, in, tl, vn, vo, kc, acc);
    } else {
        if (p == 0)
            tile_body<C, kNormLog, false>(xi, in, tl, vn, vo, kc, acc);
        else
            tile_body<C, kNormLog, true>(xi, in, tl, vn, vo, kc, acc);
    }
    const BatchRows<2 * C + 2> rows{a.rows, round, a.sync, 0, 0, t};
    write_partial_row<C>(acc, rows);
}

// Owner step of instance i for pass p: reduce its tile rows, decide, record,
// publish.  Returns false (all threads) if a wait was abandoned.
template <int C>
__device__ bool owner_step(const BatchArgs& a, int i, const BatchInst& in, int p, uint32_t round) {
    __shared__ Reduced<C> s_r;
    const BatchRows<2 * C + 2> rows{a.rows + (int64_t)in.tile0 * kBatchRowWords, round, a.sync,
                                    (uint64_t)wall_clock64(), a.spin_ticks, 0};
    if (!reduce_rows<C>(rows, in.ntiles, in.kahan_only, s_r)) return false;
    if (threadIdx.x == 0) {
        double* hv = a.hist + in.hist;
        double* hd = hv + (int64_t)(in.max_iter + 2) * C;
        double* hJ = hd + (in.max_iter + 2);
        double vcur[C];
#pragma unroll
        for (int k = 0; k < C; ++k) vcur[k] = hv[(int64_t)p * C + k];
        Step<C> s;
        decide<C>(s_r, p, vcur, in.eps, in.max_iter, s);
        BatchRec* rec = a.recs + i;
        hJ[p] = s.J;
        hd[p] = s.delta;
        float vn[C], vo[C];
#pragma unroll
        for (int k = 0; k < C; ++k) {
            rec->vres[k] = vcur[k];
            vo[k] = (float)vcur[k];
            vn[k] = s.done ? vo[k] : (float)s.vnext[k];
            if (!s.done) hv[(int64_t)(p + 1) * C + k] = s.vnext[k];
        }
        rec->iters = p;
        rec->J = s.J;
        rec->delta = s.delta;
        rec->passes = p + 1;
        rec->status = s.status;
        rec->done = s.done;
        if (!s.done) rec->pass = p + 1;
        write_decision(a.dec + (int64_t)i * kBatchDecWords, round, vn, vo, C, s.done ? p : p + 1, s.done);
        if (s.done) __hip_atomic_fetch_sub(&a.sync->active, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return true;
}

__device__ __forceinline__ void batch_publish_round(BatchSync* sy, uint32_t round) {
    __hip_atomic_fetch_max(&sy->gen_max, round, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

__global__ __launch_bounds__(kBlock) void fcm_batch_kernel(BatchArgs a) {
    const int G = gridDim.x;
    const int tid = threadIdx.x;
    BatchSync* sy = a.sync;
    __shared__ float s_vn[kMaxC], s_vo[kMaxC];
    __shared__ int s_state, s_p;
    uint32_t round = a.round0;

    if (a.do_init) {
        ++round;
        for (int64_t t = blockIdx.x; t < a.ntiles; t += G) {
            const BatchTile tl = a.tiles[t];
            const BatchInst& in = a.inst[tl.inst];
            const uint8_t* xi = a.x + in.base;
            uint32_t lo = 255u, hi = 0u;
            const uint4* body = reinterpret_cast<const uint4*>(xi + in.head);
            for (int64_t c = tl.c0 + tid; c < tl.c1; c += kBlock) {
                const uint4 w = body[c];
                const uint32_t words[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const uint32_t v = (words[q] >> (8 * b)) & 0xFFu;
                        lo = min(lo, v);
                        hi = max(hi, v);
                    }
                }
            }
            if (tl.ragged) {
                const int64_t tail0 = in.head + 16 * in.nbody;
                const int64_t nr = in.head + (in.n - tail0);
                if (tid < nr) {
                    const int64_t i = tid < in.head ? (int64_t)tid : tail0 + (tid - in.head);
                    lo = min(lo, (uint32_t)xi[i]);
                    hi = max(hi, (uint32_t)xi[i]);
                }
            }
            block_minmax(lo, hi);
            if (tid == 0) {
                store_tagged(a.mm + 2 * t, round, lo);
                store_tagged(a.mm + 2 * t + 1, round, hi);
            }
            __syncthreads();
        }
        for (int i = blockIdx.x; i < a.I; i += G) {
            const BatchInst& in = a.inst[i];
            const uint64_t t0 = wall_clock64();
            auto get = [&](int b, uint32_t& l, uint32_t& h) {
                uint32_t raw[2];
                if (!batch_poll<2>(a.mm + 2 * ((int64_t)in.tile0 + b), round, raw, sy, t0, a.spin_ticks)) return false;
                l = raw[0];
                h = raw[1];
                return true;
            };
            uint32_t lo, hi;
            if (!reduce_minmax(get, in.ntiles, lo, hi)) return;
            if (tid == 0) {
                double* hv = a.hist + in.hist;
                float v[kMaxC];
                double v64[kMaxC];
                start_centroids(in.C, lo, hi, in.given, in.v0, in.dv0, v64);
                for (int k = 0; k < kMaxC; ++k) {
                    v[k] = 0.f;
                    if (k < in.C) {
                        hv[k] = v64[k];
                        v[k] = (float)v64[k];
                    }
                }
                BatchRec* rec = a.recs + i;
                rec->pass = 0;
                rec->done = 0;
                rec->iters = -1;
                rec->status = FCM_RUNNING;
                rec->passes = 0;
                rec->lo = (int32_t)lo;
                rec->hi = (int32_t)hi;
                rec->delta = __builtin_nan("");
                rec->J = __builtin_nan("");
                for (int k = 0; k < kMaxC; ++k) rec->vres[k] = (double)v[k];
                write_decision(a.dec + (int64_t)i * kBatchDecWords, round, v, v, in.C, 0, 0);
            }
            __syncthreads();
        }
    }

    for (int sweep = 0; sweep < a.max_sweeps; ++sweep) {
        if (__hip_atomic_load(&sy->active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) break;
        const uint32_t rd = round, rw = round + 1;
        for (int64_t t = blockIdx.x; t < a.ntiles; t += G) {
            const BatchTile tl = a.tiles[t];
            const BatchInst& in = a.inst[tl.inst];
            if (tid == 0) {
                float vn[kMaxC], vo[kMaxC];
                int p = 0;
                s_state = read_decision(a.dec + (int64_t)tl.inst * kBatchDecWords, rd, a.round0 + 1u, sy, a.spin_ticks,
                                        vn, vo, p);
                for (int k = 0; k < kMaxC; ++k) {
                    s_vn[k] = vn[k];
                    s_vo[k] = vo[k];
                }
                s_p = p;
            }
            __syncthreads();
            const int state = s_state;
            if (state < 0) return;
            if (state > 0) {
                switch (in.C) {
                    case 2: tile_pass<2>(a, t, in, tl, s_p, s_vn, s_vo, rw); break;
                    case 3: tile_pass<3>(a, t, in, tl, s_p, s_vn, s_vo, rw); break;
                    case 4: tile_pass<4>(a, t, in, tl, s_p, s_vn, s_vo, rw); break;
                    case 5: tile_pass<5>(a, t, in, tl, s_p, s_vn, s_vo, rw); break;
                    case 6: tile_pass<6>(a, t, in, tl, s_p, s_vn, s_vo, rw); break;
                    case 7: tile_pass<7>(a, t, in, tl, s_p, s_vn, s_vo, rw); break;
                    default: tile_pass<8>(a, t, in, tl, s_p, s_vn, s_vo, rw); break;
                }
            }
            __syncthreads();
        }
        for (int i = blockIdx.x; i < a.I; i += G) {
            const BatchInst& in = a.inst[i];
            if (tid == 0) {
                s_state = a.recs[i].done;
                s_p = a.recs[i].pass;
            }
            __syncthreads();
            if (!s_state) {
                bool ok;
                switch (in.C) {
                    case 2: ok = owner_step<2>(a, i, in, s_p, rw); break;
                    case 3: ok = owner_step<3>(a, i, in, s_p, rw); break;
                    case 4: ok = owner_step<4>(a, i, in, s_p, rw); break;
                    case 5: ok = owner_step<5>(a, i, in, s_p, rw); break;
                    case 6: ok = owner_step<6>(a, i, in, s_p, rw); break;
                    case 7: ok = owner_step<7>(a, i, in, s_p, rw); break;
                    default: ok = owner_step<8>(a, i, in, s_p, rw); break;
                }
                if (!ok) return;
            }
            __syncthreads();
        }
        round = rw;
    }
    if (tid == 0) batch_publish_round(sy, round);
}

// Labels of every instance: per tile, the 256-entry nearest-centroid table of
// its instance (FP64, ties to the lowest index), then the gather.
__global__ __launch_bounds__(kBlock) void fcm_batch_labels_kernel(BatchLabelArgs a) {
    __shared__ uint8_t lut[256];
    const int tid = threadIdx.x;
    for (int64_t t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        const BatchTile tl = a.tiles[t];
        const BatchInst& in = a.inst[tl.inst];
        const BatchRec& rec = a.recs[tl.inst];
        const int T = rec.iters < 0 ? 0 : rec.iters;
        const double* v = a.hist + in.hist + (int64_t)T * in.C;
        for (int g = tid; g < 256; g += kBlock) {
            int best = 0;
            double bd = fabs((double)g - v[0]);
            for (int k = 1; k < in.C; ++k) {
                const double d = fabs((double)g - v[k]);
                if (d < bd) {
                    bd = d;
                    best = k;
                }
            }
            lut[g] = (uint8_t)best;
        }
        __syncthreads();
        const uint8_t* xi = a.x + in.base;
        uint8_t* li = a.labels + in.base;
        if (a.bytewise) {
            // voxels of the tile's chunks, one byte at a time (output alignment differs)
            for (int64_t i = in.head + 16 * tl.c0 + tid; i < in.head + 16 * tl.c1; i += kBlock) li[i] = lut[xi[i]];
        } else {
            const uint4* src = reinterpret_cast<const uint4*>(xi + in.head);
            uint4* dst = reinterpret_cast<uint4*>(li + in.head);
            for (int64_t c = tl.c0 + tid; c < tl.c1; c += kBlock) {
                const uint4 w = src[c];
                const uint32_t words[4] = {w.x, w.y, w.z, w.w};
                uint32_t o[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t x = words[q];
                    o[q] = (uint32_t)lut[x & 0xFFu] | ((uint32_t)lut[(x >> 8) & 0xFFu] << 8) |
                           ((uint32_t)lut[(x >> 16) & 0xFFu] << 16) | ((uint32_t)lut[x >> 24] << 24);
                }
                dst[c] = make_uint4(o[0], o[1], o[2], o[3]);
            }
        }
        if (tl.ragged) {
            const int64_t tail0 = in.head + 16 * in.nbody;
            const int64_t nr = in.head + (in.n - tail0);
            if (tid < nr) {
                const int64_t i = tid < in.head ? (int64_t)tid : tail0 + (tid - in.head);
                li[i] = lut[xi[i]];
            }
        }
        __syncthreads();
    }
}

// Network training targets: instance i's v^T sorted ascending (insertion
// sort of at most kMaxC values), each divided by 255 in FP64 and rounded once
// to FP32.  One thread per instance.
__global__ __launch_bounds__(kBlock) void fcm_batch_targets_kernel(const BatchRec* recs, int32_t I, int32_t C,
                                                                    float* out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= I) return;
    double v[kMaxC];
    for (int k = 0; k < C; ++k) {
        const double x = recs[i].vres[k];
        int j = k;
        while (j > 0 && v[j - 1] > x) {
            v[j] = v[j - 1];
            --j;
        }
        v[j] = x;
    }
    for (int k = 0; k < C; ++k) out[i * C + k] = (float)(v[k] / 255.0);
}

hipError_t launch_batch_targets(const BatchRec* recs, int32_t I, int32_t C, float* out, hipStream_t s) {
    hipLaunchKernelGGL(fcm_batch_targets_kernel, dim3((unsigned)((I + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       recs, I, C, out);
    return hipGetLastError();
}

hipError_t batch_max_grid(int ncu, int* max_grid) {
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void*>(fcm_batch_kernel), kBlock, 0);
    if (e != hipSuccess) return e;
    *max_grid = per_cu * ncu;
    return hipSuccess;
}

hipError_t launch_batch(const BatchArgs& a, int grid, hipStream_t s) {
    BatchArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(fcm_batch_kernel), dim3(grid), dim3(kBlock), args,
                                      0, s);
}

hipError_t launch_batch_labels(const BatchLabelArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(fcm_batch_labels_kernel, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace fcm
