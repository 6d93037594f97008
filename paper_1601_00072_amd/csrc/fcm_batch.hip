// Batched solver: many instances (slices and volumes of uneven size, each
// with its own C, m, eps and max_iter) converge in one persistent launch.
//
// The input is a concatenation of instances; the host cuts every instance
// into tiles of 16-voxel chunks (a coarse set, and a fine set for the later
// passes).  Each instance runs the same phases as a single solve -- phase 0
// finds its grey-level range and v^0, phase p + 1 is fused pass p -- at its
// own pace; no instance waits for another.  An instance's control word
// (fcm_internal.h) counts the tiles of its current phase handed out and
// finished:
//   claim   a free block takes a tile of the instance it worked on last if
//           that has tiles open, else of the first instance with open tiles
//           in its own rotation order (blocks start their rotations at
//           spread positions), with one atomic add on the control word; it
//           reads the phase's decision (tagged words) and runs the tile:
//           min/max for phase 0, the fused pass (Eq.4, Eq.3 sums, Eq.1 term,
//           change) otherwise, writing one tagged partial row;
//   arrive  a second atomic add counts the tile as finished; the block that
//           finishes the phase's last tile reduces the instance's rows in tile
//           order (FP64, or compensated FP32), applies Eq.3 and the stopping
//           rule of Algorithm 1, records the history, then opens the next
//           phase with its tile 0 already taken by itself: it goes on with
//           that tile at once, with the decision still in LDS, and publishes
//           the decision only for the other blocks that will take the
//           phase's other tiles.  A phase with a single tile therefore never
//           leaves the block: its row is reduced from LDS, with no arrival and
//           no global read, so a small instance is solved by one block at the
//           speed of its arithmetic.
// A block waits only for tagged words that a finished tile or phase has
// already written (bounded polls), never for work of another block in
// progress, so no grid-wide residency is needed; the rows are reduced in the
// same order whichever blocks ran the tiles, so results are reproducible run
// to run.  Every wait is bounded by a wall-clock limit and an abort word.
// Blocks leave when no instance is left, or once they outnumber the tiles of
// the unfinished instances.

#include "fcm_device.h"

namespace fcm {

namespace {

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

// The one row of a phase that has a single tile, kept in LDS by the block
// that runs it (same folded values as a tagged row).
template <int K>
struct LocalRows {
    float* W;
    __device__ __forceinline__ void put_pair(int q, float s, float c) const { W[q] = s - c; }
    __device__ __forceinline__ void put_max(int q, float m) const { W[q] = m; }
    template <int R>
    __device__ __forceinline__ bool get(int, float (&v)[R]) const {
        static_assert(R == 2 * (K - 1) + 1, "row format");
#pragma unroll
        for (int q = 0; q < K - 1; ++q) {
            v[2 * q] = W[q];
            v[2 * q + 1] = 0.f;
        }
        v[R - 1] = W[K - 1];
        return true;
    }
};

// The decision a block's tile is computed with (a copy in LDS): v^p and
// v^(p-1) in FP32, p, and v^p in FP64 for completing the pass.
struct Decision {
    float vn[kMaxC], vo[kMaxC];
    double v64[kMaxC];
    int p;
};

// The tile set of a phase: coarse for phase 0 and the early passes, fine
// (more, smaller tiles) from pass fine_from on, where few instances remain
// and each pass of the longest ones is on the critical path.  A function of
// the phase only, so every run adds an instance's partial sums in the same
// order.
__device__ __forceinline__ int tile_set(const BatchArgs& a, uint32_t phase) {
    return phase >= 1u && (int)phase - 1 >= a.fine_from ? 1 : 0;
}

__device__ __forceinline__ int phase_tiles(const BatchArgs& a, int i, uint32_t phase) {
    return a.ntiles[2 * i + tile_set(a, phase)];
}

// Decision of pass p for the other blocks (tagged words, fcm_internal.h),
// written by lanes 0 .. kMaxC of the calling block.
__device__ __forceinline__ void publish_decision(uint64_t* dec, uint32_t round, const float* vn, const float* vo,
                                                 const double* v64, int C, int p) {
    const int k = threadIdx.x;
    if (k < kMaxC) {
        const uint64_t bits = k < C ? __builtin_bit_cast(uint64_t, v64[k]) : 0ull;
        store_tagged(dec + k, round, __builtin_bit_cast(uint32_t, k < C ? vn[k] : 0.f));
        store_tagged(dec + kMaxC + k, round, __builtin_bit_cast(uint32_t, k < C ? vo[k] : 0.f));
        store_tagged(dec + kBatchDecF64 + 2 * k, round, (uint32_t)bits);
        store_tagged(dec + kBatchDecF64 + 2 * k + 1, round, (uint32_t)(bits >> 32));
    } else if (k == kMaxC) {
        store_tagged(dec + 2 * kMaxC, round, (uint32_t)p);
    }
}

// Fused pass over one tile's voxels (thread-strided chunks, the next chunk
// loaded while the current one is computed, plus the instance's ragged
// voxels on its first tile).
template <int C, int FORM, bool OLD, int BS>
__device__ __forceinline__ void tile_body(const uint8_t* xi, const BatchInst& in, const BatchTile& tl,
                                          const float (&vn)[C], const float (&vo)[C], const Consts& kc, Acc<C>& acc) {
    const int tid = threadIdx.x;
    const uint4* body = reinterpret_cast<const uint4*>(xi + in.head);
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    int64_t c = tl.c0 + tid;
    uint4 cur = c < tl.c1 ? body[c] : z;
    while (c < tl.c1) {
        const int64_t cn = c + BS;
        const uint4 nx = cn < tl.c1 ? body[cn] : z;
        chunk16<C, FORM, OLD>(cur, vn, vo, kc, acc);
        cur = nx;
        c = cn;
    }
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

// One tile of fused pass d.p; its partial row goes to the tagged row buffer,
// or to LDS (`lrow`) when the phase has a single tile.
template <int C, int BS>
__device__ __forceinline__ void tile_pass(const BatchArgs& a, int64_t t, const BatchInst& in, const BatchTile& tl,
                                          const Decision& d, uint32_t round, float* lrow) {
    float vn[C], vo[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
        vn[k] = d.vn[k];
        vo[k] = d.vo[k];
    }
    const int p = d.p;
    const uint8_t* xi = a.x + in.base;
    const Consts kc{in.alpha, in.mexp};
    Acc<C> acc;
    acc.zero();
    const bool fast = separated<C>(vn) && (p == 0 || separated<C>(vo));
    if (fast && in.mclass == kM2) {
        if (p == 0)
            tile_body<C, kProdM2, false, BS>(xi, in, tl, vn, vo, kc, acc);
        else
            tile_body<C, kProdM2, true, BS>(xi, in, tl, vn, vo, kc, acc);
    } else if (fast) {
        if (p == 0)
            tile_body<C, kProdPow, false, BS>(xi, in, tl, vn, vo, kc, acc);
        else
            tile_body<C, kProdPow, true, BS>(xi, in, tl, vn, vo, kc, acc);
    } else {
        if (p == 0)
            tile_body<C, kNormLog, false, BS>(xi, in, tl, vn, vo, kc, acc);
        else
            tile_body<C, kNormLog, true, BS>(xi, in, tl, vn, vo, kc, acc);
    }
    if (lrow) {
        write_partial_row<C, BS>(acc, LocalRows<2 * C + 2>{lrow});
    } else {
        const BatchRows<2 * C + 2> rows{a.rows, round, a.sync, 0, 0, t};
        write_partial_row<C, BS>(acc, rows);
    }
}

// Phase 0 of one tile: the grey-level range of its voxels as two tagged
// words (or in LDS, `lmm`, when the phase has a single tile).
template <int BS>
__device__ __forceinline__ void tile_range(const BatchArgs& a, int64_t t, const BatchInst& in, const BatchTile& tl,
                                           uint32_t round, uint32_t* lmm) {
    const int tid = threadIdx.x;
    const uint8_t* xi = a.x + in.base;
    uint32_t lo = 255u, hi = 0u;
    const uint4* body = reinterpret_cast<const uint4*>(xi + in.head);
    for (int64_t c = tl.c0 + tid; c < tl.c1; c += BS) {
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
    block_minmax<BS>(lo, hi);
    if (tid == 0) {
        if (lmm) {
            lmm[0] = lo;
            lmm[1] = hi;
        } else {
            store_tagged(a.rows + t * kBatchRowWords, round, lo);
            store_tagged(a.rows + t * kBatchRowWords + 1, round, hi);
        }
    }
}

// Results (history, record, commit times) are written by whichever block
// completes a phase, on any XCD, and the same record by several of them: the
// stores go with agent scope, so that no XCD's L2 keeps an older copy that a
// later write-back could put over a newer one.
__device__ __forceinline__ void put_f64(double* p, double v) {
    __hip_atomic_store(reinterpret_cast<uint64_t*>(p), __builtin_bit_cast(uint64_t, v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void put_i32(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void put_u64(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Commit time of phase q of an instance (wall clock), after its history.
__device__ __forceinline__ uint64_t* commit_times(const BatchArgs& a, const BatchInst& in) {
    return reinterpret_cast<uint64_t*>(a.hist + in.hist + (int64_t)(in.max_iter + 2) * (in.C + 2));
}

// Opens the next phase (tag `round`) of instance i with its tile 0 already
// taken by the calling block (thread 0), which goes on with it at once.
__device__ __forceinline__ void open_phase(const BatchArgs& a, int i, uint32_t round) {
    __hip_atomic_store(a.ctl + i, ((uint64_t)round << 32) | kBatchClaim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    (void)__hip_atomic_fetch_add(&a.sync->epoch, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Completion of phase 0 (block that finished its last tile): reduce the
// ranges (tagged rows, or `lmm` for a single tile), v^0 into the record and
// the history, then pass 0 opens with this block on its tile 0 and the
// decision in `d` (published for the other blocks when the pass has more
// tiles).  Returns false (all threads) if a wait was abandoned.
template <int BS>
__device__ __forceinline__ bool finish_range(const BatchArgs& a, int i, const BatchInst& in, uint32_t round,
                                             const uint32_t* lmm, Decision& d) {
    uint32_t lo, hi;
    if (lmm) {
        lo = lmm[0];
        hi = lmm[1];
    } else {
        const uint64_t t0 = wall_clock64();
        auto get = [&](int b, uint32_t& l, uint32_t& h) {
            uint32_t raw[2];
            if (!batch_poll<2>(a.rows + ((int64_t)in.tile0 + b) * kBatchRowWords, round, raw, a.sync, t0,
                               a.spin_ticks))
                return false;
            l = raw[0];
            h = raw[1];
            return true;
        };
        if (!reduce_minmax<BS>(get, in.ntiles, lo, hi)) return false;
    }
    if (threadIdx.x == 0) {
        double* hv = a.hist + in.hist;
        double v64[kMaxC];
        start_centroids(in.C, lo, hi, in.given, in.v0, in.dv0, v64);
        for (int k = 0; k < kMaxC; ++k) {
            const float v = k < in.C ? (float)v64[k] : 0.f;
            if (k < in.C) put_f64(hv + k, v64[k]);
            d.vn[k] = d.vo[k] = v;
            d.v64[k] = (double)v;
        }
        d.p = 0;
        BatchRec* rec = a.recs + i;
        put_i32(&rec->pass, 0);
        put_i32(&rec->done, 0);
        put_i32(&rec->iters, -1);
        put_i32(&rec->status, FCM_RUNNING);
        put_i32(&rec->passes, 0);
        put_i32(&rec->lo, (int32_t)lo);
        put_i32(&rec->hi, (int32_t)hi);
        put_f64(&rec->delta, __builtin_nan(""));
        put_f64(&rec->J, __builtin_nan(""));
        for (int k = 0; k < kMaxC; ++k) put_f64(&rec->vres[k], (double)d.vn[k]);
        put_u64(commit_times(a, in), wall_clock64());
    }
    __syncthreads();
    if (phase_tiles(a, i, 1u) > 1)
        publish_decision(a.dec + (int64_t)i * kBatchDecWords, round + 1, d.vn, d.vo, d.v64, in.C, 0);
    __syncthreads();
    if (threadIdx.x == 0) open_phase(a, i, round + 1);
    return true;
}

// Completion of pass p (block that finished its last tile): reduce the tile
// rows in tile order (or the one row in LDS), apply Eq.3 and the stopping
// rule, record, then retire the instance or open pass p + 1 with this block
// on its tile 0 and the decision in `d`.  Returns 0 (all threads) if a wait
// was abandoned, 1 if the instance finished, 2 if pass p + 1 was opened.
template <int C, int BS>
__device__ __forceinline__ int finish_pass(const BatchArgs& a, int i, const BatchInst& in, int p, uint32_t round,
                                           const float* lrow, Decision& d) {
    __shared__ Reduced<C> s_r;
    __shared__ Step<C> s_s;
    __shared__ double s_vcur[C];
    const bool fine = tile_set(a, round - a.round0 - 1u) != 0;
    if (lrow) {
        if (!reduce_rows<C, BS>(LocalRows<2 * C + 2>{const_cast<float*>(lrow)}, 1, in.kahan_only, s_r)) return 0;
    } else {
        const BatchRows<2 * C + 2> rows{a.rows + (int64_t)(fine ? in.tile0f : in.tile0) * kBatchRowWords, round,
                                        a.sync, (uint64_t)wall_clock64(), a.spin_ticks, 0};
        if (!reduce_rows<C, BS>(rows, fine ? in.ntilesf : in.ntiles, in.kahan_only, s_r)) return 0;
    }
    const int tid = threadIdx.x;
    if (tid == 0) {
        double vcur[C];
#pragma unroll
        for (int k = 0; k < C; ++k) {
            vcur[k] = d.v64[k];
            s_vcur[k] = vcur[k];
        }
        decide<C>(s_r, p, vcur, in.eps, in.max_iter, s_s);
    }
    __syncthreads();
    double* hv = a.hist + in.hist;
    BatchRec* rec = a.recs + i;
    const bool done = s_s.done != 0;
    if (tid < C) {
        put_f64(&rec->vres[tid], s_vcur[tid]);
        if (!done) put_f64(hv + (int64_t)(p + 1) * C + tid, s_s.vnext[tid]);
    } else if (tid == 64) {
        double* hd = hv + (int64_t)(in.max_iter + 2) * C;
        double* hJ = hd + (in.max_iter + 2);
        put_f64(hJ + p, s_s.J);
        put_f64(hd + p, s_s.delta);
        put_i32(&rec->iters, p);
        put_f64(&rec->J, s_s.J);
        put_f64(&rec->delta, s_s.delta);
        put_i32(&rec->passes, p + 1);
        put_i32(&rec->status, s_s.status);
        put_i32(&rec->done, s_s.done);
        if (!done) put_i32(&rec->pass, p + 1);
        put_u64(commit_times(a, in) + p + 1, wall_clock64());
    }
    if (done) {
        if (tid == 0) {
            __hip_atomic_store(a.ctl + i, ((uint64_t)(round + 1) << 32) | kBatchDoneClaims, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_sub(&a.sync->tiles_left, (uint32_t)max(in.ntiles, in.ntilesf), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_sub(&a.sync->active, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        return 1;
    }
    // the decision of pass p + 1: this block's copy, and the other blocks'
    // tagged words when the pass has more than one tile
    if (tid < kMaxC) {
        d.vo[tid] = tid < C ? (float)s_vcur[tid] : 0.f;
        d.vn[tid] = tid < C ? (float)s_s.vnext[tid] : 0.f;
        d.v64[tid] = tid < C ? s_s.vnext[tid] : 0.0;
    }
    if (tid == 0) d.p = p + 1;
    __syncthreads();
    if (phase_tiles(a, i, round + 1u - a.round0 - 1u) > 1)
        publish_decision(a.dec + (int64_t)i * kBatchDecWords, round + 1, d.vn, d.vo, d.v64, C, p + 1);
    __syncthreads();
    if (tid == 0) open_phase(a, i, round + 1);
    return 2;
}

// Block-wide choice of an instance with tiles left: every thread inspects the
// instances at rotation positions tid, tid + BS, ... from `start`; the
// nearest in rotation order wins.  Blocks start their rotations at spread
// positions, so that free blocks seldom race for the same tile.  Returns the
// instance or -1 (all threads).
template <int BS>
__device__ __forceinline__ int pick_instance(const BatchArgs& a, int start) {
    constexpr int NW = BS / 64;
    __shared__ int s_pos[NW];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    int best = 0x7FFFFFFF;
    for (int j = tid; j < a.I; j += BS) {
        int i = start + j;
        if (i >= a.I) i -= a.I;
        const uint64_t w = __hip_atomic_load(a.ctl + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t phase = (uint32_t)(w >> 32) - a.round0 - 1u;
        if ((uint32_t)(w & 0xFFFFu) < (uint32_t)phase_tiles(a, i, phase)) {
            best = j;
            break;  // later positions of this thread are further away
        }
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) best = min(best, __shfl_xor(best, off, 64));
    if (lane == 0) s_pos[wid] = best;
    __syncthreads();
    best = s_pos[0];
    for (int w = 1; w < NW; ++w) best = min(best, s_pos[w]);
    __syncthreads();
    if (best == 0x7FFFFFFF) return -1;
    const int i = start + best;
    return i >= a.I ? i - a.I : i;
}

}  // namespace

// BS threads per block; registers for two waves per SIMD (the second bound
// counts waves per SIMD), so 512 / BS blocks share a CU
template <int BS>
__global__ __launch_bounds__(BS, 2) void fcm_batch_kernel(BatchArgs a) {
    const int tid = threadIdx.x;
    BatchSync* sy = a.sync;
    __shared__ Decision s_d;
    __shared__ float s_row[2 * kMaxC + 2];
    __shared__ uint32_t s_mm[2];
    __shared__ int s_inst, s_k, s_last, s_go, s_ok;
    __shared__ uint32_t s_tag;
    if (blockIdx.x == 0 && tid == 0) sy->t_start = wall_clock64();
    const int start = (int)(((uint64_t)blockIdx.x * (uint32_t)a.I) / gridDim.x);
    uint64_t idle0 = wall_clock64();
    int spins = 0;
    int cur = -1;      // the instance of this block's last tile: tried first
    uint32_t seen = 0xFFFFFFFFu;  // epoch before this block's last scan that found nothing (thread 0)
    uint32_t ep = 0;              // epoch read at the top of this round (thread 0)
    bool have = false; // the block holds its next tile (tile 0 of a phase it opened, or the next open
                       // tile of the phase it works on) and that phase's decision
    int inst = -1, k = 0;
    uint32_t tag = 0;
    while (true) {
        // Shared values are copied to registers between two barriers before
        // thread 0 writes them again, so no wave can see a later value.
        __syncthreads();
        if (!have) {
            if (tid == 0) {
                const uint32_t active = __hip_atomic_load(&sy->active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t left = __hip_atomic_load(&sy->tiles_left, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t ab = __hip_atomic_load(&sy->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ep = __hip_atomic_load(&sy->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_go = active != 0u && ab == 0u && blockIdx.x < left;
                // stay with the last instance while it has tiles open: no
                // scan, and the blocks that share an instance stay together;
                // after a scan that found nothing, scan again only once a
                // phase has opened since (-3: nothing new)
                s_inst = ep == seen ? -3 : -2;
                if (cur >= 0) {
                    const uint64_t w = __hip_atomic_load(a.ctl + cur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const uint32_t phase = (uint32_t)(w >> 32) - a.round0 - 1u;
                    if ((uint32_t)(w & 0xFFFFu) < (uint32_t)phase_tiles(a, cur, phase)) s_inst = cur;
                }
            }
            __syncthreads();
            const int go = s_go, sticky = s_inst;
            __syncthreads();
            if (!go) break;
            const int i = sticky >= 0 ? sticky : (sticky == -3 ? -1 : pick_instance<BS>(a, start));
            if (tid == 0) {
                s_inst = -1;
                if (i >= 0) {
                    const uint64_t old = __hip_atomic_fetch_add(a.ctl + i, kBatchClaim, __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_AGENT);
                    const uint32_t kk = (uint32_t)(old & 0xFFFFu);
                    const uint32_t phase = (uint32_t)(old >> 32) - a.round0 - 1u;
                    if (kk < (uint32_t)phase_tiles(a, i, phase)) {
                        s_inst = i;
                        s_k = (int)kk;
                        s_tag = (uint32_t)(old >> 32);
                    }
                }
            }
            __syncthreads();
            inst = s_inst;
            k = s_k;
            tag = s_tag;
            if (inst < 0) {
                // nothing to take right now (every open tile is being run, or
                // the instances are between phases): back off, bounded by the
                // wait limit; a lost race for a tile retries at once
                if (tid == 0) {
                    // the epoch was read before the scan, so a phase opened
                    // during the scan makes the next round scan again
                    if (i < 0 && sticky != -3) seen = ep;
                    if (wall_clock64() - idle0 > a.spin_ticks) {
                        // the next round reads the abort word and leaves
                        __hip_atomic_store(&sy->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    } else if (i < 0) {
                        ++spins;
                        if (spins < 8)
                            __builtin_amdgcn_s_sleep(2);
                        else if (spins < 64)
                            __builtin_amdgcn_s_sleep(8);
                        else
                            __builtin_amdgcn_s_sleep(32);
                    }
                }
                continue;
            }
            if (tag - a.round0 - 1u >= 1u) {
                // the decision of the pass (and v^p in FP64 for completing it)
                if (tid == 0) {
                    uint32_t raw[kBatchDecWords];
                    s_ok = batch_poll<kBatchDecWords>(a.dec + (int64_t)inst * kBatchDecWords, tag, raw, sy,
                                                      wall_clock64(), a.spin_ticks);
                    for (int q = 0; q < kMaxC; ++q) {
                        const uint64_t bits =
                            (uint64_t)raw[kBatchDecF64 + 2 * q] | ((uint64_t)raw[kBatchDecF64 + 2 * q + 1] << 32);
                        s_d.vn[q] = __builtin_bit_cast(float, raw[q]);
                        s_d.vo[q] = __builtin_bit_cast(float, raw[kMaxC + q]);
                        s_d.v64[q] = __builtin_bit_cast(double, bits);
                    }
                    s_d.p = (int)raw[2 * kMaxC];
                }
                __syncthreads();
                if (!s_ok) break;
            }
        }
        have = false;
        spins = 0;
        cur = inst;
        const BatchInst& in = a.inst[inst];
        const uint32_t phase = tag - a.round0 - 1u;
        const int fine = tile_set(a, phase);
        const int ntiles = fine ? in.ntilesf : in.ntiles;
        const bool local = ntiles == 1;
        const int64_t t = (int64_t)(fine ? in.tile0f : in.tile0) + k;
        const BatchTile tl = a.tiles[t];
        if (phase == 0u) {
            tile_range<BS>(a, t, in, tl, tag, local ? s_mm : nullptr);
        } else {
            float* lrow = local ? s_row : nullptr;
            switch (in.C) {
                case 2: tile_pass<2, BS>(a, t, in, tl, s_d, tag, lrow); break;
                case 3: tile_pass<3, BS>(a, t, in, tl, s_d, tag, lrow); break;
                case 4: tile_pass<4, BS>(a, t, in, tl, s_d, tag, lrow); break;
                case 5: tile_pass<5, BS>(a, t, in, tl, s_d, tag, lrow); break;
                case 6: tile_pass<6, BS>(a, t, in, tl, s_d, tag, lrow); break;
                case 7: tile_pass<7, BS>(a, t, in, tl, s_d, tag, lrow); break;
                default: tile_pass<8, BS>(a, t, in, tl, s_d, tag, lrow); break;
            }
        }
        __syncthreads();  // the row is written (issued) before the arrival
        bool last = true;
        if (!local) {
            // one atomic add marks this tile finished and takes the next open
            // tile of the same phase, whose decision this block already holds
            if (tid == 0) {
                const uint64_t old = __hip_atomic_fetch_add(a.ctl + inst, kBatchArrive | kBatchClaim,
                                                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_last = (int)((old >> 16) & 0xFFFFu) == ntiles - 1;
                s_k = (int)(old & 0xFFFFu);
            }
            __syncthreads();
            last = s_last != 0;
            const int next = s_k;
            if (!last && next < ntiles) {
                have = true;
                k = next;
                idle0 = wall_clock64();
                continue;
            }
        }
        if (last) {
            int r;
            if (phase == 0u) {
                r = finish_range<BS>(a, inst, in, tag, local ? s_mm : nullptr, s_d) ? 2 : 0;
            } else {
                const int p = (int)phase - 1;
                const float* lrow = local ? s_row : nullptr;
                switch (in.C) {
                    case 2: r = finish_pass<2, BS>(a, inst, in, p, tag, lrow, s_d); break;
                    case 3: r = finish_pass<3, BS>(a, inst, in, p, tag, lrow, s_d); break;
                    case 4: r = finish_pass<4, BS>(a, inst, in, p, tag, lrow, s_d); break;
                    case 5: r = finish_pass<5, BS>(a, inst, in, p, tag, lrow, s_d); break;
                    case 6: r = finish_pass<6, BS>(a, inst, in, p, tag, lrow, s_d); break;
                    case 7: r = finish_pass<7, BS>(a, inst, in, p, tag, lrow, s_d); break;
                    default: r = finish_pass<8, BS>(a, inst, in, p, tag, lrow, s_d); break;
                }
            }
            if (r == 0) break;
            if (r == 2) {  // go on with tile 0 of the phase just opened
                have = true;
                k = 0;
                tag = tag + 1u;
            }
        }
        idle0 = wall_clock64();
    }
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

hipError_t batch_max_grid(int block, int ncu, int* max_grid) {
    int per_cu = 0;
    const void* k = block == 512   ? reinterpret_cast<const void*>(fcm_batch_kernel<512>)
                    : block == 128 ? reinterpret_cast<const void*>(fcm_batch_kernel<128>)
                                   : reinterpret_cast<const void*>(fcm_batch_kernel<256>);
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, block, 0);
    if (e != hipSuccess) return e;
    *max_grid = per_cu * ncu;
    return hipSuccess;
}

hipError_t launch_batch(const BatchArgs& a, int block, int grid, hipStream_t s) {
    if (block == 512)
        hipLaunchKernelGGL(fcm_batch_kernel<512>, dim3(grid), dim3(512), 0, s, a);
    else if (block == 128)
        hipLaunchKernelGGL(fcm_batch_kernel<128>, dim3(grid), dim3(128), 0, s, a);
    else
        hipLaunchKernelGGL(fcm_batch_kernel<256>, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_batch_labels(const BatchLabelArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(fcm_batch_labels_kernel, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace fcm
