// gfx950 device code of the Fuzzy C-Means iteration (Sec. 2.1, Sec. 4 of the paper).
// Templates shared by the per-cluster-count translation units fcm_pass_c*.hip.
//
// One fused streaming pass per iteration replaces the paper's per-cluster
// kernel sequence (per-pixel numerator/denominator kernel, two shared-memory
// reductions, a one-thread final sum, a membership kernel, Sec. 4.2-4.3):
//
//   pass p reads every voxel once (1 byte, 16-byte vector loads) and, in
//   registers, evaluates U^p from v^p and -- for p >= 1 -- U^(p-1) from
//   v^(p-1) (Eq.4), the per-voxel change max_j |u_j^p - u_j^(p-1)|, the
//   weights a_j = (u_j^p)^m, the centroid sums sum a_j x and sum a_j (Eq.3)
//   and the objective term sum_j a_j (x - v_j)^2 (Eq.1).  Memberships are
//   never stored.  Per-thread sums use FP32 with Kahan compensation per
//   16-voxel chunk; a block reduces them with wave64 DPP butterflies and an
//   LDS step into one partial row.  The partial rows are reduced in a fixed
//   order in FP64 -- or compensated FP32 -- into v^(p+1) (Eq.3), delta^p and
//   J^p, and the stopping rule of Algorithm 1 is applied on the device.
//
// Two drivers share that pass:
//   fcm_pass_kernel     one launch per pass; the last block to arrive (atomic
//                       ticket) reduces the rows and updates the state.
//   fcm_persist_kernel  one cooperative launch per solve (data range, v^0 and
//                       every pass); one grid barrier per pass, after which
//                       every block reduces all rows itself in the same order,
//                       so all blocks hold bitwise identical centroids and the
//                       same stopping decision without a second barrier.  Rows
//                       alternate between two buffers by pass parity.  Every
//                       barrier wait is bounded by a wall-clock limit and an
//                       abort flag, so every wave always exits.
//
// Membership form for m = 2 (exact algebra of Eq.4): with q_k = (x - v_k)^2,
// u_k = P_k / sum_j P_j where P_k = prod_{j != k} q_j, so one reciprocal
// serves all C memberships; u_k q_k is the same for every k and equals the
// voxel's objective term sum_k u_k^2 q_k.  Since u_k is proportional to
// q_k^(-alpha), alpha = 1/(m-1), other m follow from the m = 2 memberships u2:
// u_k = u2_k^alpha / sum_j u2_j^alpha (squares for m = 1.5, log2/exp2 else).
//
// Zero distances are exact: q_k = (x - v_k)^2 with no floor, so a voxel on a
// centroid gets membership exactly 1 there and exactly 0 elsewhere, and a
// cluster with no support keeps a zero denominator, as in the oracle.  The
// product forms run only when every centroid of both sets lies in [0, 255]
// with pairwise gaps >= 2^-6: then at most one q_k of a voxel is below 2^-14
// and every leave-one-out product lies in [2^-98, 2^112], inside the normal
// FP32 range.  Otherwise (coinciding or out-of-range centroids, a uniform
// per-pass decision) the pass uses the normalised form
// w_k = 2^(alpha (L_min - L_k)), L_k = log2 q_k clamped to [-1000, 256], which
// gives exact zeros and the equal split over coinciding centroids.

#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fcm.h"
#include "fcm_internal.h"
#include "fcm_learn_dev.h"

namespace fcm {

constexpr int kWaves = kBlock / 64;

// ---------------------------------------------------------------------------
// wave64 helpers
// ---------------------------------------------------------------------------

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}

__device__ __forceinline__ float readlane_f(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

// Sum over the 64 lanes of a fully active wave; every lane gets the same value.
// Butterfly within rows of 16 (xor 1, xor 2, half-mirror, mirror), then the
// four row sums in a fixed order.
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_mov<0x141>(v);  // row_half_mirror
    v += dpp_mov<0x140>(v);  // row_mirror
    return (readlane_f(v, 0) + readlane_f(v, 16)) + (readlane_f(v, 32) + readlane_f(v, 48));
}

__device__ __forceinline__ float wave_max(float v) {
    v = fmaxf(v, dpp_mov<0xB1>(v));
    v = fmaxf(v, dpp_mov<0x4E>(v));
    v = fmaxf(v, dpp_mov<0x141>(v));
    v = fmaxf(v, dpp_mov<0x140>(v));
    return fmaxf(fmaxf(readlane_f(v, 0), readlane_f(v, 16)), fmaxf(readlane_f(v, 32), readlane_f(v, 48)));
}

template <int CTRL>
__device__ __forceinline__ double dpp_mov_f64(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// FP64 sum over the 64 lanes of a fully active wave, same butterfly as
// wave_sum.  Each level adds a lane's value and its partner's, which is the
// same sum in both lanes (addition commutes), so every lane -- and every
// block holding the same values in the same lanes -- gets identical bits.
__device__ __forceinline__ double wave_sum_f64(double v) {
    v += dpp_mov_f64<0xB1>(v);
    v += dpp_mov_f64<0x4E>(v);
    v += dpp_mov_f64<0x141>(v);
    v += dpp_mov_f64<0x140>(v);
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) v = min(v, (uint32_t)__shfl_xor((int)v, off, 64));
    return v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off, 64));
    return v;
}

// Kahan step: s + (-c) carries the running sum, c the lost low part.
__device__ __forceinline__ void kahan_add(float& s, float& c, float v) {
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Error-free sum: s + e == a + b exactly.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// One butterfly level of a compensated (hi, lo) pair sum.  two_sum returns
// the exact rounding error, so partners compute identical bits.
template <int CTRL>
__device__ __forceinline__ void pair_level(float& hi, float& lo) {
    const float oh = dpp_mov<CTRL>(hi), ol = dpp_mov<CTRL>(lo);
    float s, e;
    two_sum(hi, oh, s, e);
    lo = (lo + ol) + e;
    hi = s;
}

// Compensated FP32 sum of (hi, lo) pairs over a fully active wave; the result
// (identical in every lane) is returned in hi, lo.
__device__ __forceinline__ void wave_sum_pair(float& hi, float& lo) {
    pair_level<0xB1>(hi, lo);
    pair_level<0x4E>(hi, lo);
    pair_level<0x141>(hi, lo);
    pair_level<0x140>(hi, lo);
    float h = readlane_f(hi, 0), l = readlane_f(lo, 0);
#pragma unroll
    for (int r = 16; r < 64; r += 16) {
        float s, e;
        two_sum(h, readlane_f(hi, r), s, e);
        l = (l + readlane_f(lo, r)) + e;
        h = s;
    }
    hi = h;
    lo = l;
}

template <typename T>
__device__ __forceinline__ void store_coherent(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ T load_coherent(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Marks this block's arrival after its partial row is written; returns true
// in every thread of the last block to arrive.
__device__ __forceinline__ bool arrive_last(uint32_t* ticket) {
    __shared__ int s_last;
    __syncthreads();
    if (threadIdx.x < 64) __threadfence();
    if (threadIdx.x == 0) {
        const uint32_t prev = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    const bool last = s_last != 0;
    if (last) __threadfence();
    return last;
}

// --- cross-block exchange of a cooperative launch ---------------------------
//
// Values travel as 64-bit words (round << 32) | payload, written and read with
// relaxed agent-scope atomics.  A 64-bit access is single-copy atomic, so each
// word proves by itself that it belongs to the current round: no flags, no
// fences and no second load after a wait.  Round r: every block writes its
// partial row as tagged words; block 0 polls the rows themselves, reduces,
// decides and writes the tagged broadcast words; the other blocks poll those.
// Every poll loop is bounded by a wall-clock limit; a timeout sets `abort`,
// which every other poll also watches, so all blocks exit.  Tags of earlier
// rounds never match (the round count only grows; buffers start zeroed).

__device__ __forceinline__ uint64_t tagged(uint32_t round, uint32_t payload) {
    return ((uint64_t)round << 32) | payload;
}

__device__ __forceinline__ void store_tagged(uint64_t* p, uint32_t round, uint32_t payload) {
    __hip_atomic_store(p, tagged(round, payload), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// one poll step's bookkeeping; true when the caller must give up.  The wall
// clock is read every step, the shared abort word only every 32nd (it costs a
// memory round trip); short sleeps first, longer ones once the wait drags on.
__device__ __forceinline__ bool poll_expired(SyncState* sy, uint64_t t0, uint64_t limit_ticks, int& spins) {
    if (wall_clock64() - t0 > limit_ticks) {
        __hip_atomic_store(&sy->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return true;
    }
    if ((spins & 31) == 31 && __hip_atomic_load(&sy->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return true;
    ++spins;
    if (spins < 64)
        __builtin_amdgcn_s_sleep(1);
    else
        __builtin_amdgcn_s_sleep(8);
    return false;
}

__device__ __forceinline__ bool poll_expired(BatchSync* sy, uint64_t t0, uint64_t limit_ticks, int& spins) {
    if (wall_clock64() - t0 > limit_ticks) {
        __hip_atomic_store(&sy->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return true;
    }
    if ((spins & 31) == 31 && __hip_atomic_load(&sy->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return true;
    ++spins;
    if (spins < 64)
        __builtin_amdgcn_s_sleep(1);
    else
        __builtin_amdgcn_s_sleep(8);
    return false;
}

// Wait until the K words at src carry `round`; payloads into out.  A short
// wait re-reads the whole group (its words are issued back to back, so a poll
// costs one memory round trip); once the wait drags on, only the group's last
// word (stored last by the writer) is watched, with back-off, and the group
// is read again when it arrives -- this bounds the load traffic when many
// blocks wait on many rows (a large all-gather grid).
constexpr int kFastPolls = 4;

template <int K>
__device__ __forceinline__ bool poll_tagged(const uint64_t* src, uint32_t round, uint32_t (&out)[K], SyncState* sy,
                                            uint64_t t0, uint64_t limit_ticks) {
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
        if (poll_expired(sy, t0, limit_ticks, spins)) return false;
        if (spins < kFastPolls) continue;
        while (true) {
            const uint64_t w = __hip_atomic_load(src + K - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((uint32_t)(w >> 32) == round) break;
            if (poll_expired(sy, t0, limit_ticks, spins)) return false;
        }
    }
}

// Row formats.  A block's row holds, for each of the 2C + 1 sums (num[C],
// den[C], J), a (sum, compensation) pair, then the max change; readers see it
// as R = 4C + 3 floats.

// Column-major float rows [R][G] in plain memory (one launch per pass; the
// last block reads them after the ticket's acquire).
struct PlainRows {
    float* P;
    int G;
    __device__ __forceinline__ void put_pair(int q, float s, float c) const {
        store_coherent(P + (2 * q) * G + blockIdx.x, s);
        store_coherent(P + (2 * q + 1) * G + blockIdx.x, c);
    }
    __device__ __forceinline__ void put_max(int q, float m) const { store_coherent(P + (2 * q) * G + blockIdx.x, m); }
    template <int R>
    __device__ __forceinline__ bool get(int b, float (&v)[R]) const {
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = P[r * G + b];
        return true;
    }
};

// Row-major tagged rows [G][stride], K = 2C + 2 words used (persistent
// launch).  Each pair is folded to one FP32 value (sum - comp, within half an
// ulp) so that a row is K self-validating words; a reader polls the whole row
// in one round trip.
template <int K>
struct TaggedRows {
    static constexpr int S = tagged_stride(K);
    uint64_t* W;
    uint32_t round;
    SyncState* sy;
    uint64_t t0, limit;
    bool two_level;  // read only by the block's XCD leader (the stores are agent-scope either way)
    __device__ __forceinline__ void put(int q, uint32_t payload) const {
        store_tagged(W + (size_t)blockIdx.x * S + q, round, payload);
    }
    __device__ __forceinline__ void put_pair(int q, float s, float c) const {
        put(q, __builtin_bit_cast(uint32_t, s - c));
    }
    __device__ __forceinline__ void put_max(int q, float m) const { put(q, __builtin_bit_cast(uint32_t, m)); }
    template <int R>
    __device__ __forceinline__ bool get(int b, float (&v)[R]) const {
        static_assert(R == 2 * (K - 1) + 1, "row format");
        uint32_t raw[K];
        if (!poll_tagged<K>(W + (size_t)b * S, round, raw, sy, t0, limit)) return false;
#pragma unroll
        for (int q = 0; q < K - 1; ++q) {
            v[2 * q] = __builtin_bit_cast(float, raw[q]);
            v[2 * q + 1] = 0.f;
        }
        v[R - 1] = __builtin_bit_cast(float, raw[K - 1]);
        return true;
    }
};

// Broadcast of block 0's decision: C centroids and (next pass, flag, done);
// the flag tells, after the data-range pass, whether the two-level exchange
// may be used.
template <int C>
__device__ __forceinline__ void publish_decision(SyncState* sy, uint32_t round, const float* v, int p, int done,
                                                 int flag = 0) {
#pragma unroll
    for (int k = 0; k < C; ++k) store_tagged(sy->bcw + k, round, __builtin_bit_cast(uint32_t, v[k]));
    store_tagged(sy->bcw + C, round, ((uint32_t)p << 2) | ((uint32_t)(flag != 0) << 1) | (uint32_t)(done != 0));
}

template <int C>
__device__ __forceinline__ bool await_decision(SyncState* sy, uint32_t round, uint64_t limit_ticks, float* v, int& p,
                                               int& done, int* flag = nullptr) {
    uint32_t raw[C + 1];
    if (!poll_tagged<C + 1>(sy->bcw, round, raw, sy, wall_clock64(), limit_ticks)) return false;
#pragma unroll
    for (int k = 0; k < C; ++k) v[k] = __builtin_bit_cast(float, raw[k]);
    p = (int)(raw[C] >> 2);
    done = (int)(raw[C] & 1u);
    if (flag) *flag = (int)((raw[C] >> 1) & 1u);
    return true;
}

// ---------------------------------------------------------------------------
// memberships of one voxel (Eq.4)
// ---------------------------------------------------------------------------

template <int C>
__device__ __forceinline__ void sq_dist(float x, const float (&v)[C], float (&q)[C]) {
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const float d = x - v[k];
        q[k] = d * d;
    }
}

// log2 q clamped so that q = 0 maps to a finite floor far below any other level
__device__ __forceinline__ float log2q(float q) {
    return __builtin_amdgcn_fmed3f(__builtin_amdgcn_logf(q), -1000.0f, 256.0f);
}

// P_k = prod_{j != k} q_j from prefix and suffix products (3C - 6 products).
template <int C>
__device__ __forceinline__ void leave_one_out(const float (&q)[C], float (&P)[C]) {
    float pre[C], suf[C];
    pre[1] = q[0];
#pragma unroll
    for (int k = 2; k < C; ++k) pre[k] = pre[k - 1] * q[k - 1];
    suf[C - 1] = q[C - 1];
#pragma unroll
    for (int k = C - 2; k >= 1; --k) suf[k] = q[k] * suf[k + 1];
    P[0] = suf[1];
    P[C - 1] = pre[C - 1];
#pragma unroll
    for (int k = 1; k < C - 1; ++k) P[k] = pre[k] * suf[k + 1];
}

struct Consts {
    float alpha, mexp;
};

// Membership forms.  The three product forms need separated centroids in
// [0, 255] (see the header comment); kNormLog works for any centroids.
enum Form : int {
    kProdM2 = 0,    // u = P / sum P                                  (m = 2)
    kProdM15 = 1,   // u = u2^2 / sum u2^2, u2 the m = 2 memberships   (m = 1.5)
    kProdPow = 2,   // u = u2^alpha / sum u2^alpha via log2/exp2        (other m)
    kNormLog = 3,   // u = w / sum w, w = 2^(alpha (L_min - L)), L = log2 q
};

// m = 2 memberships from squared distances: u_k = P_k / sum_j P_j.
template <int C>
__device__ __forceinline__ void prod_u(const float (&q)[C], float (&u)[C]) {
    float P[C];
    leave_one_out<C>(q, P);
    float S = P[0];
#pragma unroll
    for (int j = 1; j < C; ++j) S += P[j];
    const float r = __builtin_amdgcn_rcpf(S);
#pragma unroll
    for (int j = 0; j < C; ++j) u[j] = P[j] * r;
}

// Memberships of one voxel (Eq.4) and, when FULL, a = u^m and the voxel's
// objective term sum_j a_j q_j (Eq.1).  Working from u2 (in [0, 1], dominant
// entries >= 1/C) keeps the log2/exp2 arguments of the other forms small.
template <int C, int FORM, bool FULL>
__device__ __forceinline__ void memb(float x, const float (&v)[C], const Consts& k, float (&u)[C], float (&a)[C],
                                     float& Jv) {
    float q[C];
    sq_dist<C>(x, v, q);
    if constexpr (FORM == kNormLog) {
        float t[C];
#pragma unroll
        for (int j = 0; j < C; ++j) t[j] = log2q(q[j]);
        float Lmin = t[0];
#pragma unroll
        for (int j = 1; j < C; ++j) Lmin = fminf(Lmin, t[j]);
        float S = 0.f;
#pragma unroll
        for (int j = 0; j < C; ++j) {
            t[j] = (Lmin - t[j]) * k.alpha;  // log2 w_j <= 0
            u[j] = __builtin_amdgcn_exp2f(t[j]);
            S += u[j];
        }
        const float r = __builtin_amdgcn_rcpf(S);
#pragma unroll
        for (int j = 0; j < C; ++j) u[j] *= r;
        if constexpr (FULL) {
            const float lS = __builtin_amdgcn_logf(S);
            Jv = 0.f;
#pragma unroll
            for (int j = 0; j < C; ++j) {
                a[j] = __builtin_amdgcn_exp2f(k.mexp * (t[j] - lS));
                Jv = fmaf(a[j], q[j], Jv);
            }
        }
    } else {
        float u2[C];
        prod_u<C>(q, u2);
        if constexpr (FORM == kProdM2) {
#pragma unroll
            for (int j = 0; j < C; ++j) u[j] = u2[j];
            if constexpr (FULL) {
#pragma unroll
                for (int j = 0; j < C; ++j) a[j] = u[j] * u[j];
                Jv = u[0] * q[0];  // u_k q_k is the same for every k when m = 2
            }
        } else if constexpr (FORM == kProdM15) {
            float S = 0.f;
#pragma unroll
            for (int j = 0; j < C; ++j) {
                u[j] = u2[j] * u2[j];
                S += u[j];
            }
            const float r = __builtin_amdgcn_rcpf(S);
#pragma unroll
            for (int j = 0; j < C; ++j) u[j] *= r;
            if constexpr (FULL) {
                Jv = 0.f;
#pragma unroll
                for (int j = 0; j < C; ++j) {
                    a[j] = u[j] * __builtin_amdgcn_sqrtf(u[j]);
                    Jv = fmaf(a[j], q[j], Jv);
                }
            }
        } else {
            float t[C];
#pragma unroll
            for (int j = 0; j < C; ++j) t[j] = __builtin_amdgcn_fmed3f(__builtin_amdgcn_logf(u2[j]), -1000.0f, 0.0f);
            float tmax = t[0];
#pragma unroll
            for (int j = 1; j < C; ++j) tmax = fmaxf(tmax, t[j]);
            float S = 0.f;
#pragma unroll
            for (int j = 0; j < C; ++j) {
                t[j] = (t[j] - tmax) * k.alpha;  // log2 w_j <= 0, max 0
                u[j] = __builtin_amdgcn_exp2f(t[j]);
                S += u[j];
            }
            const float r = __builtin_amdgcn_rcpf(S);
#pragma unroll
            for (int j = 0; j < C; ++j) u[j] *= r;
            if constexpr (FULL) {
                const float lS = __builtin_amdgcn_logf(S);
                Jv = 0.f;
#pragma unroll
                for (int j = 0; j < C; ++j) {
                    a[j] = __builtin_amdgcn_exp2f(k.mexp * (t[j] - lS));
                    Jv = fmaf(a[j], q[j], Jv);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// per-thread accumulation
// ---------------------------------------------------------------------------

template <int C>
struct Acc {
    float ns[C], nc[C], ds[C], dc[C];
    float js, jc, dmax;
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int k = 0; k < C; ++k) ns[k] = nc[k] = ds[k] = dc[k] = 0.f;
        js = jc = dmax = 0.f;
    }
};

template <int C>
struct Group {
    float n[C], d[C], j;
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int k = 0; k < C; ++k) n[k] = d[k] = 0.f;
        j = 0.f;
    }
};

template <int C, int FORM, bool OLD>
__device__ __forceinline__ void voxel(float x, const float (&vn)[C], const float (&vo)[C], const Consts& k,
                                      Group<C>& g, float& dmax) {
    float u[C], a[C], Jv;
    memb<C, FORM, true>(x, vn, k, u, a, Jv);
    if constexpr (OLD) {
        float uo[C], ao[C], Jo;
        memb<C, FORM, false>(x, vo, k, uo, ao, Jo);
#pragma unroll
        for (int j = 0; j < C; ++j) dmax = fmaxf(dmax, fabsf(u[j] - uo[j]));
    }
#pragma unroll
    for (int j = 0; j < C; ++j) {
        g.n[j] = fmaf(a[j], x, g.n[j]);
        g.d[j] += a[j];
    }
    g.j += Jv;
}

template <int C>
__device__ __forceinline__ void fold_group(Acc<C>& acc, const Group<C>& g) {
#pragma unroll
    for (int k = 0; k < C; ++k) {
        kahan_add(acc.ns[k], acc.nc[k], g.n[k]);
        kahan_add(acc.ds[k], acc.dc[k], g.d[k]);
    }
    kahan_add(acc.js, acc.jc, g.j);
}

template <int C, int FORM, bool OLD>
__device__ __forceinline__ void chunk16(uint4 w, const float (&vn)[C], const float (&vo)[C], const Consts& k,
                                        Acc<C>& acc) {
    Group<C> g;
    g.zero();
    const uint32_t words[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const float x = (float)((words[i] >> (8 * b)) & 0xFFu);
            voxel<C, FORM, OLD>(x, vn, vo, k, g, acc.dmax);
        }
    }
    fold_group<C>(acc, g);
}

// Range and separation test of a centroid set for the product forms (uniform).
template <int C>
__device__ __forceinline__ bool separated(const float (&v)[C]) {
    bool ok = true;
#pragma unroll
    for (int i = 0; i < C; ++i) {
        ok = ok && v[i] >= 0.0f && v[i] <= 255.0f;
#pragma unroll
        for (int j = i + 1; j < C; ++j) ok = ok && fabsf(v[i] - v[j]) >= 0.015625f;
    }
    return ok;
}

// The voxels of this thread for one pass.  `resident`: the thread owns at most
// one 16-voxel chunk, already in `mine` (uniform across the grid).
template <int C, int FORM, int UNROLL, bool OLD>
__device__ __forceinline__ void pass_body(const PassArgs& a, const float (&vn)[C], const float (&vo)[C],
                                          const Consts& kc, Acc<C>& acc, bool resident, uint4 mine) {
    const int tid = threadIdx.x;
    const uint4* body = reinterpret_cast<const uint4*>(a.x + a.head);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    int64_t c = (int64_t)blockIdx.x * kBlock + tid;
    const int64_t nb = a.nbody;
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    if (resident) {
        if (c < nb) chunk16<C, FORM, OLD>(mine, vn, vo, kc, acc);
    } else if constexpr (UNROLL == 1) {
        uint4 cur = c < nb ? body[c] : z;
        while (c < nb) {
            const int64_t cn = c + stride;
            const uint4 nx = cn < nb ? body[cn] : z;
            chunk16<C, FORM, OLD>(cur, vn, vo, kc, acc);
            cur = nx;
            c = cn;
        }
    } else {
        uint4 c0 = c < nb ? body[c] : z;
        uint4 c1 = c + stride < nb ? body[c + stride] : z;
        while (c < nb) {
            const int64_t cn = c + 2 * stride;
            const uint4 n0 = cn < nb ? body[cn] : z;
            const uint4 n1 = cn + stride < nb ? body[cn + stride] : z;
            chunk16<C, FORM, OLD>(c0, vn, vo, kc, acc);
            if (c + stride < nb) chunk16<C, FORM, OLD>(c1, vn, vo, kc, acc);
            c0 = n0;
            c1 = n1;
            c = cn;
        }
    }
    // unaligned head and tail (< 16 voxels each) go to block 0
    if (blockIdx.x == 0) {
        const int64_t tail0 = a.head + 16 * nb;
        const int64_t nr = a.head + (a.n - tail0);
        if (tid < nr) {
            const int64_t i = tid < a.head ? (int64_t)tid : tail0 + (tid - a.head);
            Group<C> g;
            g.zero();
            voxel<C, FORM, OLD>((float)a.x[i], vn, vo, kc, g, acc.dmax);
            fold_group<C>(acc, g);
        }
    }
}

// Pass p of this block with the form chosen for the two centroid sets.
template <int C, int MK, int UNROLL>
__device__ __forceinline__ void run_pass(const PassArgs& a, int p, const float (&vn)[C], const float (&vo)[C],
                                         Acc<C>& acc, bool resident, uint4 mine) {
    constexpr int FAST = MK == kM2 ? kProdM2 : (MK == kM15 ? kProdM15 : kProdPow);
    const Consts kc{a.alpha, a.mexp};
    acc.zero();
    if (separated<C>(vn) && (p == 0 || separated<C>(vo))) {
        if (p == 0)
            pass_body<C, FAST, UNROLL, false>(a, vn, vo, kc, acc, resident, mine);
        else
            pass_body<C, FAST, UNROLL, true>(a, vn, vo, kc, acc, resident, mine);
    } else {
        if (p == 0)
            pass_body<C, kNormLog, UNROLL, false>(a, vn, vo, kc, acc, resident, mine);
        else
            pass_body<C, kNormLog, UNROLL, true>(a, vn, vo, kc, acc, resident, mine);
    }
}

// ---------------------------------------------------------------------------
// reductions across blocks: Eq.3 update and the stopping rule
// ---------------------------------------------------------------------------

// Block reduction of the thread sums into this block's partial row: wave
// butterflies, then the waves in order (Kahan).  Row entries: for each k < C
// num (sum, comp), den (sum, comp); then J (sum, comp); then max |dU|.
template <int C, int BS = kBlock, typename Rows>
__device__ __forceinline__ void write_partial_row(const Acc<C>& acc, const Rows& rows) {
    constexpr int NQ = 2 * C + 1;
    constexpr int NW = BS / 64;
    __shared__ float s_red[NW][NQ + 1];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    float f[NQ];
#pragma unroll
    for (int k = 0; k < C; ++k) {
        f[k] = acc.ns[k] - acc.nc[k];
        f[C + k] = acc.ds[k] - acc.dc[k];
    }
    f[2 * C] = acc.js - acc.jc;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const float s = wave_sum(f[q]);
        if (lane == 0) s_red[wid][q] = s;
    }
    const float m = wave_max(acc.dmax);
    if (lane == 0) s_red[wid][NQ] = m;
    __syncthreads();
    if (tid < NQ) {
        float s = 0.f, c = 0.f;
        for (int w = 0; w < NW; ++w) kahan_add(s, c, s_red[w][tid]);
        rows.put_pair(tid, s, c);
    } else if (tid == NQ) {
        float mm = s_red[0][NQ];
        for (int w = 1; w < NW; ++w) mm = fmaxf(mm, s_red[w][NQ]);
        rows.put_max(NQ, mm);
    }
}

template <int C>
struct Reduced {
    double res[2 * C + 1];  // num[C], den[C], J
    float dm;               // max |dU|
};

// Whole-block reduction of the G partial rows in a fixed order (thread t takes
// rows t, t + blockDim, ...; then wave butterflies and the waves in order); the
// result is written to `out` (shared) and valid in every thread after the
// call.  Returns false in every thread if a row could not be obtained.
template <int C, int BS = kBlock, typename Rows>
__device__ bool reduce_rows(const Rows& rows, int G, int kahan_only, Reduced<C>& out) {
    constexpr int NQ = 2 * C + 1;
    constexpr int R = partial_rows(C);
    constexpr int NW = BS / 64;
    __shared__ double s_sum[NW][NQ];
    __shared__ float s_lo[NW][NQ];
    __shared__ float s_max[NW];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    float dm = 0.f;
    int bad = 0;
    double acc[NQ];
    float hi[NQ], lo[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        acc[q] = 0.0;
        hi[q] = lo[q] = 0.f;
    }
    for (int b = tid; b < G; b += BS) {
        float v[R];
        if (!rows.template get<R>(b, v)) {
            bad = 1;
            break;
        }
        if (!kahan_only) {
            // FP64 over the block partials, each taken as (sum - comp)
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc[q] += (double)v[2 * q] - (double)v[2 * q + 1];
        } else {
            // compensated FP32 throughout: (hi, lo) pairs combined error-free
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                float s, e;
                two_sum(hi[q], v[2 * q], s, e);
                hi[q] = s;
                lo[q] += e - v[2 * q + 1];
            }
        }
        dm = fmaxf(dm, v[R - 1]);
    }
    if (__syncthreads_or(bad)) return false;
    if (!kahan_only) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const double s = wave_sum_f64(acc[q]);
            if (lane == 0) s_sum[wid][q] = s;
        }
    } else {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            wave_sum_pair(hi[q], lo[q]);
            if (lane == 0) {
                s_sum[wid][q] = (double)hi[q];
                s_lo[wid][q] = lo[q];
            }
        }
    }
    const float m = wave_max(dm);
    if (lane == 0) s_max[wid] = m;
    __syncthreads();
    if (tid < NQ) {
        double r;
        if (!kahan_only) {
            r = s_sum[0][tid];
            for (int w = 1; w < NW; ++w) r += s_sum[w][tid];
        } else {
            float h = (float)s_sum[0][tid], l = s_lo[0][tid];
            for (int w = 1; w < NW; ++w) {
                float s, e;
                two_sum(h, (float)s_sum[w][tid], s, e);
                h = s;
                l += e + s_lo[w][tid];
            }
            r = (double)(h + l);
        }
        out.res[tid] = r;
    } else if (tid == NQ) {
        float mm = s_max[0];
        for (int w = 1; w < NW; ++w) mm = fmaxf(mm, s_max[w]);
        out.dm = mm;
    }
    __syncthreads();
    return true;
}

// Two-level exchange of a persistent launch (each block's row already
// stored, with agent scope like every exchange word).  Level 1: block
// x < kXcds polls the rows of blocks x, x + kXcds, ... (which share its XCD
// when the blocks were dealt to the XCDs in turn; one row per thread),
// adds them in FP64 in that order (wave butterflies, then the waves in
// order) and stores its XCD row.  Level 2:
// every block polls the (up to) kXcds XCD rows and adds them in XCD order, so
// all blocks hold bitwise identical sums and take the decision themselves.
// False in every thread if a wait hit its time limit.
template <int C>
__device__ bool xcd_exchange(const TaggedRows<2 * C + 2>& rows, int G, uint32_t round, SyncState* sy,
                             uint64_t limit, Reduced<C>& out) {
    constexpr int NQ = 2 * C + 1;
    constexpr int R = partial_rows(C);
    constexpr int XW = 2 * NQ + 1;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    uint64_t* xr = &sy->xrow[round & 1u][0][0];
    int bad = 0;
    if ((int)blockIdx.x < kXcds) {
        __shared__ double s_l1[kWaves][NQ];
        __shared__ float s_l1m[kWaves];
        const int x = blockIdx.x;
        const int nx = (G - x + kXcds - 1) / kXcds;  // rows x, x + kXcds, ... below G
        double acc[NQ];
        float dm = 0.f;
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
        for (int i = tid; i < nx; i += kBlock) {
            float v[R];
            if (!rows.template get<R>(x + kXcds * i, v)) {
                bad = 1;
                break;
            }
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc[q] += (double)v[2 * q] - (double)v[2 * q + 1];
            dm = fmaxf(dm, v[R - 1]);
        }
        if (__syncthreads_or(bad)) return false;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const double r = wave_sum_f64(acc[q]);
            if (lane == 0) s_l1[wid][q] = r;
        }
        const float m = wave_max(dm);
        if (lane == 0) s_l1m[wid] = m;
        __syncthreads();
        if (tid < NQ) {
            double r = s_l1[0][tid];
            for (int w = 1; w < kWaves; ++w) r += s_l1[w][tid];
            const uint64_t bits = __builtin_bit_cast(uint64_t, r);
            store_tagged(xr + x * kXcdRowWords + 2 * tid, round, (uint32_t)bits);
            store_tagged(xr + x * kXcdRowWords + 2 * tid + 1, round, (uint32_t)(bits >> 32));
        } else if (tid == NQ) {
            float mm = s_l1m[0];
            for (int w = 1; w < kWaves; ++w) mm = fmaxf(mm, s_l1m[w]);
            store_tagged(xr + x * kXcdRowWords + 2 * NQ, round, __builtin_bit_cast(uint32_t, mm));
        }
    }
    __shared__ double s_l2[kXcds][NQ];
    __shared__ float s_l2m[kXcds];
    const int nxcd = G < kXcds ? G : kXcds;
    if (tid < nxcd) {
        uint32_t raw[XW];
        if (!poll_tagged<XW>(xr + tid * kXcdRowWords, round, raw, sy, wall_clock64(), limit)) {
            bad = 1;
        } else {
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                s_l2[tid][q] = __builtin_bit_cast(double, (uint64_t)raw[2 * q] | ((uint64_t)raw[2 * q + 1] << 32));
            s_l2m[tid] = __builtin_bit_cast(float, raw[2 * NQ]);
        }
    }
    if (__syncthreads_or(bad)) return false;
    if (tid < NQ) {
        double r = s_l2[0][tid];
        for (int x = 1; x < nxcd; ++x) r += s_l2[x][tid];
        out.res[tid] = r;
    } else if (tid == NQ) {
        float mm = s_l2m[0];
        for (int x = 1; x < nxcd; ++x) mm = fmaxf(mm, s_l2m[x]);
        out.dm = mm;
    }
    __syncthreads();
    return true;
}

// Outcome of pass p (Eq.3 update and Algorithm 1's test), computed identically
// by whoever calls it.
template <int C>
struct Step {
    double vnext[C];
    double delta, J;
    int status, done;
};

template <int C>
__device__ __forceinline__ void decide(const Reduced<C>& r, int p, const double* vcur, double eps, int max_iter,
                                       Step<C>& s) {
    bool bad = false;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const double num = r.res[k], den = r.res[C + k];
        s.vnext[k] = den > 0.0 ? num / den : vcur[k];
        if (!isfinite(s.vnext[k])) bad = true;
    }
    s.J = r.res[2 * C];
    if (!isfinite(s.J)) bad = true;
    s.delta = p > 0 ? (double)r.dm : __builtin_nan("");
    s.status = FCM_RUNNING;
    s.done = 0;
    if (bad) {
        s.status = FCM_ENUMERIC;
        s.done = 1;
    } else if (p >= 1 && s.delta < eps) {
        s.status = FCM_OK;
        s.done = 1;
    } else if (p >= max_iter) {
        s.status = FCM_NOT_CONVERGED;
        s.done = 1;
    }
}

// Record pass p in the history and the state (one thread of one block).
template <int C>
__device__ __forceinline__ void commit(const PassArgs& a, int p, const double* vcur, const Step<C>& s) {
    DevState* st = a.st;
    a.hist_J[p] = s.J;
    a.hist_d[p] = s.delta;
#pragma unroll
    for (int k = 0; k < C; ++k) st->vres[k] = vcur[k];
    st->iters = p;
    st->J = s.J;
    st->delta = s.delta;
    st->passes = p + 1;
    st->sync.passes_total += 1;
    if (!s.done) {
#pragma unroll
        for (int k = 0; k < C; ++k) {
            a.hist_v[(int64_t)(p + 1) * C + k] = s.vnext[k];
            st->v32[(p + 1) & 1][k] = (float)s.vnext[k];
        }
        st->pass = p + 1;
    }
    st->status = s.status;
    st->done = s.done;
}

// ---------------------------------------------------------------------------
// driver 1: one launch per pass
// ---------------------------------------------------------------------------

template <int C, int MK, int UNROLL>
__global__ __launch_bounds__(kBlock) void fcm_pass_kernel(PassArgs a) {
    DevState* st = a.st;
    if (st->done) return;
    const int p = st->pass;
    float vn[C], vo[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
        vn[k] = st->v32[p & 1][k];
        vo[k] = st->v32[(p + 1) & 1][k];
    }
    Acc<C> acc;
    run_pass<C, MK, UNROLL>(a, p, vn, vo, acc, false, make_uint4(0u, 0u, 0u, 0u));
    const int G = gridDim.x;
    const PlainRows rows{a.partials, G};
    write_partial_row<C>(acc, rows);
    if (!arrive_last(&st->ticket)) return;
    __shared__ Reduced<C> s_r;
    reduce_rows<C>(rows, G, a.kahan_only, s_r);
    if (threadIdx.x == 0) {
        double vcur[C];
#pragma unroll
        for (int k = 0; k < C; ++k) vcur[k] = a.hist_v[(int64_t)p * C + k];
        Step<C> s;
        decide<C>(s_r, p, vcur, a.eps, a.max_iter, s);
        commit<C>(a, p, vcur, s);
        st->ticket = 0;
    }
}

// ---------------------------------------------------------------------------
// data range and initial centroids
// ---------------------------------------------------------------------------

// min and max grey level of this thread's voxels (grid-stride chunks + ragged)
// Grey-level range of this thread's voxels; with `bins` (a shared 256-entry
// table) also their histogram.
__device__ __forceinline__ void thread_minmax(const uint8_t* x, int64_t n, int64_t head, int64_t nbody,
                                              uint32_t& lo, uint32_t& hi, uint32_t* bins = nullptr) {
    const int tid = threadIdx.x;
    const uint4* body = reinterpret_cast<const uint4*>(x + head);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + tid; c < nbody; c += stride) {
        const uint4 w = body[c];
        const uint32_t words[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const uint32_t v = (words[i] >> (8 * b)) & 0xFFu;
                lo = min(lo, v);
                hi = max(hi, v);
                if (bins) atomicAdd(bins + v, 1u);
            }
        }
    }
    if (blockIdx.x == 0) {
        const int64_t tail0 = head + 16 * nbody;
        const int64_t nr = head + (n - tail0);
        if (tid < nr) {
            const int64_t i = tid < head ? (int64_t)tid : tail0 + (tid - head);
            lo = min(lo, (uint32_t)x[i]);
            hi = max(hi, (uint32_t)x[i]);
            if (bins) atomicAdd(bins + x[i], 1u);
        }
    }
}

// block min/max; (lo, hi) is valid in thread 0 after the call
template <int BS = kBlock>
__device__ __forceinline__ void block_minmax(uint32_t& lo, uint32_t& hi) {
    constexpr int NW = BS / 64;
    __shared__ uint32_t s_lo[NW], s_hi[NW];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    lo = wave_min_u32(lo);
    hi = wave_max_u32(hi);
    if (lane == 0) {
        s_lo[wid] = lo;
        s_hi[wid] = hi;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < NW; ++w) {
            lo = min(lo, s_lo[w]);
            hi = max(hi, s_hi[w]);
        }
    }
}

// Whole-block reduction of the G (lo, hi) rows obtained through
// get(b, lo_b, hi_b); valid in every thread after the call.  Returns false in
// every thread if a row could not be obtained.
template <int BS = kBlock, typename Get>
__device__ __forceinline__ bool reduce_minmax(const Get& get, int G, uint32_t& lo, uint32_t& hi) {
    constexpr int NW = BS / 64;
    __shared__ uint32_t s_lo[NW], s_hi[NW];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    lo = 255u;
    hi = 0u;
    int bad = 0;
    for (int b = tid; b < G; b += BS) {
        uint32_t l, h;
        if (!get(b, l, h)) {
            bad = 1;
            break;
        }
        lo = min(lo, l);
        hi = max(hi, h);
    }
    if (__syncthreads_or(bad)) return false;
    lo = wave_min_u32(lo);
    hi = wave_max_u32(hi);
    if (lane == 0) {
        s_lo[wid] = lo;
        s_hi[wid] = hi;
    }
    __syncthreads();
    lo = s_lo[0];
    hi = s_hi[0];
    for (int w = 1; w < NW; ++w) {
        lo = min(lo, s_lo[w]);
        hi = max(hi, s_hi[w]);
    }
    __syncthreads();
    return true;
}

// v^0 (C values, FP64 holding FP32 values) for start mode `mode`:
//   0  evenly spaced: lo + k (hi - lo) / (C - 1), the product exact, the
//      quotient and the sum rounded once each in FP64, then rounded to FP32;
//   1  the given values v0[k];
//   2  the values dv0[k] in device memory (written by an earlier kernel, e.g.
//      the learned warm start); any non-finite value selects mode 0.
__device__ __forceinline__ void start_centroids(int C, uint32_t lo, uint32_t hi, int mode, const double* v0,
                                                const double* dv0, double* out) {
    bool spaced = mode == 0;
    if (mode == 2)
        for (int k = 0; k < C; ++k)
            if (!isfinite(dv0[k])) spaced = true;
    for (int k = 0; k < C; ++k) {
        float v32;
        if (spaced)
            v32 = (float)((double)lo + (double)(k * (int)(hi - lo)) / (double)(C - 1));
        else
            v32 = (float)(mode == 1 ? v0[k] : dv0[k]);
        out[k] = (double)v32;
    }
}

// Write the start of a solve into the state (one thread).
__device__ __forceinline__ void commit_start(DevState* st, double* hist_v, int C, uint32_t lo, uint32_t hi,
                                             const double* v) {
    for (int k = 0; k < kMaxC; ++k) {
        float v32 = 0.f;
        if (k < C) {
            v32 = (float)v[k];
            hist_v[k] = v[k];
        }
        st->v32[0][k] = v32;
        st->v32[1][k] = v32;
        st->vres[k] = (double)v32;
    }
    st->lo = (int32_t)lo;
    st->hi = (int32_t)hi;
    st->pass = 0;
    st->iters = -1;
    st->passes = 0;
    st->status = FCM_RUNNING;
    st->delta = __builtin_nan("");
    st->J = __builtin_nan("");
    st->done = 0;
}

// ---------------------------------------------------------------------------
// defuzzification inside the solve
// ---------------------------------------------------------------------------

// LUT[g] = argmin_j |g - v_j| in FP64, ties to the lowest j (the nearest
// centroid is the cluster of maximal membership for m > 1).
__device__ __forceinline__ void label_table(const double* v, int C, uint8_t* lut) {
    for (int g = threadIdx.x; g < 256; g += kBlock) {
        int best = 0;
        double bd = fabs((double)g - v[0]);
        for (int k = 1; k < C; ++k) {
            const double d = fabs((double)g - v[k]);
            if (d < bd) {
                bd = d;
                best = k;
            }
        }
        lut[g] = (uint8_t)best;
    }
}

__device__ __forceinline__ uint4 label_chunk(uint4 w, const uint8_t* lut) {
    const uint32_t words[4] = {w.x, w.y, w.z, w.w};
    uint32_t o[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t x = words[i];
        o[i] = (uint32_t)lut[x & 0xFFu] | ((uint32_t)lut[(x >> 8) & 0xFFu] << 8) |
               ((uint32_t)lut[(x >> 16) & 0xFFu] << 16) | ((uint32_t)lut[x >> 24] << 24);
    }
    return make_uint4(o[0], o[1], o[2], o[3]);
}

// Labels of every voxel of the launch's share (grid-stride chunks; the
// thread's resident chunk from registers), head and tail by block 0.
__device__ __forceinline__ void write_labels(const PassArgs& a, const uint8_t* lut, bool resident, uint4 mine) {
    const int tid = threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t gt = (int64_t)blockIdx.x * kBlock + tid;
    if (a.labels_bytewise) {
        for (int64_t i = gt; i < a.n; i += stride) a.labels[i] = lut[a.x[i]];
        return;
    }
    const uint4* in = reinterpret_cast<const uint4*>(a.x + a.head);
    uint4* out = reinterpret_cast<uint4*>(a.labels + a.head);
    if (resident) {
        if (gt < a.nbody) out[gt] = label_chunk(mine, lut);
    } else {
        for (int64_t c = gt; c < a.nbody; c += stride) out[c] = label_chunk(in[c], lut);
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

// ---------------------------------------------------------------------------
// driver 2: one cooperative launch per solve
// ---------------------------------------------------------------------------

template <int C, int MK, int UNROLL>
__global__ __launch_bounds__(kBlock) void fcm_persist_kernel(PassArgs a) {
    DevState* st = a.st;
    SyncState* sy = &st->sync;
    const int G = gridDim.x;
    const int tid = threadIdx.x;
    const bool leader = blockIdx.x == 0;
    __shared__ double s_v64[C];
    __shared__ float s_vn[C], s_vo[C];
    __shared__ int s_p, s_done, s_ok, s_xcd;
    if (tid == 0) {
        s_ok = 1;
        s_xcd = 0;  // set after the data-range pass when the two-level exchange is usable
    }
    __shared__ Reduced<C> s_r;
    // the last round of the previous launch (written by its block 0 before it
    // ended); tags of this launch start above it
    uint32_t round = __hip_atomic_load(&sy->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

    if (a.do_init) {
        // learned start: the data-range pass also counts the grey levels
        // (shared table per block, then global counters), and block 0 runs
        // the network on the histogram before the first pass
        const bool learned = a.given == 3;
        __shared__ uint32_t s_bins[kWaves][256];  // one table per wave: fewer same-address conflicts
        if (learned) {
#pragma unroll
            for (int w = 0; w < kWaves; ++w) s_bins[w][tid] = 0u;
            __syncthreads();
        }
        uint32_t lo = 255u, hi = 0u;
        thread_minmax(a.x, a.n, a.head, a.nbody, lo, hi, learned ? s_bins[tid >> 6] : nullptr);
        block_minmax(lo, hi);
        if (learned) {
            __syncthreads();
            uint32_t c = 0u;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) c += s_bins[w][tid];
            // block b adds into copy b mod kHistCopies, so that a busy grey
            // level sees kHistCopies times fewer same-address atomics.  The
            // returned value is consumed so that the wave waits until its add
            // has been performed before the barrier.
            if (c) {
                const uint32_t old = __hip_atomic_fetch_add(a.ghist + (blockIdx.x % kHistCopies) * 256 + tid, c,
                                                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                asm volatile("" ::"v"(old));
            }
            __syncthreads();
        }
        ++round;
        uint64_t* mm = a.mm_rows + (size_t)(round & 1u) * 2 * G;
        // the XCD the block runs on travels with its range (two-level exchange)
        const uint32_t xcc = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 0xFu;  // HW_REG_XCC_ID
        if (tid == 0) {
            // the block's counts are released before its range row
            if (learned) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            store_tagged(mm + 2 * blockIdx.x, round, lo | (xcc << 8));
            store_tagged(mm + 2 * blockIdx.x + 1, round, hi);
        }
        if (leader || a.allgather) {
            const uint64_t t0 = wall_clock64();
            // blocks b and b + kXcds share an XCD when the blocks were dealt
            // to the XCDs in turn, from any starting XCD: XCD(b) - b is the
            // same (mod kXcds) for every block, block 0's XCD here
            int deal_bad = 0;
            auto get = [&](int b, uint32_t& l, uint32_t& h) {
                uint32_t raw[2];
                if (!poll_tagged<2>(mm + 2 * b, round, raw, sy, t0, a.spin_ticks)) return false;
                l = raw[0] & 0xFFu;
                h = raw[1];
                if ((((raw[0] >> 8) - (uint32_t)b - xcc) & (kXcds - 1)) != 0u) deal_bad = 1;
                return true;
            };
            if (!reduce_minmax(get, G, lo, hi)) return;
            const int xcd_ok = a.xcd && leader && !__syncthreads_or(deal_bad);
            __shared__ double s_w0[kMaxC];
            if (learned) {
                // every block whose range row was seen released its counts
                // first.  With all-gather every block runs the network itself
                // on the same counts (same code, same result: no broadcast);
                // otherwise block 0 does and broadcasts the start.
                __shared__ float s_h[256], s_a0[256], s_a1[128], s_a2[64], s_tmp[256], s_y[kMaxC];
                // The counters are read with device-scope atomic loads, which
                // are served at the same coherence point where the adds were
                // performed; each writer's adds had completed (their results
                // were consumed) before its release fence and range row, and
                // these loads are issued only after the barrier that follows
                // the polls that saw every range row.  An acquire fence here
                // would add nothing for atomic loads but cost ~5 us (an L2
                // invalidation in every wave).
                uint32_t part[kHistCopies];
#pragma unroll
                for (int c = 0; c < kHistCopies; ++c)
                    part[c] = __hip_atomic_load(a.ghist + c * 256 + tid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                uint32_t cnt = 0u;
#pragma unroll
                for (int c = 0; c < kHistCopies; ++c) cnt += part[c];
                // the counters of the next learned launch (the other buffer)
                // start at zero: no block of this launch touches them
                if (leader)
                    for (int c = 0; c < kHistCopies; ++c) a.ghist_next[c * 256 + tid] = 0u;
                s_h[tid] = hist_norm(cnt, a.n);
                __syncthreads();
                mlp_block_forward<true>(a.mlp_w, s_h, C, s_a0, s_a1, s_a2, s_tmp, s_y);
                __syncthreads();
                if (tid == 0) warm_post_one(s_y, (int)lo, (int)hi, C, s_w0);
            }
            if (tid == 0) {
                double v[C];
                start_centroids(C, lo, hi, learned ? 2 : a.given, a.v0, learned ? s_w0 : a.dv0, v);
                for (int k = 0; k < C; ++k) {
                    s_v64[k] = v[k];
                    s_vn[k] = (float)v[k];
                    s_vo[k] = (float)v[k];
                }
                s_p = 0;
                s_done = 0;
                s_xcd = xcd_ok;
                if (leader) commit_start(st, a.hist_v, C, lo, hi, v);
                if (!a.allgather) publish_decision<C>(sy, round, s_vn, 0, 0, xcd_ok);
            }
        } else {
            if (tid == 0) {
                float v[C];
                int p = 0, done = 0, xf = 0;
                s_ok = await_decision<C>(sy, round, a.spin_ticks, v, p, done, &xf);
#pragma unroll
                for (int k = 0; k < C; ++k) {
                    s_vn[k] = s_vo[k] = v[k];
                    s_v64[k] = (double)v[k];  // v^0 is FP32-exact
                }
                s_p = p;
                s_done = done;
                s_xcd = a.xcd && xf;
            }
            __syncthreads();
            if (!s_ok) return;
        }
    } else {
        if (tid == 0) {
            s_p = st->pass;
            s_done = st->done;
        }
        __syncthreads();
        if (tid < C) {
            const int p = s_p;
            s_v64[tid] = a.hist_v[(int64_t)p * C + tid];
            s_vn[tid] = st->v32[p & 1][tid];
            s_vo[tid] = st->v32[(p + 1) & 1][tid];
        }
    }
    __syncthreads();

    // the thread's only chunk stays in registers when the grid covers the data
    const int64_t stride = (int64_t)G * kBlock;
    const bool resident = a.nbody <= stride;
    uint4 mine = make_uint4(0u, 0u, 0u, 0u);
    {
        const int64_t c = (int64_t)blockIdx.x * kBlock + tid;
        if (resident && c < a.nbody) mine = reinterpret_cast<const uint4*>(a.x + a.head)[c];
    }

    for (int budget = a.max_passes; budget > 0 && !s_done; --budget) {
        const int p = s_p;
        float vn[C], vo[C];
#pragma unroll
        for (int k = 0; k < C; ++k) {
            vn[k] = s_vn[k];
            vo[k] = s_vo[k];
        }
        Acc<C> acc;
        run_pass<C, MK, UNROLL>(a, p, vn, vo, acc, resident, mine);
        ++round;
        constexpr int K = 2 * C + 2;
        const bool two_level = s_xcd != 0;
        const TaggedRows<K> rows{a.rows + (size_t)(round & 1u) * TaggedRows<K>::S * G, round, sy,
                                 (uint64_t)wall_clock64(), a.spin_ticks, two_level};
        write_partial_row<C>(acc, rows);
        if (leader || a.allgather || two_level) {
            // every block of an all-gather or two-level launch reduces the
            // same rows in the same order, so all hold bitwise identical results
            if (two_level) {
                if (!xcd_exchange<C>(rows, G, round, sy, a.spin_ticks, s_r)) return;
            } else if (!reduce_rows<C>(rows, G, a.kahan_only, s_r)) {
                return;
            }
            if (tid == 0) {
                double vcur[C];
#pragma unroll
                for (int k = 0; k < C; ++k) vcur[k] = s_v64[k];
                Step<C> s;
                decide<C>(s_r, p, vcur, a.eps, a.max_iter, s);
                if (leader) commit<C>(a, p, vcur, s);
                if (s.done && a.labels && !a.allgather && !two_level) {
                    // the result in FP64 for the other blocks' label tables,
                    // tagged like the decision (which is stored after it)
#pragma unroll
                    for (int k = 0; k < C; ++k) {
                        const uint64_t bits = __builtin_bit_cast(uint64_t, vcur[k]);
                        store_tagged(sy->fin + 2 * k, round, (uint32_t)bits);
                        store_tagged(sy->fin + 2 * k + 1, round, (uint32_t)(bits >> 32));
                    }
                }
                if (!s.done) {
#pragma unroll
                    for (int k = 0; k < C; ++k) {
                        s_vo[k] = s_vn[k];
                        s_vn[k] = (float)s.vnext[k];
                        s_v64[k] = s.vnext[k];
                    }
                    s_p = p + 1;
                }
                s_done = s.done;
                if (!a.allgather && !two_level) publish_decision<C>(sy, round, s_vn, s_p, s.done);
            }
        } else if (tid == 0) {
            float v[C];
            int pn = 0, done = 0;
            s_ok = await_decision<C>(sy, round, a.spin_ticks, v, pn, done);
            s_done = done;
            if (s_ok && !done) {
#pragma unroll
                for (int k = 0; k < C; ++k) {
                    s_vo[k] = s_vn[k];
                    s_vn[k] = v[k];
                }
                s_p = pn;
            }
            if (s_ok && done && a.labels) {
                uint32_t raw[2 * C];
                s_ok = poll_tagged<2 * C>(sy->fin, round, raw, sy, wall_clock64(), a.spin_ticks);
#pragma unroll
                for (int k = 0; k < C; ++k)
                    s_v64[k] = __builtin_bit_cast(double, (uint64_t)raw[2 * k] | ((uint64_t)raw[2 * k + 1] << 32));
            }
        }
        __syncthreads();
        if (!leader && !a.allgather && !two_level && !s_ok) return;
    }
    if (leader && tid == 0) sy->gen = round;
    if (a.labels && s_done) {
        // v^T is in s_v64 in every block (its own decision, or block 0's)
        __shared__ uint8_t s_lut[256];
        label_table(s_v64, C, s_lut);
        __syncthreads();
        write_labels(a, s_lut, resident, mine);
    }
}

}  // namespace fcm
