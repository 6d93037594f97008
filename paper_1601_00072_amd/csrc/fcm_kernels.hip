// gfx950 kernels of the Fuzzy C-Means iteration (Sec. 2.1, Sec. 4 of the paper).
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
//   LDS step into one partial row.  The last block to arrive (atomic ticket)
//   reduces all rows in a fixed order in FP64 -- or compensated FP32 --
//   forms v^(p+1) (Eq.3), records delta^p and J^p, and applies the stopping
//   rule of Algorithm 1 on the device.
//
// Membership form for m = 2 (exact algebra of Eq.4): with q_k = (x - v_k)^2,
// u_k = P_k / sum_j P_j where P_k = prod_{j != k} q_j, so one reciprocal
// serves all C memberships; u_k q_k is the same for every k and equals the
// voxel's objective term sum_k u_k^2 q_k.  For other m:
// u_k = w_k / sum_j w_j with w_k = 2^(alpha (L_min - L_k)), L_k = log2 q_k,
// alpha = 1/(m-1), which keeps every weight in (0, 1].
//
// Zero distances are exact: q_k = (x - v_k)^2 with no floor, so a voxel on a
// centroid gets membership exactly 1 there and exactly 0 elsewhere, and a
// cluster with no support keeps a zero denominator, as in the oracle.  The
// product form runs only when every centroid of both sets lies in [0, 255]
// with pairwise gaps >= 2^-6: then at most one q_k of a voxel is below 2^-14
// and every leave-one-out product lies in [2^-98, 2^112], inside the normal
// FP32 range.  Otherwise (coinciding or out-of-range centroids, a uniform
// per-pass decision) the pass uses the normalised form with L_k clamped to
// [-1000, 256], which gives exact zeros and the equal split over coinciding
// centroids without overflow.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fcm.h"
#include "fcm_internal.h"

namespace fcm {

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

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
    return v;
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
// objective term sum_j a_j q_j (Eq.1).
// Since u_k is proportional to q_k^(-alpha) = (q_k^-1)^alpha, every m follows
// from the m = 2 memberships u2: u_k = u2_k^alpha / sum_j u2_j^alpha.  Working
// from u2 (in [0, 1], dominant entries >= 1/C) keeps log2/exp2 arguments small.
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

// ---------------------------------------------------------------------------
// final reduction of a pass (last block): Eq.3 update and the stopping rule
// ---------------------------------------------------------------------------

template <int C>
__device__ void finish_pass(const PassArgs& a, int p) {
    constexpr int NQ = 2 * C + 1;   // num[C], den[C], J
    constexpr int R = partial_rows(C);
    constexpr int W = kBlock / 64;
    __shared__ double s_sum[W][NQ];
    __shared__ float s_lo[W][NQ];
    __shared__ float s_max[W];
    const int G = gridDim.x;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const float* P = a.partials;
    float dm = 0.f;
    double res[NQ];

    if (!a.kahan_only) {
        // FP64 over the block partials, each taken as (sum - comp)
        double acc[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
        for (int b = tid; b < G; b += kBlock) {
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                acc[q] += (double)load_coherent(P + (2 * q) * G + b) - (double)load_coherent(P + (2 * q + 1) * G + b);
            dm = fmaxf(dm, load_coherent(P + (R - 1) * G + b));
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const double s = wave_sum_f64(acc[q]);
            if (lane == 0) s_sum[wid][q] = s;
        }
        const float m = wave_max(dm);
        if (lane == 0) s_max[wid] = m;
        __syncthreads();
        if (tid != 0) return;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double s = s_sum[0][q];
            for (int w = 1; w < W; ++w) s += s_sum[w][q];
            res[q] = s;
        }
    } else {
        // compensated FP32 throughout: (hi, lo) pairs combined error-free
        float hi[NQ], lo[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) hi[q] = lo[q] = 0.f;
        for (int b = tid; b < G; b += kBlock) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const float v = load_coherent(P + (2 * q) * G + b);
                const float c = load_coherent(P + (2 * q + 1) * G + b);
                float s, e;
                two_sum(hi[q], v, s, e);
                hi[q] = s;
                lo[q] += e - c;
            }
            dm = fmaxf(dm, load_coherent(P + (R - 1) * G + b));
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            for (int off = 1; off < 64; off <<= 1) {
                const float oh = __shfl_xor(hi[q], off, 64);
                const float ol = __shfl_xor(lo[q], off, 64);
                float s, e;
                // order the operands so both lanes of a pair compute the same bits
                const bool low = (lane & off) == 0;
                two_sum(low ? hi[q] : oh, low ? oh : hi[q], s, e);
                lo[q] = (low ? lo[q] + ol : ol + lo[q]) + e;
                hi[q] = s;
            }
            if (lane == 0) {
                s_sum[wid][q] = (double)hi[q];
                s_lo[wid][q] = lo[q];
            }
        }
        const float m = wave_max(dm);
        if (lane == 0) s_max[wid] = m;
        __syncthreads();
        if (tid != 0) return;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            float h = (float)s_sum[0][q], l = s_lo[0][q];
            for (int w = 1; w < W; ++w) {
                float s, e;
                two_sum(h, (float)s_sum[w][q], s, e);
                h = s;
                l += e + s_lo[w][q];
            }
            res[q] = (double)(h + l);
        }
    }
    // ---- thread 0 only from here ----
    dm = s_max[0];
    for (int w = 1; w < W; ++w) dm = fmaxf(dm, s_max[w]);

    DevState* st = a.st;
    bool bad = false;
    double vnext[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const double vk = a.hist_v[(int64_t)p * C + k];
        const double num = res[k], den = res[C + k];
        vnext[k] = den > 0.0 ? num / den : vk;
        if (!isfinite(vnext[k])) bad = true;
        st->vres[k] = vk;
    }
    const double J = res[2 * C];
    if (!isfinite(J)) bad = true;
    const double delta = p > 0 ? (double)dm : __builtin_nan("");
    a.hist_J[p] = J;
    a.hist_d[p] = delta;
    st->iters = p;
    st->J = J;
    st->delta = delta;
    st->passes = p + 1;
    int status = FCM_RUNNING;
    int done = 0;
    if (bad) {
        status = FCM_ENUMERIC;
        done = 1;
    } else if (p >= 1 && delta < a.eps) {
        status = FCM_OK;
        done = 1;
    } else if (p >= a.max_iter) {
        status = FCM_NOT_CONVERGED;
        done = 1;
    } else {
#pragma unroll
        for (int k = 0; k < C; ++k) {
            a.hist_v[(int64_t)(p + 1) * C + k] = vnext[k];
            st->v32[(p + 1) & 1][k] = (float)vnext[k];
        }
        st->pass = p + 1;
    }
    st->status = status;
    st->ticket = 0;
    st->done = done;
}

// ---------------------------------------------------------------------------
// the fused pass
// ---------------------------------------------------------------------------
// Range and separation test of a centroid set for the product form (uniform).
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


template <int C, int FORM, int UNROLL, bool OLD>
__device__ __forceinline__ void pass_body(const PassArgs& a, const float (&vn)[C], const float (&vo)[C],
                                          const Consts& kc, Acc<C>& acc) {
    const int tid = threadIdx.x;
    const uint4* body = reinterpret_cast<const uint4*>(a.x + a.head);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    int64_t c = (int64_t)blockIdx.x * kBlock + tid;
    const int64_t nb = a.nbody;
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    if constexpr (UNROLL == 1) {
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
    acc.zero();
    constexpr int FAST = MK == kM2 ? kProdM2 : (MK == kM15 ? kProdM15 : kProdPow);
    const Consts kc{a.alpha, a.mexp};
    if (separated<C>(vn) && (p == 0 || separated<C>(vo))) {
        if (p == 0)
            pass_body<C, FAST, UNROLL, false>(a, vn, vo, kc, acc);
        else
            pass_body<C, FAST, UNROLL, true>(a, vn, vo, kc, acc);
    } else {
        if (p == 0)
            pass_body<C, kNormLog, UNROLL, false>(a, vn, vo, kc, acc);
        else
            pass_body<C, kNormLog, UNROLL, true>(a, vn, vo, kc, acc);
    }

    // block reduction: wave butterflies, then waves in order with Kahan
    constexpr int NQ = 2 * C + 1;
    constexpr int W = kBlock / 64;
    __shared__ float s_red[W][NQ + 1];
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
    const int G = gridDim.x;
    if (tid < NQ) {
        float s = 0.f, c = 0.f;
        for (int w = 0; w < W; ++w) kahan_add(s, c, s_red[w][tid]);
        store_coherent(a.partials + (2 * tid) * G + blockIdx.x, s);
        store_coherent(a.partials + (2 * tid + 1) * G + blockIdx.x, c);
    } else if (tid == NQ) {
        float mm = s_red[0][NQ];
        for (int w = 1; w < W; ++w) mm = fmaxf(mm, s_red[w][NQ]);
        store_coherent(a.partials + (2 * NQ) * G + blockIdx.x, mm);
    }
    if (!arrive_last(&st->ticket)) return;
    finish_pass<C>(a, p);
}

// ---------------------------------------------------------------------------
// data range and initial centroids
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void fcm_init_kernel(InitArgs a) {
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    uint32_t lo = 255u, hi = 0u;
    const uint4* body = reinterpret_cast<const uint4*>(a.x + a.head);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + tid; c < a.nbody; c += stride) {
        const uint4 w = body[c];
        const uint32_t words[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const uint32_t v = (words[i] >> (8 * b)) & 0xFFu;
                lo = min(lo, v);
                hi = max(hi, v);
            }
        }
    }
    if (blockIdx.x == 0) {
        const int64_t tail0 = a.head + 16 * a.nbody;
        const int64_t nr = a.head + (a.n - tail0);
        if (tid < nr) {
            const int64_t i = tid < a.head ? (int64_t)tid : tail0 + (tid - a.head);
            lo = min(lo, (uint32_t)a.x[i]);
            hi = max(hi, (uint32_t)a.x[i]);
        }
    }
    __shared__ uint32_t s_lo[kBlock / 64], s_hi[kBlock / 64];
    lo = wave_min_u32(lo);
    hi = wave_max_u32(hi);
    if (lane == 0) {
        s_lo[wid] = lo;
        s_hi[wid] = hi;
    }
    __syncthreads();
    const int G = gridDim.x;
    if (tid == 0) {
        for (int w = 1; w < kBlock / 64; ++w) {
            lo = min(lo, s_lo[w]);
            hi = max(hi, s_hi[w]);
        }
        store_coherent(a.partials + blockIdx.x, lo);
        store_coherent(a.partials + G + blockIdx.x, hi);
    }
    if (!arrive_last(&a.st->ticket)) return;
    if (tid != 0) return;
    lo = 255u;
    hi = 0u;
    for (int b = 0; b < G; ++b) {
        lo = min(lo, load_coherent(a.partials + b));
        hi = max(hi, load_coherent(a.partials + G + b));
    }
    DevState* st = a.st;
    const int C = a.C;
    for (int k = 0; k < kMaxC; ++k) {
        float v32 = 0.f;
        if (k < C) {
            if (a.given) {
                v32 = (float)a.v0[k];
            } else {
                // lo + k (hi - lo) / (C - 1): the product is exact, the quotient and
                // the sum are rounded once each in FP64, then rounded to FP32
                const double v = (double)lo + (double)(k * (int)(hi - lo)) / (double)(C - 1);
                v32 = (float)v;
            }
            a.hist_v[k] = (double)v32;
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
    st->ticket = 0;
    st->done = 0;
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

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_init(const InitArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(fcm_init_kernel, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_labels(const LabelArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(fcm_labels_kernel, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

using PassFn = void (*)(PassArgs);

template <int C, int MK>
static PassFn pick_u(int unroll) {
    return unroll == 2 ? fcm_pass_kernel<C, MK, 2> : fcm_pass_kernel<C, MK, 1>;
}

template <int C>
static PassFn pick_c(int mclass, int unroll) {
    if (mclass == kM2) return pick_u<C, kM2>(unroll);
    if (mclass == kM15) return pick_u<C, kM15>(unroll);
    return pick_u<C, kMGeneric>(unroll);
}

static PassFn pick(int C, int mclass, int unroll) {
    if ((mclass != kM2 && mclass != kM15 && mclass != kMGeneric) || (unroll != 1 && unroll != 2)) return nullptr;
    switch (C) {
        case 2: return pick_c<2>(mclass, unroll);
        case 3: return pick_c<3>(mclass, unroll);
        case 4: return pick_c<4>(mclass, unroll);
        case 5: return pick_c<5>(mclass, unroll);
        case 6: return pick_c<6>(mclass, unroll);
        case 7: return pick_c<7>(mclass, unroll);
        case 8: return pick_c<8>(mclass, unroll);
        default: return nullptr;
    }
}

bool pass_supported(int C, int mclass, int unroll) { return pick(C, mclass, unroll) != nullptr; }

hipError_t launch_pass(const PassArgs& a, int C, int mclass, int unroll, int grid, hipStream_t s) {
    PassFn f = pick(C, mclass, unroll);
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace fcm
