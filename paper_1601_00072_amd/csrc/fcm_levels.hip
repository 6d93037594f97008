// Histogram-domain FCM: Algorithm 1 run over the grey levels of an 8-bit
// input instead of its voxels.
//
// Every sum of Eq.1 and Eq.3 over the voxels regroups exactly by grey level,
// sum_i f(x_i) = sum_g h_g f(g), and the memberships of Eq.4 depend on a
// voxel only through its grey level, so the largest membership change of
// Algorithm 1 is the largest change over the levels present.  After one
// histogram pass the whole iteration therefore runs on at most 256 levels
// (the binning idea the paper cites in Sec. 3, made exact here because the
// data are 8-bit).  One block does it: thread g owns grey level g; the
// per-level memberships, the weighted sums, the objective and the change
// are FP64; the sums over the levels use fixed-order wave reductions.  The
// history and the state are written in the same layout as the per-voxel
// drivers, so results, trajectories and labels read the same way.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fcm.h"
#include "fcm_device.h"
#include "fcm_internal.h"

namespace fcm {

namespace {

// Eq.4 at grey level g for centroids v, in the normalised form
// u_k = w_k / sum_j w_j with w_k = (d_min / d_k)^(2/(m-1)) <= 1, and the
// zero-distance rule (equal split over the clusters at distance 0).
template <int C>
__device__ __forceinline__ void level_memberships(double g, const double (&v)[C], double m, double (&u)[C]) {
    double d[C];
    double dmin = 1.0e308;
    int nz = 0;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        d[k] = fabs(g - v[k]);
        dmin = fmin(dmin, d[k]);
        nz += d[k] == 0.0;
    }
    if (nz) {
#pragma unroll
        for (int k = 0; k < C; ++k) u[k] = d[k] == 0.0 ? 1.0 / nz : 0.0;
        return;
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const double r = dmin / d[k];
        u[k] = m == 2.0 ? r * r : pow(r, 2.0 / (m - 1.0));
        s += u[k];
    }
#pragma unroll
    for (int k = 0; k < C; ++k) u[k] /= s;
}

__device__ __forceinline__ double wave_max_f64(double v) {
    v = fmax(v, dpp_mov_f64<0xB1>(v));
    v = fmax(v, dpp_mov_f64<0x4E>(v));
    v = fmax(v, dpp_mov_f64<0x141>(v));
    v = fmax(v, dpp_mov_f64<0x140>(v));
    return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}

template <int C>
__global__ __launch_bounds__(256) void fcm_levels_kernel(LevelArgs a) {
    constexpr int NQ = 2 * C + 1;
    const int g = threadIdx.x, lane = g & 63, wid = g >> 6;
    DevState* st = a.st;
    const uint32_t cnt = a.counts[g];
    const double c = (double)cnt, x = (double)g;
    __shared__ double s_v[C], s_vp[C];
    __shared__ double s_sum[4][NQ + 1];
    __shared__ int s_p, s_done;
    if (a.do_init) {
        __shared__ uint32_t s_lo[4], s_hi[4];
        uint32_t lo = cnt ? g : 255u, hi = cnt ? g : 0u;
        lo = wave_min_u32(lo);
        hi = wave_max_u32(hi);
        if (lane == 0) {
            s_lo[wid] = lo;
            s_hi[wid] = hi;
        }
        __syncthreads();
        if (g == 0) {
            for (int w = 1; w < 4; ++w) {
                lo = min(lo, s_lo[w]);
                hi = max(hi, s_hi[w]);
            }
            double v[C];
            start_centroids(C, lo, hi, a.given, a.v0, a.dv0, v);
            commit_start(st, a.hist_v, C, lo, hi, v);
            for (int k = 0; k < C; ++k) s_v[k] = v[k];
            s_p = 0;
            s_done = 0;
        }
    } else if (g == 0) {
        s_p = st->pass;
        s_done = st->done;
        for (int k = 0; k < C; ++k) {
            s_v[k] = a.hist_v[(int64_t)s_p * C + k];
            s_vp[k] = s_p > 0 ? a.hist_v[(int64_t)(s_p - 1) * C + k] : s_v[k];
        }
    }
    __syncthreads();
    for (int budget = a.max_passes; budget > 0 && !s_done; --budget) {
        const int p = s_p;
        double v[C], u[C];
#pragma unroll
        for (int k = 0; k < C; ++k) v[k] = s_v[k];
        level_memberships<C>(x, v, a.m, u);
        double dm = 0.0;
        if (p > 0 && cnt) {
            double vp[C], up[C];
#pragma unroll
            for (int k = 0; k < C; ++k) vp[k] = s_vp[k];
            level_memberships<C>(x, vp, a.m, up);
#pragma unroll
            for (int k = 0; k < C; ++k) dm = fmax(dm, fabs(u[k] - up[k]));
        }
        double q[NQ];
        double J = 0.0;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const double w = c * (a.m == 2.0 ? u[k] * u[k] : pow(u[k], a.m));
            q[k] = w * x;                       // sum of u^m x (Eq.3 numerator)
            q[C + k] = w;                       // sum of u^m (Eq.3 denominator)
            J += w * (x - v[k]) * (x - v[k]);   // Eq.1
        }
        q[2 * C] = J;
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            const double r = wave_sum_f64(q[i]);
            if (lane == 0) s_sum[wid][i] = r;
        }
        const double mx = wave_max_f64(dm);
        if (lane == 0) s_sum[wid][NQ] = mx;
        __syncthreads();
        if (g == 0) {
            double r[NQ];
            for (int i = 0; i < NQ; ++i) r[i] = ((s_sum[0][i] + s_sum[1][i]) + s_sum[2][i]) + s_sum[3][i];
            const double delta =
                p > 0 ? fmax(fmax(s_sum[0][NQ], s_sum[1][NQ]), fmax(s_sum[2][NQ], s_sum[3][NQ])) : __builtin_nan("");
            double vnext[C];
            bool bad = false;
            for (int k = 0; k < C; ++k) {
                vnext[k] = r[C + k] > 0.0 ? r[k] / r[C + k] : v[k];
                bad = bad || !isfinite(vnext[k]);
            }
            bad = bad || !isfinite(r[2 * C]);
            int status = FCM_RUNNING, done = 0;
            if (bad) {
                status = FCM_ENUMERIC;
                done = 1;
            } else if (p >= 1 && delta < a.eps) {
                status = FCM_OK;
                done = 1;
            } else if (p >= a.max_iter) {
                status = FCM_NOT_CONVERGED;
                done = 1;
            }
            a.hist_J[p] = r[2 * C];
            a.hist_d[p] = delta;
            for (int k = 0; k < C; ++k) st->vres[k] = v[k];
            st->iters = p;
            st->J = r[2 * C];
            st->delta = delta;
            st->passes = p + 1;
            st->sync.passes_total += 1;
            if (!done) {
                for (int k = 0; k < C; ++k) {
                    a.hist_v[(int64_t)(p + 1) * C + k] = vnext[k];
                    st->v32[(p + 1) & 1][k] = (float)vnext[k];
                    s_vp[k] = v[k];
                    s_v[k] = vnext[k];
                }
                st->pass = p + 1;
                s_p = p + 1;
            }
            st->status = status;
            st->done = done;
            s_done = done;
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_levels(const LevelArgs& a, int C, hipStream_t s) {
    switch (C) {
        case 2: hipLaunchKernelGGL(fcm_levels_kernel<2>, dim3(1), dim3(256), 0, s, a); break;
        case 3: hipLaunchKernelGGL(fcm_levels_kernel<3>, dim3(1), dim3(256), 0, s, a); break;
        case 4: hipLaunchKernelGGL(fcm_levels_kernel<4>, dim3(1), dim3(256), 0, s, a); break;
        case 5: hipLaunchKernelGGL(fcm_levels_kernel<5>, dim3(1), dim3(256), 0, s, a); break;
        case 6: hipLaunchKernelGGL(fcm_levels_kernel<6>, dim3(1), dim3(256), 0, s, a); break;
        case 7: hipLaunchKernelGGL(fcm_levels_kernel<7>, dim3(1), dim3(256), 0, s, a); break;
        case 8: hipLaunchKernelGGL(fcm_levels_kernel<8>, dim3(1), dim3(256), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fcm
