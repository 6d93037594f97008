/* Oracle-F: plain FP64 Fuzzy C-Means over the voxels, threaded over the host
 * cores.  TEST INFRASTRUCTURE ONLY: called by the tests and by the CPU leg of
 * the benchmark, never by the product path; shares nothing with the HIP
 * library.
 *
 * It computes Algorithm 1 with the centroid-first start, exactly as the
 * literal oracle (fcm_ref.py) does, in the w / sum w form of Eq.4:
 *   u_k = w_k / sum_j w_j,  w_k = (d_min / d_k)^(2/(m-1)),  d_k = |x - v_k|
 * (the same ratio as the printed double sum, scaled by d_min so that every
 * w_k <= 1); a voxel at distance 0 from some centroids splits its membership
 * equally over them.  Per iteration t >= 1:
 *   v^t     = sum_i (u_i^(t-1))^m x_i / sum_i (u_i^(t-1))^m          (Eq.3)
 *             (a centroid with a zero denominator keeps its value)
 *   U^t     = Eq.4 at v^t
 *   delta^t = max_ik |u_ik^t - u_ik^(t-1)|;  stop with T = t once delta^t < eps
 *   J^t     = sum_i sum_k (u_ik^t)^m (x_i - v_k^t)^2                  (Eq.1)
 * U is not stored: a voxel's memberships at v^(t-1) are evaluated again from
 * v^(t-1) when they are needed, which gives the same numbers.  The voxels are
 * cut into one contiguous static chunk per thread, each thread sums its chunk
 * in index order, and the chunk sums are added in thread order. */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <omp.h>

#define MAXC 8

static void memberships(double x, const double* v, int C, double m, double* u) {
    double d[MAXC], dmin = INFINITY;
    int zeros = 0;
    for (int k = 0; k < C; ++k) {
        d[k] = fabs(x - v[k]);
        if (d[k] < dmin) dmin = d[k];
        zeros += d[k] == 0.0;
    }
    if (zeros) {
        for (int k = 0; k < C; ++k) u[k] = d[k] == 0.0 ? 1.0 / zeros : 0.0;
        return;
    }
    const double e = 2.0 / (m - 1.0);
    double s = 0.0;
    for (int k = 0; k < C; ++k) {
        u[k] = pow(dmin / d[k], e);
        s += u[k];
    }
    for (int k = 0; k < C; ++k) u[k] /= s;
}

/* One sweep over the voxels: memberships at v_cur (U^t), and at v_prev
 * (U^(t-1)) when v_prev is given.  Outputs: the Eq.3 sums of U^t (num, den),
 * J at (U^t, v_cur), and max |U^t - U^(t-1)|. */
static void sweep(const uint8_t* x, int64_t n, int C, double m, const double* v_prev, const double* v_cur,
                  int threads, double* num, double* den, double* J, double* delta) {
    double* part = (double*)calloc((size_t)threads * (2 * MAXC + 2), sizeof(double));
#pragma omp parallel num_threads(threads)
    {
        const int p = omp_get_thread_num(), P = omp_get_num_threads();
        const int64_t i0 = n * p / P, i1 = n * (p + 1) / P;
        double* mine = part + (size_t)p * (2 * MAXC + 2);
        double u[MAXC], uo[MAXC];
        for (int64_t i = i0; i < i1; ++i) {
            const double xi = (double)x[i];
            memberships(xi, v_cur, C, m, u);
            if (v_prev) {
                memberships(xi, v_prev, C, m, uo);
                for (int k = 0; k < C; ++k) {
                    const double dd = fabs(u[k] - uo[k]);
                    if (dd > mine[2 * MAXC + 1]) mine[2 * MAXC + 1] = dd;
                }
            }
            for (int k = 0; k < C; ++k) {
                const double a = pow(u[k], m);
                mine[k] += a * xi;
                mine[MAXC + k] += a;
                mine[2 * MAXC] += a * (xi - v_cur[k]) * (xi - v_cur[k]);
            }
        }
    }
    for (int k = 0; k < C; ++k) num[k] = den[k] = 0.0;
    *J = 0.0;
    *delta = 0.0;
    for (int p = 0; p < threads; ++p) {
        const double* q = part + (size_t)p * (2 * MAXC + 2);
        for (int k = 0; k < C; ++k) {
            num[k] += q[k];
            den[k] += q[MAXC + k];
        }
        *J += q[2 * MAXC];
        if (q[2 * MAXC + 1] > *delta) *delta = q[2 * MAXC + 1];
    }
    free(part);
}

/* v0: C start centroids.  Histories (caller-owned, max_iter + 1 entries):
 * v_hist[t * C + k], d_hist[t] (d_hist[0] = NaN), J_hist[t].  Returns T;
 * *status = 0 (converged) or 1 (max_iter reached).  threads < 1 = all. */
int oracle_f_solve(const uint8_t* x, int64_t n, int C, double m, double eps, int max_iter, const double* v0,
                   int threads, double* v_hist, double* d_hist, double* J_hist, int* status) {
    if (C < 1 || C > MAXC || n < 1 || max_iter < 1) return -1;
    if (threads < 1) threads = omp_get_max_threads();
    double v[MAXC], vp[MAXC], num[MAXC], den[MAXC], J, delta;
    memcpy(v, v0, sizeof(double) * C);
    sweep(x, n, C, m, NULL, v, threads, num, den, &J, &delta);
    memcpy(v_hist, v, sizeof(double) * C);
    d_hist[0] = NAN;
    J_hist[0] = J;
    *status = 1;
    int T = max_iter;
    for (int t = 1; t <= max_iter; ++t) {
        memcpy(vp, v, sizeof(double) * C);
        for (int k = 0; k < C; ++k)
            if (den[k] > 0.0) v[k] = num[k] / den[k];
        sweep(x, n, C, m, vp, v, threads, num, den, &J, &delta);
        memcpy(v_hist + (size_t)t * C, v, sizeof(double) * C);
        d_hist[t] = delta;
        J_hist[t] = J;
        if (delta < eps) {
            T = t;
            *status = 0;
            break;
        }
    }
    return T;
}
