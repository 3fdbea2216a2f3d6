// NCG vector layer of Algorithm 2 on the flat unknown x of Eq. (5): the step
// x + alpha p, the preconditioned direction with beta of Eq. (8), the
// backtracking line search of Algorithm 4 on the quartic coefficients, and
// the fixed-order FP64 reductions everything else uses.  These are streaming
// (HBM-bound) kernels: grid-stride loops over the vectors, FP64 dots reduced
// per block into one partial each, partials summed by one workgroup in a
// fixed order.
#include <math.h>

#include "internal.h"

namespace alsncg {
namespace {

constexpr int kVecThreads = 256;
constexpr int kVecBlocks = 2048;  // fixed: the reduction order must not depend on n

// ---------------------------------------------------------------- reductions

constexpr int kSumBlocks = 256;
constexpr int kSumThreads = 256;
constexpr int kMaxCols = 8;

// Stage 1: block k sums rows [k R / B, (k + 1) R / B) of every column into
// stage[k * cols + c]; stage 2 (one block) sums the B partials.  The split of
// the rows depends only on R, so the result is the same on every run.
__global__ __launch_bounds__(kSumThreads) void sum_columns_stage1(const double *__restrict__ parts,
                                                                  int64_t rows, int cols,
                                                                  double *__restrict__ stage) {
    __shared__ double red[kMaxCols][kSumThreads];
    const int64_t r0 = rows * blockIdx.x / gridDim.x, r1 = rows * (blockIdx.x + 1) / gridDim.x;
    double acc[kMaxCols];
#pragma unroll
    for (int k = 0; k < kMaxCols; ++k) acc[k] = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kSumThreads)
#pragma unroll
        for (int k = 0; k < kMaxCols; ++k)
            if (k < cols) acc[k] += parts[r * cols + k];
#pragma unroll
    for (int k = 0; k < kMaxCols; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = kSumThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < kMaxCols; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if ((int)threadIdx.x < cols) stage[(int64_t)blockIdx.x * cols + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(kSumThreads) void sum_columns_stage2(const double *__restrict__ stage,
                                                                  int nblocks, int cols,
                                                                  double *__restrict__ out,
                                                                  int accumulate) {
    __shared__ double red[kMaxCols][kSumThreads];
#pragma unroll
    for (int k = 0; k < kMaxCols; ++k)
        red[k][threadIdx.x] = (k < cols && (int)threadIdx.x < nblocks) ? stage[threadIdx.x * cols + k] : 0.0;
    __syncthreads();
    for (int w = kSumThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < kMaxCols; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if ((int)threadIdx.x < cols)
        out[threadIdx.x] = accumulate ? out[threadIdx.x] + red[threadIdx.x][0] : red[threadIdx.x][0];
}

template <int NV>
__device__ inline void block_sum_store(double (&v)[NV], double *dst) {
    __shared__ double red[NV][kVecThreads / kWave];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        v[k] = sum64(v[k]);
        if (lane == 0) red[k][wv] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < kVecThreads / kWave; ++w) s += red[k][w];
            dst[k] = s;
        }
    }
}

// ---------------------------------------------------------------- axpy

template <typename T>
__global__ __launch_bounds__(kVecThreads) void axpy_kernel(int64_t n, T *__restrict__ x,
                                                           const T *__restrict__ p,
                                                           const double *__restrict__ alpha) {
    const double a = *alpha;
    for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kVecThreads)
        x[i] = (T)((double)x[i] + a * (double)p[i]);
}

template <typename T>
__global__ __launch_bounds__(kVecThreads) void axpby_kernel(int64_t n, double a,
                                                            const T *__restrict__ x, double b,
                                                            T *__restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kVecThreads) {
        const double yv = b != 0.0 ? b * (double)y[i] : 0.0;
        y[i] = (T)(a * (double)x[i] + yv);
    }
}

// ---------------------------------------------------------------- direction

// gbar = x - xbar (stored over xbar); partial sums of
//   [gbar.(g_new - g_old), gbar.g_new, g_new.g_new].
template <typename T>
__global__ __launch_bounds__(kVecThreads) void direction_dots_kernel(
    int64_t n, const T *__restrict__ x, T *__restrict__ xbar, const T *__restrict__ gn,
    const T *__restrict__ go, double *__restrict__ part) {
    double v[3] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kVecThreads) {
        const T gb = x[i] - xbar[i];
        xbar[i] = gb;
        const double g1 = (double)gn[i];
        const double g0 = go ? (double)go[i] : 0.0;
        v[0] += (double)gb * (g1 - g0);
        v[1] += (double)gb * g1;
        v[2] += g1 * g1;
    }
    block_sum_store<3>(v, part + 3 * (int64_t)blockIdx.x);
}

// scal[0] = den (in: gbar_k.g_k, out: gbar_{k+1}.g_{k+1}); scal[1] = beta;
// scal[2] = ||g||^2; scal[3] = numerator of Eq. (8).
__global__ void direction_beta_kernel(const double *__restrict__ sums, double *__restrict__ scal,
                                      int restart, const double *__restrict__ restart_dev,
                                      int pr_plus) {
    const double num = sums[0], den_new = sums[1], gg = sums[2];
    const double den = scal[0];
    if (restart_dev && *restart_dev != 0.0) restart = 1;
    double beta = 0.0;
    if (!restart && den != 0.0 && isfinite(den)) beta = num / den;
    if (!isfinite(beta)) beta = 0.0;
    if (pr_plus && beta < 0.0) beta = 0.0;
    scal[0] = den_new;
    scal[1] = beta;
    scal[2] = gg;
    scal[3] = num;
}

template <typename T>
__global__ __launch_bounds__(kVecThreads) void direction_update_kernel(
    int64_t n, const T *__restrict__ gbar, T *__restrict__ p, const double *__restrict__ scal) {
    const double beta = scal[1];
    for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kVecThreads)
        p[i] = (T)(beta * (double)p[i] - (double)gbar[i]);
}

// ---------------------------------------------------------------- backtracking

// First alpha = alpha0 tau^n (n < max_trials) passing the divided Armijo
// test; alpha = 0, n = -1 when none passes or C1 >= 0.
__device__ void backtrack_search(const double *C, double alpha0, double tau, double c,
                                 int max_trials, double *alpha_out, int *n_out) {
    // no FMA contraction: the accept/reject decision must be taken with the
    // same roundings as a plain evaluation of the test
#pragma clang fp contract(off)
    const double c1 = C[1], c2 = C[2], c3 = C[3], c4 = C[4];
    double alpha = alpha0, acc = 0.0;
    int n = -1;
    if (c1 < 0.0) {
        for (int t = 0; t < max_trials; ++t) {
            const double test = (1.0 - c) * c1 + alpha * (c2 + alpha * (c3 + alpha * c4));
            if (test <= 0.0) {
                n = t;
                acc = alpha;
                break;
            }
            alpha = tau * alpha;
        }
    }
    *alpha_out = acc;
    *n_out = n;
}

// Exact line search on the same quartic: the global minimiser over alpha > 0
// of Q(alpha) = sum C[n] alpha^n.  The real roots of Q'(alpha) = C1 + 2 C2 a
// + 3 C3 a^2 + 4 C4 a^3 on (0, B] (B a Cauchy bound) are bracketed between
// the roots of Q'' and found by bisection to full precision; the root with
// the smallest Q is kept if it passes the divided Armijo test.  alpha = 0,
// n = -1 when C1 >= 0, when Q has no minimiser on alpha > 0, or when the test
// fails; else n = 0.
__device__ void quartic_min_search(const double *C, double c, double *alpha_out, int *n_out) {
#pragma clang fp contract(off)
    const double c1 = C[1], c2 = C[2], c3 = C[3], c4 = C[4];
    *alpha_out = 0.0;
    *n_out = -1;
    if (!(c1 < 0.0)) return;
    // Q'(a) = d0 + d1 a + d2 a^2 + d3 a^3
    const double d0 = c1, d1 = 2.0 * c2, d2 = 3.0 * c3, d3 = 4.0 * c4;
    double lead;
    int deg;
    if (d3 != 0.0) {
        deg = 3;
        lead = d3;
    } else if (d2 != 0.0) {
        deg = 2;
        lead = d2;
    } else if (d1 != 0.0) {
        deg = 1;
        lead = d1;
    } else {
        return;  // Q' = C1 < 0 everywhere: no minimiser
    }
    if (!(lead > 0.0)) return;  // Q' -> -inf: Q unbounded below along p
    const double B = 1.0 + fmax(fabs(d0 / lead), fmax(fabs(d1 / lead), fabs(d2 / lead)));
    auto dq = [&](double a) { return d0 + a * (d1 + a * (d2 + a * d3)); };
    auto q = [&](double a) { return C[0] + a * (c1 + a * (c2 + a * (c3 + a * c4))); };
    // breakpoints: positive roots of Q''(a) = d1 + 2 d2 a + 3 d3 a^2 below B
    double bp[4];
    int nb = 0;
    bp[nb++] = 0.0;
    if (deg == 3) {
        const double A2 = 3.0 * d3, A1 = 2.0 * d2, A0 = d1;
        const double disc = A1 * A1 - 4.0 * A2 * A0;
        if (disc >= 0.0) {
            const double sq = sqrt(disc);
            double r0 = (-A1 - sq) / (2.0 * A2), r1 = (-A1 + sq) / (2.0 * A2);
            if (r0 > r1) { const double t = r0; r0 = r1; r1 = t; }
            if (r0 > 0.0 && r0 < B) bp[nb++] = r0;
            if (r1 > 0.0 && r1 < B) bp[nb++] = r1;
        }
    } else if (deg == 2) {
        const double r = -d1 / (2.0 * d2);
        if (r > 0.0 && r < B) bp[nb++] = r;
    }
    bp[nb++] = B;
    double best = 0.0, qbest = 0.0;
    bool found = false;
    for (int k = 0; k + 1 < nb; ++k) {
        double lo = bp[k], hi = bp[k + 1];
        const double flo = dq(lo), fhi = dq(hi);
        if (!(flo < 0.0 && fhi >= 0.0)) continue;  // a minimum of Q lies where Q' crosses upward
        for (int it = 0; it < 200 && hi - lo > 0.0; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            if (dq(mid) < 0.0) lo = mid; else hi = mid;
        }
        const double a = hi;
        const double qa = q(a);
        if (!found || qa < qbest) {
            best = a;
            qbest = qa;
            found = true;
        }
    }
    if (!found) return;
    const double test = (1.0 - c) * c1 + best * (c2 + best * (c3 + best * c4));
    if (test <= 0.0) {
        *alpha_out = best;
        *n_out = 0;
    }
}

// Q(alpha) = f(x + alpha p) by Horner from the highest coefficient, no
// contraction (the same roundings as a plain evaluation on the host).
__device__ double quartic_value(const double *C, double alpha) {
#pragma clang fp contract(off)
    return (((C[4] * alpha + C[3]) * alpha + C[2]) * alpha + C[1]) * alpha + C[0];
}

__global__ void quartic_min_kernel(const double *__restrict__ C, double c,
                                   double *__restrict__ alpha_out, int32_t *__restrict__ trials_out,
                                   double *__restrict__ q_out) {
    double a;
    int n;
    quartic_min_search(C, c, &a, &n);
    *alpha_out = a;
    if (trials_out) *trials_out = n;
    if (q_out) *q_out = n < 0 ? NAN : quartic_value(C, a);
}

__global__ void backtrack_kernel(const double *__restrict__ C, double alpha0, double tau, double c,
                                 int max_trials, double *__restrict__ alpha_out,
                                 int32_t *__restrict__ trials_out, double *__restrict__ q_out) {
    double a;
    int n;
    backtrack_search(C, alpha0, tau, c, max_trials, &a, &n);
    *alpha_out = a;
    if (trials_out) *trials_out = n;
    if (q_out) *q_out = n < 0 ? NAN : quartic_value(C, a);
}

// ---------------------------------------------------------------- device-side step control
//
// state (double[32]): [0..4] C of the first direction, [5] its alpha, [6] its
// trial count, [7] restart flag; [8..12], [13], [14] the same for the restarted
// direction -gbar; [16..20] accepted C, [21] step applied (alpha, or 1 for the
// ALS point), [22] trials (-1: safeguard), [23] restarted, [24] safeguarded,
// [25] f(x_{k+1}) = Q(alpha) (NaN after a safeguard step), [26] total
// restarts, [27] total safeguards, [28] iterations.

__device__ void line_search(int exact, const double *C, double alpha0, double tau, double c,
                            int max_trials, double *a, int *n) {
    if (exact)
        quartic_min_search(C, c, a, n);
    else
        backtrack_search(C, alpha0, tau, c, max_trials, a, n);
}

__global__ void ls_first_kernel(double *__restrict__ st, int exact, double alpha0, double tau,
                                double c, int max_trials) {
    double a;
    int n;
    line_search(exact, st, alpha0, tau, c, max_trials, &a, &n);
    st[5] = a;
    st[6] = (double)n;
    st[7] = (st[1] >= 0.0 || n < 0) ? 1.0 : 0.0;
}

template <typename T>
__global__ __launch_bounds__(kVecThreads) void ls_restart_dir_kernel(int64_t n, T *__restrict__ p,
                                                                     const T *__restrict__ gbar,
                                                                     const double *__restrict__ st) {
    if (st[7] == 0.0) return;
    for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kVecThreads)
        p[i] = (T)(-(double)gbar[i]);
}

__global__ void ls_final_kernel(double *__restrict__ st, int exact, double alpha0, double tau,
                                double c, int max_trials) {
#pragma clang fp contract(off)
    const bool restarted = st[7] != 0.0;
    const double *C = st;
    double alpha = st[5];
    int n = (int)st[6];
    bool safe = false;
    if (restarted) {
        line_search(exact, st + 8, alpha0, tau, c, max_trials, &alpha, &n);
        st[13] = alpha;
        st[14] = (double)n;
        C = st + 8;
        safe = C[1] >= 0.0 || n < 0;
    }
    for (int k = 0; k < 5; ++k) st[16 + k] = C[k];
    st[21] = safe ? 1.0 : alpha;
    st[22] = safe ? -1.0 : (double)n;
    st[23] = restarted ? 1.0 : 0.0;
    st[24] = safe ? 1.0 : 0.0;
    st[25] = safe ? NAN : quartic_value(C, alpha);
    st[26] += restarted ? 1.0 : 0.0;
    st[27] += safe ? 1.0 : 0.0;
    st[28] += 1.0;
}

}  // namespace

void launch_sum_columns(const double *parts, int64_t rows, int cols, double *out, int accumulate,
                        double *stage, hipStream_t s) {
    hipLaunchKernelGGL(sum_columns_stage1, dim3(kSumBlocks), dim3(kSumThreads), 0, s, parts, rows,
                       cols, stage);
    hipLaunchKernelGGL(sum_columns_stage2, dim3(1), dim3(kSumThreads), 0, s, stage, kSumBlocks,
                       cols, out, accumulate);
}

int launch_quartic_min(const double *coeffs, double c, double *alpha_out, int32_t *trials_out,
                       double *q_out, hipStream_t s) {
    hipLaunchKernelGGL(quartic_min_kernel, dim3(1), dim3(1), 0, s, coeffs, c, alpha_out, trials_out,
                       q_out);
    return hipGetLastError() == hipSuccess ? ALS_OK : ALS_E_HIP;
}

int launch_backtrack(const double *coeffs, double alpha0, double tau, double c, int max_trials,
                     double *alpha_out, int32_t *trials_out, double *q_out, hipStream_t s) {
    hipLaunchKernelGGL(backtrack_kernel, dim3(1), dim3(1), 0, s, coeffs, alpha0, tau, c,
                       max_trials, alpha_out, trials_out, q_out);
    return hipGetLastError() == hipSuccess ? ALS_OK : ALS_E_HIP;
}

static unsigned vec_grid(int64_t n) {
    const int64_t b = (n + kVecThreads - 1) / kVecThreads;
    return (unsigned)(b < 1 ? 1 : (b > kVecBlocks ? kVecBlocks : b));
}

int launch_axpy(int64_t n, void *x, const void *p, const double *alpha, als_dtype dt,
                hipStream_t s) {
    if (n == 0) return ALS_OK;
    if (dt == ALS_F32)
        hipLaunchKernelGGL(axpy_kernel<float>, dim3(vec_grid(n)), dim3(kVecThreads), 0, s, n,
                           (float *)x, (const float *)p, alpha);
    else if (dt == ALS_F64)
        hipLaunchKernelGGL(axpy_kernel<double>, dim3(vec_grid(n)), dim3(kVecThreads), 0, s, n,
                           (double *)x, (const double *)p, alpha);
    else
        return ALS_E_INVAL;
    return hipGetLastError() == hipSuccess ? ALS_OK : ALS_E_HIP;
}

int launch_axpby(int64_t n, double a, const void *x, double b, void *y, als_dtype dt,
                 hipStream_t s) {
    if (n == 0) return ALS_OK;
    if (dt == ALS_F32)
        hipLaunchKernelGGL(axpby_kernel<float>, dim3(vec_grid(n)), dim3(kVecThreads), 0, s, n, a,
                           (const float *)x, b, (float *)y);
    else if (dt == ALS_F64)
        hipLaunchKernelGGL(axpby_kernel<double>, dim3(vec_grid(n)), dim3(kVecThreads), 0, s, n, a,
                           (const double *)x, b, (double *)y);
    else
        return ALS_E_INVAL;
    return hipGetLastError() == hipSuccess ? ALS_OK : ALS_E_HIP;
}

int launch_ls_first(double *state, int exact, double alpha0, double tau, double c, int max_trials,
                    hipStream_t s) {
    hipLaunchKernelGGL(ls_first_kernel, dim3(1), dim3(1), 0, s, state, exact, alpha0, tau, c,
                       max_trials);
    return hipGetLastError() == hipSuccess ? ALS_OK : ALS_E_HIP;
}

int launch_ls_final(double *state, int exact, double alpha0, double tau, double c, int max_trials,
                    hipStream_t s) {
    hipLaunchKernelGGL(ls_final_kernel, dim3(1), dim3(1), 0, s, state, exact, alpha0, tau, c,
                       max_trials);
    return hipGetLastError() == hipSuccess ? ALS_OK : ALS_E_HIP;
}

int launch_ls_restart_dir(int64_t n, void *p, const void *gbar, const double *state, als_dtype dt,
                          hipStream_t s) {
    if (n == 0) return ALS_OK;
    if (dt == ALS_F32)
        hipLaunchKernelGGL(ls_restart_dir_kernel<float>, dim3(vec_grid(n)), dim3(kVecThreads), 0, s,
                           n, (float *)p, (const float *)gbar, state);
    else if (dt == ALS_F64)
        hipLaunchKernelGGL(ls_restart_dir_kernel<double>, dim3(vec_grid(n)), dim3(kVecThreads), 0, s,
                           n, (double *)p, (const double *)gbar, state);
    else
        return ALS_E_INVAL;
    return hipGetLastError() == hipSuccess ? ALS_OK : ALS_E_HIP;
}

int launch_direction(Ctx *ctx, int64_t n, const void *x, void *xbar, const void *g_new,
                     const void *g_old, void *p, double *scal, int restart,
                     const double *restart_dev, int pr_plus, als_dtype dt, hipStream_t s) {
    int err = ALS_OK;
    double *part = (double *)ctx->workspace(
        (size_t)(kVecBlocks * 3 + 8 + kSumStageDoubles) * sizeof(double), s, &err);
    if (!part) return err;
    double *sums = part + kVecBlocks * 3;
    double *stage = sums + 8;
    // fixed grid so the reduction order is the same for every n
    const unsigned grid = kVecBlocks;
    if (dt == ALS_F32)
        hipLaunchKernelGGL(direction_dots_kernel<float>, dim3(grid), dim3(kVecThreads), 0, s, n,
                           (const float *)x, (float *)xbar, (const float *)g_new,
                           restart ? nullptr : (const float *)g_old, part);
    else if (dt == ALS_F64)
        hipLaunchKernelGGL(direction_dots_kernel<double>, dim3(grid), dim3(kVecThreads), 0, s, n,
                           (const double *)x, (double *)xbar, (const double *)g_new,
                           restart ? nullptr : (const double *)g_old, part);
    else
        return ALS_E_INVAL;
    launch_sum_columns(part, kVecBlocks, 3, sums, 0, stage, s);
    hipLaunchKernelGGL(direction_beta_kernel, dim3(1), dim3(1), 0, s, sums, scal, restart,
                       restart_dev, pr_plus);
    if (dt == ALS_F32)
        hipLaunchKernelGGL(direction_update_kernel<float>, dim3(vec_grid(n)), dim3(kVecThreads), 0,
                           s, n, (const float *)xbar, (float *)p, scal);
    else
        hipLaunchKernelGGL(direction_update_kernel<double>, dim3(vec_grid(n)), dim3(kVecThreads), 0,
                           s, n, (const double *)xbar, (double *)p, scal);
    return hipGetLastError() == hipSuccess ? ALS_OK : ALS_E_HIP;
}

}  // namespace alsncg
