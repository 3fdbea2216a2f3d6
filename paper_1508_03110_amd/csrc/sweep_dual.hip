// Dual-form half-sweep for short rows (Eq. (3)/(4) of the paper).
//
// For a row with n_i ratings the solution of Eq. (3),
//     x_i = (Y_I^T Y_I + lambda n_i I)^{-1} Y_I^T r_i       (n_f x n_f system),
// equals, for lambda > 0, by the push-through identity
//     x_i = Y_I^T (Y_I Y_I^T + lambda n_i I)^{-1} r_i       (n_i x n_i system).
// When n_i is well below n_f the second form needs fewer tiles in the MFMA
// Gram (K = Y_I Y_I^T contracts over the n_f factor columns) and a much
// shorter Cholesky (n_i pivots instead of n_f).  Rows are binned by
// NBD = ceil((n_i + 2) / 16), the number of 16-wide tiles of their system;
// one kernel instance per bin, one wavefront per row.  Rows with a single
// rating take the closed form of the 1 x 1 system instead (sweep_one_kernel,
// four rows per wavefront).
//
// Slots of the dual system: slot a < n_i is the a-th rated row y_a; slot n_i
// holds the right-hand side r (set after the Gram, so the factorisation
// leaves z' = R^{-T} r in that column, as the augmented column of the primal
// kernel does); slot n_i + 1 is the gradient point x_at when the fused
// gradient is requested, so the same MFMAs produce y_a . x_at for every a;
// further slots are zero padding.  The fused gradient is then
//     g_i = 2 sum_a (y_a . x_at - r_a) y_a + 2 lambda n_i x_at.
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "internal.h"
#include "rowsolve.h"

namespace alsncg {
namespace {

template <typename T, int VW> struct DVec {
    typedef T type __attribute__((ext_vector_type(VW)));
};
template <typename T> struct DVec<T, 1> {
    typedef T type;
};

template <typename T, int VW>
__device__ __forceinline__ T delem(const typename DVec<T, VW>::type &v, int e) {
    if constexpr (VW == 1) {
        return v;
    } else {
        return v[e];
    }
}

// Rated rows read per batch in the output loop.
constexpr int kOutBatch = 8;

// Wavefronts per SIMD asked of the compiler: the small systems need few
// registers, so more rows are resident to hide the gathers and the pivot
// chain.
template <typename T, int NBD> struct DualOcc {
    static constexpr int waves = sizeof(T) == 4 ? (NBD <= 3 ? 4 : NBD <= 4 ? 3 : 2)
                                                : (NBD <= 2 ? 2 : 1);
};

// Shared memory of one row: the solve's scratch plus ratings, y_a . x_at and
// the row's item ids in slot order.
template <typename T, int NBD> struct DualShared {
    static constexpr int NP = 16 * NBD;
    static constexpr int solve = Shared<T, NBD>::size;
};

// Load one step of the dual Gram: lane (g, c) reads, for every tile row block
// p, VW consecutive factor columns of slot 16 p + c.  VW = 4: columns
// 16 ls + 4 g .. + 3 (one 16-byte load; n_f % 4 == 0 so a vector is wholly
// in or out); VW = 1: column 4 ls + g.  Out-of-range columns read a clamped
// address inside the row and are zeroed when consumed.
template <typename T, int NBD, int VW>
__device__ __forceinline__ void dual_load(typename DVec<T, VW>::type (&v)[NBD],
                                          const T *const (&src)[NBD], int ls, int n_f, int g) {
    typedef typename DVec<T, VW>::type V;
    const int col = VW == 4 ? 16 * ls + 4 * g : 4 * ls + g;
    const int cc = col < n_f ? col : n_f - VW;
#pragma unroll
    for (int p = 0; p < NBD; ++p) v[p] = *(const V *)(src[p] + cc);
}

template <typename T, int NBD, int VW>
__device__ __forceinline__ void dual_consume(typename Mfma<T>::acc4 (&A)[Tri<NBD>::NT],
                                             const typename DVec<T, VW>::type (&v)[NBD],
                                             const bool (&msk)[NBD], int ls, int n_f, int g) {
    const int col = VW == 4 ? 16 * ls + 4 * g : 4 * ls + g;
    const bool ok = col < n_f;
#pragma unroll
    for (int e = 0; e < VW; ++e) {
        T a[NBD];
#pragma unroll
        for (int p = 0; p < NBD; ++p) a[p] = (ok && msk[p]) ? delem<T, VW>(v[p], e) : T(0);
#pragma unroll
        for (int p = 0; p < NBD; ++p)
#pragma unroll
            for (int q = p; q < NBD; ++q)
                A[Tri<NBD>::id(p, q)] = Mfma<T>::mma(a[p], a[q], A[Tri<NBD>::id(p, q)]);
    }
}

// x = Y_I^T z (z in xs) and, with grow, g = 2 Y_I^T (e - r) + 2 lambda n x_at;
// lane k owns factor columns k + 64 h, h < NH.  The rated rows are read
// again (from L2: the Gram has just read them) in batches of kOutBatch, all
// loads of a batch in flight together (one load per step of the sum would
// wait a full memory latency per rating).
template <typename T, int NH>
__device__ __forceinline__ void dual_output(const T *__restrict__ Y, const int32_t *ish,
                                            const T *xs, const T *esh, const T *rsh, int n,
                                            int n_f, int ld, T reg2, const T *xat, T *xrow,
                                            T *grow, bool bad) {
    const int lane = threadIdx.x & 63;
    T ux[NH], gx[NH];
    int kc[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        ux[h] = T(0);
        gx[h] = T(0);
        kc[h] = min(lane + kWave * h, n_f - 1);
    }
    for (int a0 = 0; a0 < n; a0 += kOutBatch) {
        T y[kOutBatch][NH];
#pragma unroll
        for (int u = 0; u < kOutBatch; ++u) {
            const T *yr = Y + (int64_t)ish[min(a0 + u, n - 1)] * ld;
#pragma unroll
            for (int h = 0; h < NH; ++h) y[u][h] = yr[kc[h]];
        }
#pragma unroll
        for (int u = 0; u < kOutBatch; ++u) {
            const int a = a0 + u;
            const T za = a < n ? xs[a] : T(0);
            const T ea = (grow && a < n) ? esh[a] - rsh[a] : T(0);
#pragma unroll
            for (int h = 0; h < NH; ++h) {
                ux[h] += za * y[u][h];
                gx[h] += ea * y[u][h];
            }
        }
    }
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        const int k = lane + kWave * h;
        if (k < n_f) {
            if (grow) grow[k] = T(2) * gx[h] + reg2 * xat[k];
            xrow[k] = bad ? T(NAN) : ux[h];
        }
    }
}

// f(p, q) for every upper tile p <= q < NB with compile-time p and q, so that
// accumulator tiles are only ever indexed by constants (a run-time index
// would move the whole tile array to scratch memory).
template <int NB, int P = 0, int Q = 0, typename F>
__device__ __forceinline__ void for_tiles(F &&f) {
    if constexpr (P < NB) {
        if constexpr (Q < NB) {
            f(std::integral_constant<int, P>{}, std::integral_constant<int, Q>{});
            for_tiles<NB, P, Q + 1>(f);
        } else {
            for_tiles<NB, P + 1, P + 1>(f);
        }
    }
}

template <typename T, int NBD, int VW>
__global__ __launch_bounds__(64, (DualOcc<T, NBD>::waves)) void sweep_dual_kernel(
    const int32_t *__restrict__ idx, const float *__restrict__ val, const T *__restrict__ Y,
    T *__restrict__ X, int n_f, int ld, T lambda, const int32_t *__restrict__ chunk_row,
    const int64_t *__restrict__ chunk_begin, const int32_t *__restrict__ chunk_len,
    int64_t first, int64_t count, const T *__restrict__ X_at, T *__restrict__ grad_out,
    int64_t *__restrict__ bad_row) {
    typedef Tri<NBD> TR;
    typedef Mfma<T> MF;
    typedef typename MF::acc4 acc4;
    typedef typename DVec<T, VW>::type V;
    constexpr int NP = 16 * NBD;
    __shared__ T sm[Shared<T, NBD>::size];
    __shared__ T rsh[NP];       // r_a (0 past n_i)
    __shared__ T esh[NP];       // y_a . x_at
    __shared__ int32_t ish[NP]; // item ids
    if ((int64_t)blockIdx.x >= count) return;
    const int64_t q = first + blockIdx.x;
    const int lane = threadIdx.x, g = lane >> 4, c = lane & 15;
    const int64_t row = chunk_row[q], b = chunk_begin[q];
    const int n = chunk_len[q];  // 1 <= n <= NP - 2
    const bool want_g = grad_out != nullptr;
    T *xrow = X + row * (int64_t)ld;
    const T *xat = X_at ? X_at + row * (int64_t)ld : xrow;

    for (int k = lane; k < NP; k += kWave) {
        const bool in = k < n;
        rsh[k] = in ? (T)val[b + k] : T(0);
        ish[k] = in ? idx[b + k] : idx[b];
    }
    // row pointers of this lane's slots 16 p + c (masked slots read row idx[b])
    const int32_t id0 = idx[b];
    const T *src[NBD];
    bool msk[NBD];
#pragma unroll
    for (int p = 0; p < NBD; ++p) {
        const int slot = 16 * p + c;
        const bool item = slot < n;
        const bool gp = want_g && slot == n + 1;
        const int32_t j = item ? idx[b + slot] : id0;
        src[p] = gp ? xat : Y + (int64_t)j * ld;
        msk[p] = item || gp;
    }

    // ---- K = [Y_I; x_at] [Y_I; x_at]^T, upper 16x16 tiles, contraction over
    // the n_f factor columns; two register buffers, the next step's loads in
    // flight while the current step's MFMAs run
    acc4 A[TR::NT];
#pragma unroll
    for (int t = 0; t < TR::NT; ++t) A[t] = acc4{T(0), T(0), T(0), T(0)};
    const int nls = (n_f + 4 * VW - 1) / (4 * VW);
    V b0[NBD], b1[NBD];
    dual_load<T, NBD, VW>(b0, src, 0, n_f, g);
    for (int ls = 0; ls < nls; ls += 2) {
        dual_load<T, NBD, VW>(b1, src, min(ls + 1, nls - 1), n_f, g);
        dual_consume<T, NBD, VW>(A, b0, msk, ls, n_f, g);
        dual_load<T, NBD, VW>(b0, src, min(ls + 2, nls - 1), n_f, g);
        if (ls + 1 < nls) dual_consume<T, NBD, VW>(A, b1, msk, ls + 1, n_f, g);
    }
    row_sync<false>();  // rsh, ish visible

    // ---- y_a . x_at out of column n + 1, r into column n
    const int qg = (n + 1) >> 4, cg = (n + 1) & 15;
    const int qr = n >> 4, cr = n & 15;
    for_tiles<NBD>([&](auto P, auto Q) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int a = 16 * P + MF::row(g, r);
            if (want_g && Q == qg && c == cg && a < n) esh[a] = A[TR::id(P, Q)][r];
            if (Q == qr && c == cr && a < n) A[TR::id(P, Q)][r] = rsh[a];
        }
    });
    regularize<T, NBD>(A, lambda * (T)n, n);

    // ---- Cholesky of the n x n block; column n becomes z' with R^T z' = r
    T *xs = sm;
    T *ys = sm + NP;
    T *Dt = sm + 2 * NP;
    T *Yinv = Dt + Shared<T, NBD>::TS;
    const bool bad = cholesky_blocked<T, NBD, false>(A, n, Dt, Yinv);
    for_tiles<NBD>([&](auto P, auto Q) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (Q == qr && c == cr) ys[16 * P + MF::row(g, r)] = A[TR::id(P, Q)][r];
    });
    back_solve<T, NBD, false>(A, n, ys, xs, Yinv);  // xs[0..n) = K^{-1} r, then zeros

    // ---- x = Y_I^T z, g = 2 Y_I^T (e - r) + 2 lambda n x_at
    const T reg2 = T(2) * lambda * (T)n;
    T *grow = want_g ? grad_out + row * (int64_t)ld : nullptr;
    if (n_f <= kWave)
        dual_output<T, 1>(Y, ish, xs, esh, rsh, n, n_f, ld, reg2, xat, xrow, grow, bad);
    else if (n_f <= 2 * kWave)
        dual_output<T, 2>(Y, ish, xs, esh, rsh, n, n_f, ld, reg2, xat, xrow, grow, bad);
    else
        dual_output<T, 3>(Y, ish, xs, esh, rsh, n, n_f, ld, reg2, xat, xrow, grow, bad);
    if (lane == 0 && bad && bad_row) atomicMin((unsigned long long *)bad_row, (unsigned long long)row);
}

// Rows with one rating (bin 0): the dual system is 1 x 1, so
//     x = r y / (y . y + lambda)        (lambda n_i with n_i = 1),
// and the fused gradient at x_at is 2 (y . x_at - r) y + 2 lambda x_at.
// Four rows per wavefront, one per 16-lane group: lane c takes columns
// c, c + 16, ... of its row (16 consecutive elements per load step); the
// dots are reduced over the group.
constexpr int kOneCols = 9;  // columns per lane: n_f <= 144
template <typename T>
__global__ __launch_bounds__(256) void sweep_one_kernel(
    const int32_t *__restrict__ idx, const float *__restrict__ val, const T *__restrict__ Y,
    T *__restrict__ X, int n_f, int ld, T lambda, const int32_t *__restrict__ chunk_row,
    const int64_t *__restrict__ chunk_begin, int64_t first, int64_t count,
    const T *__restrict__ X_at, T *__restrict__ grad_out, int64_t *__restrict__ bad_row) {
    const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    if (t >= count) return;  // whole 16-lane groups leave together
    const int c = threadIdx.x & 15;
    const int64_t q = first + t;
    const int64_t row = chunk_row[q], b = chunk_begin[q];
    const T r = (T)val[b];
    const T *y = Y + (int64_t)idx[b] * ld;
    const T *xat = X_at ? X_at + row * (int64_t)ld : X + row * (int64_t)ld;
    const bool want_g = grad_out != nullptr;
    T yv[kOneCols], xv[kOneCols];
    T yy = T(0), e = T(0);
#pragma unroll
    for (int u = 0; u < kOneCols; ++u) {
        const int k = c + 16 * u;
        yv[u] = k < n_f ? y[k] : T(0);
        xv[u] = (want_g && k < n_f) ? xat[k] : T(0);
    }
#pragma unroll
    for (int u = 0; u < kOneCols; ++u) {
        yy += yv[u] * yv[u];
        e += yv[u] * xv[u];
    }
    yy = sum16(yy);
    e = sum16(e);
    const T den = yy + lambda;
    const bool bad = !(den > T(0));
    const T s = r / den, ge = T(2) * (e - r), gl = T(2) * lambda;
    T *xrow = X + row * (int64_t)ld;
#pragma unroll
    for (int u = 0; u < kOneCols; ++u) {
        const int k = c + 16 * u;
        if (k < n_f) {
            if (want_g) grad_out[row * (int64_t)ld + k] = ge * yv[u] + gl * xv[u];
            xrow[k] = bad ? T(NAN) : s * yv[u];
        }
    }
    if (c == 0 && bad && bad_row) atomicMin((unsigned long long *)bad_row, (unsigned long long)row);
}

template <typename T, int VW>
int run_dual(const Plan *plan, const als_csr *R, const T *Y, T *X, int n_f, int ld, T lambda,
             const T *X_at, T *grad_out, int64_t *bad_row, hipStream_t s) {
#define ALS_DUAL_BIN(NBD)                                                                          \
    if (plan->dual_count[NBD] > 0)                                                                 \
        hipLaunchKernelGGL((sweep_dual_kernel<T, NBD, VW>), dim3((unsigned)plan->dual_count[NBD]), \
                           dim3(kWave), 0, s, R->indices, R->values, Y, X, n_f, ld, lambda,        \
                           plan->chunk_row, plan->chunk_begin, plan->chunk_len,                    \
                           plan->dual_first[NBD], plan->dual_count[NBD], X_at, grad_out, bad_row);
    if (plan->dual_count[0] > 0)
        hipLaunchKernelGGL((sweep_one_kernel<T>), dim3((unsigned)((plan->dual_count[0] + 15) / 16)),
                           dim3(256), 0, s, R->indices, R->values, Y, X, n_f, ld, lambda,
                           plan->chunk_row, plan->chunk_begin, plan->dual_first[0],
                           plan->dual_count[0], X_at, grad_out, bad_row);
    ALS_DUAL_BIN(1)
    ALS_DUAL_BIN(2)
    ALS_DUAL_BIN(3)
    ALS_DUAL_BIN(4)
    ALS_DUAL_BIN(5)
    ALS_DUAL_BIN(6)
#undef ALS_DUAL_BIN
    static_assert(kDualMaxBlocks == 6, "one instance per bin");
    return hipGetLastError() == hipSuccess ? ALS_OK : ALS_E_HIP;
}

}  // namespace

int launch_sweep_dual(const Plan *plan, const als_csr *R, const void *Y, void *X, int n_f, int ld,
                      double lambda, als_dtype dt, const void *X_at, void *grad_out,
                      int64_t *bad_row, hipStream_t s) {
    if (!plan || plan->n_dual == 0) return ALS_OK;
    if (dt == ALS_F32) {
        const bool vec = n_f % 4 == 0 && ld % 4 == 0 && ((uintptr_t)Y % 16) == 0 &&
                         (!X_at || ((uintptr_t)X_at % 16) == 0) && ((uintptr_t)X % 16) == 0;
        if (vec)
            return run_dual<float, 4>(plan, R, (const float *)Y, (float *)X, n_f, ld, (float)lambda,
                                      (const float *)X_at, (float *)grad_out, bad_row, s);
        return run_dual<float, 1>(plan, R, (const float *)Y, (float *)X, n_f, ld, (float)lambda,
                                  (const float *)X_at, (float *)grad_out, bad_row, s);
    }
    if (dt == ALS_F64)
        return run_dual<double, 1>(plan, R, (const double *)Y, (double *)X, n_f, ld, lambda,
                                   (const double *)X_at, (double *)grad_out, bad_row, s);
    return ALS_E_INVAL;
}

}  // namespace alsncg
