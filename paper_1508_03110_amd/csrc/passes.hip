// Streaming passes over the ratings: the gradient of Eq. (1) (Section III-A,
// Section V-C "Gradient Evaluation") and the coefficients of the line-search
// quartic Q(alpha) = f(x + alpha p) (Section V-C "Line Search & Loss
// Function Evaluation").
//
// Both walk the same row plan as the half-sweep: one wavefront per chunk,
// L lanes per rating (L = 8 or 16), lane l = L g + c on rating t + g of each
// group of 64 / L and on factor columns c, c + L, ... of it (in vectors of
// VEC), so every gathered factor row is read as L consecutive vectors.  Dot
// products are formed in the factor type and reduced across the L lanes of a
// rating; everything that enters f, ||g||^2 or the quartic coefficients is
// accumulated in FP64 and stored as one partial per chunk (or per block),
// then summed in a fixed order, so results are bitwise reproducible.
#include <initializer_list>

#include <algorithm>

#include "internal.h"

namespace alsncg {
namespace {

// ---------------------------------------------------------------- gathered rows
//
// Lane (g, c) of a wavefront handles rating t + g of each group of 64 / L and
// the factor columns col(q) = (L q + c) * VEC, ..., + VEC - 1 for q < NV: with
// VEC = 4 the L lanes of a rating read 16 L contiguous bytes of a factor row
// per load (FP32 rows whose length and stride are multiples of 4), with
// VEC = 1 they read L consecutive elements.
//
// The VALU issue rate bounds these passes (a wavefront instruction takes 4
// cycles of a 16-lane SIMD): L = 8 halves the cross-lane reduction steps and
// the FP64 accumulation instructions per rating against L = 16, and puts
// fewer padding columns in each dot product for n_f <= 8 L VEC.
template <typename T, int VEC> struct Vec {
    typedef T type __attribute__((ext_vector_type(VEC)));
};
template <typename T> struct Vec<T, 1> {
    typedef T type;
};

template <typename T, int VEC>
__device__ __forceinline__ typename Vec<T, VEC>::type vzero() {
    return typename Vec<T, VEC>::type(T(0));
}

template <typename T, int VEC>
__device__ __forceinline__ T vdot(typename Vec<T, VEC>::type a, typename Vec<T, VEC>::type b) {
    if constexpr (VEC == 1) {
        return a * b;
    } else {
        T s = T(0);
#pragma unroll
        for (int e = 0; e < VEC; ++e) s += a[e] * b[e];
        return s;
    }
}

template <typename T, int VEC>
__device__ __forceinline__ T velem(typename Vec<T, VEC>::type v, int u) {
    if constexpr (VEC == 1) {
        return v;
    } else {
        return v[u];
    }
}
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T, int VEC, int NV, int L>
__device__ __forceinline__ void store_row(const typename Vec<T, VEC>::type (&v)[NV], T *__restrict__ base,
                                          int64_t j, int ld, int n_f, int c) {
    typedef typename Vec<T, VEC>::type V;
    T *row = base + j * ld;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const int col = (L * q + c) * VEC;
        if (col < n_f) *(V *)(row + col) = v[q];
    }
}

// Unconditional row loads for the inner loops.  For q < NV - 1 every
// vector is inside the row (NV = ceil(n_f / (L VEC))); the last one is
// clamped to the row's last vector when (L (NV - 1) + c) VEC >= n_f, so
// every load reads data of the addressed row and no lane branches.  The
// duplicated columns are cancelled by zeros in the row-side operand
// (load_own), lanes past the end of a chunk address a row of the same chunk
// and their results are discarded.
template <int VEC, int NV, int L> struct Cols {
    int last;     // element offset of this lane's last vector (clamped)
    bool last_ok; // that vector holds real columns
    __device__ Cols(int c, int n_f) {
        const int col = (L * (NV - 1) + c) * VEC;
        last_ok = col < n_f;
        last = last_ok ? col : n_f - VEC;
    }
};

template <typename T, int VEC, int NV, int L>
__device__ __forceinline__ void gather_row(typename Vec<T, VEC>::type (&v)[NV], const T *__restrict__ base,
                                           int64_t j, int ld, int c, const Cols<VEC, NV, L> &cl) {
    typedef typename Vec<T, VEC>::type V;
    const T *row = base + j * ld;
#pragma unroll
    for (int q = 0; q < NV - 1; ++q) v[q] = *(const V *)(row + (L * q + c) * VEC);
    v[NV - 1] = *(const V *)(row + cl.last);
}

// Row-side operand: the same loads, columns past n_f set to zero.
template <typename T, int VEC, int NV, int L>
__device__ __forceinline__ void load_own(typename Vec<T, VEC>::type (&v)[NV], const T *__restrict__ base,
                                         int64_t j, int ld, int c, const Cols<VEC, NV, L> &cl) {
    gather_row<T, VEC, NV, L>(v, base, j, ld, c, cl);
    if (!cl.last_ok) v[NV - 1] = vzero<T, VEC>();
}

// Minimum wavefronts per SIMD asked of the compiler for the chunk kernels:
// Gathered groups of ratings in flight per wavefront (register buffers) in
// the gradient and coefficient loops.
constexpr int kGradDepth = 2;
constexpr int kCoefDepth = 2;

// 4 for the FP32 vector-of-4 instances with one workgroup per chunk (at most
// 128 VGPRs, which they fit without spilling), no constraint for the others.
template <typename T, int VEC, bool PERSIST>
constexpr int kPassWaves = (sizeof(T) == 4 && VEC == 4 && !PERSIST) ? 4 : 1;

// Sum over the L lanes of a rating (result in all of them).
template <int L, typename T> __device__ __forceinline__ T sum_rating(T v) {
    if constexpr (L == 16) {
        return sum16(v);
    } else {
        static_assert(L == 8, "8 or 16 lanes per rating");
        if constexpr (sizeof(T) == 4) {
            // quad_perm [1,0,3,2], [2,3,0,1], then row_half_mirror (l -> 7 - l
            // within 8): the l ^ 1, l ^ 2, l ^ 4 butterfly on quad sums
            v += dpp_f32<0xB1>(v);
            v += dpp_f32<0x4E>(v);
            v += dpp_f32<0x141>(v);
            return v;
        } else {
            v += __shfl_xor(v, 1);
            v += __shfl_xor(v, 2);
            v += __shfl_xor(v, 4);
            return v;
        }
    }
}
// Sum over the 64 / L ratings of a group for equal column lane c.
template <int L, typename T> __device__ __forceinline__ T sum_group(T v) {
    if constexpr (L == 8) v += __shfl_xor(v, 8);
    return sum4g(v);
}

// ---------------------------------------------------------------- gradient

// Rows-side pass: for every row i of this orientation (users for R, items
// for R^T) with X the row-side factor and Y the gathered side:
//   G[i] = 2 lambda n_i X[i] + 2 sum_j Y[j] (X[i].Y[j] - r_ij).
// scal[2q] receives this chunk's share of f, scal[2q + 1] of ||G||^2 (rows
// that are whole in this chunk); split rows leave the regulariser and ||G||^2
// to grad_split_kernel.
template <typename T, int VEC, int NV, int L, bool PERSIST>
__global__ __launch_bounds__(64, (kPassWaves<T, VEC, PERSIST>)) void grad_chunks_kernel(
    const int64_t *__restrict__ indptr, const int32_t *__restrict__ idx,
    const float *__restrict__ val, const T *__restrict__ X, const T *__restrict__ Y, int n_f,
    int ld, double lambda, int64_t n_chunks, const int32_t *__restrict__ chunk_row,
    const int64_t *__restrict__ chunk_begin, const int32_t *__restrict__ chunk_len,
    const int32_t *__restrict__ chunk_slot, T *__restrict__ G, T *__restrict__ partial,
    double *__restrict__ scal, int data_in_f, int want_g) {
    typedef typename Vec<T, VEC>::type V;
    constexpr int GR = kWave / L;  // ratings per step
    const int64_t stride = PERSIST ? (int64_t)gridDim.x : n_chunks;
    for (int64_t q = blockIdx.x; q < n_chunks; q += stride) {
    const int lane = threadIdx.x, g = lane / L, c = lane % L;
    const Cols<VEC, NV, L> cl(c, n_f);
    const int64_t row = chunk_row[q], b = chunk_begin[q], e = b + chunk_len[q];
    const int slot = chunk_slot[q];
    V x[NV], acc[NV];
    load_own<T, VEC, NV, L>(x, X, row, ld, c, cl);
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = vzero<T, VEC>();
    double e2 = 0.0;
    if (b < e) {
        // Group X holds ratings b + X GR + g.  D buffers of gathered rows
        // rotate; a group's ids are loaded D steps before its gather (ring
        // jq), since the wait counter completes loads in issue order and a
        // later id load would make each wait drain the gathers in flight; its
        // values are loaded with the gather (no register copy of a load in
        // flight, which would wait for it).  Lanes past the end use the
        // chunk's last rating (a valid row) and contribute nothing.
        constexpr int D = kGradDepth;
        const int64_t ngr = (e - b + GR - 1) / GR;
        auto pos = [&](int64_t x) -> int64_t { return min(b + x * GR + g, e - 1); };
        auto step = [&](const V (&y)[NV], bool ok, T r) {
            T d = T(0);
#pragma unroll
            for (int k = 0; k < NV; ++k) d += vdot<T, VEC>(x[k], y[k]);
            d = sum_rating<L>(d);
            const T res = ok ? d - r : T(0);
#pragma unroll
            for (int k = 0; k < NV; ++k) acc[k] += res * y[k];
            if (c == 0) e2 += (double)res * (double)res;
        };
        V ys[D][NV];
        T rv[D];
        int jq[D];
#pragma unroll
        for (int k = 0; k < D - 1; ++k) {
            gather_row<T, VEC, NV, L>(ys[k], Y, idx[pos(k)], ld, c, cl);
            rv[k] = (T)val[pos(k)];
        }
#pragma unroll
        for (int k = D - 1; k < 2 * D - 1; ++k) jq[k % D] = idx[pos(k)];
        for (int64_t s0 = 0; s0 < ngr; s0 += D) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const int slot = (k + D - 1) % D;
                gather_row<T, VEC, NV, L>(ys[slot], Y, jq[slot], ld, c, cl);
                rv[slot] = (T)val[pos(s0 + k + D - 1)];
                jq[slot] = idx[pos(s0 + k + 2 * D - 1)];
                if (s0 + k < ngr) step(ys[k], b + (s0 + k) * GR + g < e, rv[k]);
            }
        }
    }
    if (!cl.last_ok) acc[NV - 1] = vzero<T, VEC>();  // duplicated columns
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        if constexpr (VEC == 1) {
            acc[k] = sum_group<L>(acc[k]);
        } else {
#pragma unroll
            for (int u = 0; u < VEC; ++u) acc[k][u] = sum_group<L>(acc[k][u]);
        }
    }
    e2 = sum64(e2);
    if (slot < 0) {
        const int64_t n_i = indptr[row + 1] - indptr[row];
        const T reg2 = T(2.0 * lambda * (double)n_i);
        double gn = 0.0, xn = 0.0;
        V gv[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            gv[k] = T(2) * acc[k] + reg2 * x[k];
            if (g == 0) {
                gn += (double)vdot<T, VEC>(gv[k], gv[k]);
                xn += (double)vdot<T, VEC>(x[k], x[k]);
            }
        }
        if (G && g == 0) store_row<T, VEC, NV, L>(gv, G, row, ld, n_f, c);
        gn = sum64(gn);
        xn = sum64(xn);
        if (lane == 0) {
            scal[2 * q] = (data_in_f ? e2 : 0.0) + lambda * (double)n_i * xn;
            scal[2 * q + 1] = want_g ? gn : 0.0;
        }
    } else {
        if (g == 0) store_row<T, VEC, NV, L>(acc, partial, slot, NV * L * VEC, n_f, c);
        if (lane == 0) {
            scal[2 * q] = data_in_f ? e2 : 0.0;
            scal[2 * q + 1] = 0.0;
        }
    }
    }
}

template <typename T, int NP>
__global__ __launch_bounds__(64) void grad_split_kernel(
    const int64_t *__restrict__ indptr, const T *__restrict__ X, int n_f, int ld, double lambda,
    int64_t n_split, const int32_t *__restrict__ split_row, const int32_t *__restrict__ split_slot0,
    const int32_t *__restrict__ split_nslot, const T *__restrict__ partial, T *__restrict__ G,
    double *__restrict__ scal, int want_g) {
    const int64_t s = blockIdx.x;
    if (s >= n_split) return;
    const int lane = threadIdx.x;
    const int64_t row = split_row[s], s0 = split_slot0[s];
    const int ns = split_nslot[s];
    const int64_t n_i = indptr[row + 1] - indptr[row];
    const T reg2 = T(2.0 * lambda * (double)n_i);
    double gn = 0.0, xn = 0.0;
    for (int col = lane; col < n_f; col += kWave) {
        T acc = T(0);
        for (int u = 0; u < ns; ++u) acc += partial[(s0 + u) * NP + col];
        const T x = X[row * (int64_t)ld + col];
        const T gv = T(2) * acc + reg2 * x;
        if (G) G[row * (int64_t)ld + col] = gv;
        gn += (double)gv * (double)gv;
        xn += (double)x * (double)x;
    }
    gn = sum64(gn);
    xn = sum64(xn);
    if (lane == 0) {
        scal[2 * s] = lambda * (double)n_i * xn;
        scal[2 * s + 1] = want_g ? gn : 0.0;
    }
}

// ---------------------------------------------------------------- quartic coefficients

// Per rating, with a0 = xu.xm, a1 = xu.pm + pu.xm, a2 = pu.pm, d = r - a0:
//   (r - u.m)^2 = d^2 - 2 d a1 alpha + (a1^2 - 2 d a2) alpha^2 + 2 a1 a2 alpha^3 + a2^2 alpha^4.
// The first chunk of each user row also adds that user's regulariser
// lambda n_i ||xu + alpha pu||^2.  part[5q + n] is the chunk's share of C_n.
// XU, PU: user rows (stride ld); XM, PM: the gathered item rows (stride
// ldm, e.g. 2 ld when they are the two halves of interleaved [x_j | p_j]
// rows).
template <typename T, int VEC, int NV, int L, bool PERSIST>
__global__ __launch_bounds__(64, (kPassWaves<T, VEC, PERSIST>)) void coeff_chunks_kernel(
    const int64_t *__restrict__ indptr, const int32_t *__restrict__ idx,
    const float *__restrict__ val, const T *__restrict__ XU, const T *__restrict__ XM,
    const T *__restrict__ PU, const T *__restrict__ PM, int n_f, int ld, int ldm, double lambda,
    int64_t n_chunks, const int32_t *__restrict__ chunk_row,
    const int64_t *__restrict__ chunk_begin, const int32_t *__restrict__ chunk_len,
    double *__restrict__ part, const double *__restrict__ pred) {
    typedef typename Vec<T, VEC>::type V;
    constexpr int GR = kWave / L;  // ratings per step
    if (pred && *pred == 0.0) return;
    const int64_t stride = PERSIST ? (int64_t)gridDim.x : n_chunks;
    for (int64_t q = blockIdx.x; q < n_chunks; q += stride) {
    const int lane = threadIdx.x, g = lane / L, c = lane % L;
    const Cols<VEC, NV, L> cl(c, n_f);
    const int64_t row = chunk_row[q], b = chunk_begin[q], e = b + chunk_len[q];
    V xu[NV], pu[NV];
    load_own<T, VEC, NV, L>(xu, XU, row, ld, c, cl);
    load_own<T, VEC, NV, L>(pu, PU, row, ld, c, cl);
    double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0, c4 = 0.0;
    if (b < e) {
        // Same pipeline as grad_chunks_kernel: D buffers of gathered item rows
        // (x and p), ids D steps ahead of their gathers, values with them.
        constexpr int D = kCoefDepth;
        const int64_t ngr = (e - b + GR - 1) / GR;
        auto pos = [&](int64_t x) -> int64_t { return min(b + x * GR + g, e - 1); };
        auto step = [&](const V (&xm)[NV], const V (&pm)[NV], bool ok, float r) {
            // one FMA chain per dot product (a1 takes both of its terms)
            T a0 = T(0), a1 = T(0), a2 = T(0);
#pragma unroll
            for (int k = 0; k < NV; ++k)
#pragma unroll
                for (int u = 0; u < VEC; ++u) {
                    const T xuk = velem<T, VEC>(xu[k], u), puk = velem<T, VEC>(pu[k], u);
                    const T xmk = velem<T, VEC>(xm[k], u), pmk = velem<T, VEC>(pm[k], u);
                    a0 = fma_t(xuk, xmk, a0);
                    a1 = fma_t(xuk, pmk, a1);
                    a1 = fma_t(puk, xmk, a1);
                    a2 = fma_t(puk, pmk, a2);
                }
            a0 = sum_rating<L>(a0);
            a1 = sum_rating<L>(a1);
            a2 = sum_rating<L>(a2);
            if (ok && c == 0) {
                const double d = (double)r - (double)a0, A1 = (double)a1, A2 = (double)a2;
                c0 += d * d;
                c1 += -2.0 * d * A1;
                c2 += A1 * A1 - 2.0 * d * A2;
                c3 += 2.0 * A1 * A2;
                c4 += A2 * A2;
            }
        };
        V xs[D][NV], ps[D][NV];
        float rv[D];
        int jq[D];
#pragma unroll
        for (int k = 0; k < D - 1; ++k) {
            const int j = idx[pos(k)];
            gather_row<T, VEC, NV, L>(xs[k], XM, j, ldm, c, cl);
            gather_row<T, VEC, NV, L>(ps[k], PM, j, ldm, c, cl);
            rv[k] = val[pos(k)];
        }
#pragma unroll
        for (int k = D - 1; k < 2 * D - 1; ++k) jq[k % D] = idx[pos(k)];
        for (int64_t s0 = 0; s0 < ngr; s0 += D) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const int slot = (k + D - 1) % D;
                gather_row<T, VEC, NV, L>(xs[slot], XM, jq[slot], ldm, c, cl);
                gather_row<T, VEC, NV, L>(ps[slot], PM, jq[slot], ldm, c, cl);
                rv[slot] = val[pos(s0 + k + D - 1)];
                jq[slot] = idx[pos(s0 + k + 2 * D - 1)];
                if (s0 + k < ngr) step(xs[k], ps[k], b + (s0 + k) * GR + g < e, rv[k]);
            }
        }
    }
    c0 = sum64(c0);
    c1 = sum64(c1);
    c2 = sum64(c2);
    c3 = sum64(c3);
    c4 = sum64(c4);
    if (b == indptr[row]) {
        double xx = 0.0, xp = 0.0, pp = 0.0;
#pragma unroll
        for (int k = 0; k < NV; ++k)
            if (g == 0) {
                xx += (double)vdot<T, VEC>(xu[k], xu[k]);
                xp += (double)vdot<T, VEC>(xu[k], pu[k]);
                pp += (double)vdot<T, VEC>(pu[k], pu[k]);
            }
        xx = sum64(xx);
        xp = sum64(xp);
        pp = sum64(pp);
        const double ln = lambda * (double)(indptr[row + 1] - indptr[row]);
        c0 += ln * xx;
        c1 += 2.0 * ln * xp;
        c2 += ln * pp;
    }
    if (lane == 0) {
        double *o = part + 5 * q;
        o[0] = c0;
        o[1] = c1;
        o[2] = c2;
        o[3] = c3;
        o[4] = c4;
    }
    }
}

// XP[j] = [XM[j] | PM[j]] (the first n_f columns of each, row stride 2 ld):
// the coefficient pass gathers both rows of every rated item, and one
// contiguous pair touches fewer cache lines and DRAM pages than two rows in
// separate arrays (bitwise the same arithmetic).
template <typename T>
__global__ __launch_bounds__(256) void pair_rows_kernel(const T *__restrict__ XM,
                                                        const T *__restrict__ PM, int64_t n,
                                                        int n_f, int ld, T *__restrict__ XP,
                                                        const double *__restrict__ pred) {
    if (pred && *pred == 0.0) return;
    const int lane = threadIdx.x & 63;
    for (int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); j < n;
         j += (int64_t)gridDim.x * 4) {
        for (int r = lane; r < 2 * n_f; r += kWave) {
            const int half = r >= n_f, col = r - half * n_f;
            XP[j * 2 * ld + half * ld + col] = (half ? PM : XM)[j * ld + col];
        }
    }
}

// Item regulariser lambda n_j ||xm_j + alpha pm_j||^2, n_j from the CSR of
// R^T.  Fixed grid; block k writes part[5k .. 5k + 4] (C3 = C4 = 0).
template <typename T, int NBV>
__global__ __launch_bounds__(256) void coeff_itemreg_kernel(const int64_t *__restrict__ indptr_t,
                                                            int64_t n_items,
                                                            const T *__restrict__ XM,
                                                            const T *__restrict__ PM, int n_f,
                                                            int ld, double lambda,
                                                            double *__restrict__ part,
                                                            const double *__restrict__ pred) {
    __shared__ double red[4][3];
    if (pred && *pred == 0.0) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
    double xx = 0.0, xp = 0.0, pp = 0.0;
    for (int64_t base = ((int64_t)blockIdx.x * 4 + wv) * 4; base < n_items;
         base += (int64_t)gridDim.x * 16) {
        const int64_t j = base + g;
        const bool ok = j < n_items;
        T a = T(0), bq = T(0), cc = T(0);
#pragma unroll
        for (int cb = 0; cb < NBV; ++cb) {
            const int col = 16 * cb + c;
            const bool in = ok && col < n_f;
            const T xm = in ? XM[j * ld + col] : T(0);
            const T pm = in ? PM[j * ld + col] : T(0);
            a += xm * xm;
            bq += xm * pm;
            cc += pm * pm;
        }
        a = sum16(a);
        bq = sum16(bq);
        cc = sum16(cc);
        if (ok && c == 0) {
            const double n = (double)(indptr_t[j + 1] - indptr_t[j]);
            xx += n * (double)a;
            xp += n * (double)bq;
            pp += n * (double)cc;
        }
    }
    xx = sum64(xx);
    xp = sum64(xp);
    pp = sum64(pp);
    if (lane == 0) {
        red[wv][0] = xx;
        red[wv][1] = xp;
        red[wv][2] = pp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int w = 0; w < 4; ++w) {
            s0 += red[w][0];
            s1 += red[w][1];
            s2 += red[w][2];
        }
        double *o = part + 5 * (int64_t)blockIdx.x;
        o[0] = lambda * s0;
        o[1] = 2.0 * lambda * s1;
        o[2] = lambda * s2;
        o[3] = 0.0;
        o[4] = 0.0;
    }
}

constexpr int kItemBlocks = kCoeffItemBlocks;

// Grid of a streaming-pass chunk kernel: one workgroup per chunk, or the
// plan's persistent grid.
static unsigned chunk_grid(const Plan *p) {
    return (unsigned)(p->grid_pass > 0 ? std::min<int64_t>(p->grid_pass, p->n_chunks) : p->n_chunks);
}

template <typename T, int VEC, int NV, int L>
int run_gradient(Ctx *ctx, const Plan *pR, const als_csr *R, const Plan *pRt, const als_csr *Rt,
                 const T *U, const T *M, int n_f, int ld, double lambda, T *gU, T *gM,
                 double *out2, hipStream_t s) {
    constexpr int NP = NV * L * VEC;
    if ((int64_t)L * (NV - 1) * VEC >= n_f || NP < n_f) return ALS_E_INVAL;  // see Cols
    const bool doR = (gU != nullptr) || (out2 != nullptr);
    const bool doRt = (gM != nullptr) || (out2 != nullptr);
    const int64_t rowsR = doR ? pR->n_chunks + pR->n_split_rows : 0;
    const int64_t rowsRt = doRt ? pRt->n_chunks + pRt->n_split_rows : 0;
    const size_t scal_bytes =
        align_up((size_t)((rowsR + rowsRt + 1) * 2 + kSumStageDoubles) * sizeof(double), 256);
    const size_t pR_bytes = doR ? align_up((size_t)pR->n_slots * NP * sizeof(T) + 16, 256) : 0;
    const size_t pRt_bytes = doRt ? align_up((size_t)pRt->n_slots * NP * sizeof(T) + 16, 256) : 0;
    int err = ALS_OK;
    char *ws = (char *)ctx->workspace(scal_bytes + pR_bytes + pRt_bytes, s, &err);
    if (!ws) return err;
    double *scal = (double *)ws;
    T *partR = (T *)(ws + scal_bytes);
    T *partRt = (T *)(ws + scal_bytes + pR_bytes);
    if (doR) {
        if (pR->n_chunks) {
#define ALS_GRAD_R(P)                                                                               \
    hipLaunchKernelGGL((grad_chunks_kernel<T, VEC, NV, L, P>), dim3(chunk_grid(pR)), dim3(kWave), 0, s, \
                       R->indptr, R->indices, R->values, U, M, n_f, ld, lambda, pR->n_chunks,       \
                       pR->chunk_row, pR->chunk_begin, pR->chunk_len, pR->chunk_slot, gU, partR,    \
                       scal, 1, gU != nullptr ? 1 : 0)
            if (pR->grid_pass > 0)
                ALS_GRAD_R(true);
            else
                ALS_GRAD_R(false);
#undef ALS_GRAD_R
        }
        if (pR->n_split_rows)
            hipLaunchKernelGGL((grad_split_kernel<T, NP>), dim3((unsigned)pR->n_split_rows),
                               dim3(kWave), 0, s, R->indptr, U, n_f, ld, lambda, pR->n_split_rows,
                               pR->split_row, pR->split_slot0, pR->split_nslot, partR, gU,
                               scal + 2 * pR->n_chunks, gU != nullptr ? 1 : 0);
    }
    if (doRt) {
        double *sc = scal + 2 * rowsR;
        if (pRt->n_chunks) {
#define ALS_GRAD_RT(P)                                                                               \
    hipLaunchKernelGGL((grad_chunks_kernel<T, VEC, NV, L, P>), dim3(chunk_grid(pRt)), dim3(kWave), 0, s, \
                       Rt->indptr, Rt->indices, Rt->values, M, U, n_f, ld, lambda, pRt->n_chunks,    \
                       pRt->chunk_row, pRt->chunk_begin, pRt->chunk_len, pRt->chunk_slot, gM,        \
                       partRt, sc, 0, gM != nullptr ? 1 : 0)
            if (pRt->grid_pass > 0)
                ALS_GRAD_RT(true);
            else
                ALS_GRAD_RT(false);
#undef ALS_GRAD_RT
        }
        if (pRt->n_split_rows)
            hipLaunchKernelGGL((grad_split_kernel<T, NP>), dim3((unsigned)pRt->n_split_rows),
                               dim3(kWave), 0, s, Rt->indptr, M, n_f, ld, lambda,
                               pRt->n_split_rows, pRt->split_row, pRt->split_slot0,
                               pRt->split_nslot, partRt, gM, sc + 2 * pRt->n_chunks,
                               gM != nullptr ? 1 : 0);
    }
    if (out2)
        launch_sum_columns(scal, rowsR + rowsRt, 2, out2, 0, scal + (rowsR + rowsRt + 1) * 2, s);
    return hipGetLastError() == hipSuccess ? ALS_OK : ALS_E_HIP;
}

template <typename T, int VEC, int NV, int L>
int run_coeffs(Ctx *ctx, const Plan *pR, const als_csr *R, const als_csr *Rt, const T *U,
               const T *M, const T *PU, const T *PM, int n_f, int ld, double lambda,
               double *coeffs, const double *pred, hipStream_t s, double *fixed,
               size_t fixed_doubles) {
    if ((int64_t)L * (NV - 1) * VEC >= n_f || L * NV * VEC < n_f) return ALS_E_INVAL;  // see Cols
    const int64_t rows = pR->n_chunks + kItemBlocks;
    const size_t need = (size_t)(rows * 5 + kSumStageDoubles);
    double *part = fixed;
    // gathered item rows: [x_j | p_j] pairs in workspace, or (fixed scratch)
    // the two arrays as given
    const T *GX = M, *GP = PM;
    int ldm = ld;
    if (fixed) {
        if (need > fixed_doubles) return ALS_E_BUDGET;
    } else {
        const size_t part_bytes = align_up(need * sizeof(double), 256);
        const size_t pair_bytes = (size_t)Rt->n_rows * 2 * ld * sizeof(T);
        int err = ALS_OK;
        char *ws = (char *)ctx->workspace(part_bytes + pair_bytes, s, &err);
        if (!ws) return err;
        part = (double *)ws;
        T *XP = (T *)(ws + part_bytes);
        if (Rt->n_rows > 0) {
            const unsigned blocks = (unsigned)std::min<int64_t>((Rt->n_rows + 3) / 4, 8192);
            hipLaunchKernelGGL(pair_rows_kernel<T>, dim3(blocks), dim3(256), 0, s, M, PM,
                               Rt->n_rows, n_f, ld, XP, pred);
        }
        GX = XP;
        GP = XP + ld;
        ldm = 2 * ld;
    }
    if (pR->n_chunks) {
        // a predicated pass (launched in every iteration, needed only after a
        // restart) always takes a persistent grid, so that when it is off it
        // costs a few thousand empty workgroups instead of one per chunk
        unsigned grid = chunk_grid(pR);
        const bool persist = pR->grid_pass > 0 || pred != nullptr;
        if (pred && pR->grid_pass <= 0)
            grid = (unsigned)std::min<int64_t>(pR->n_chunks, (int64_t)ctx->num_cu * 16);
#define ALS_COEF(P)                                                                             \
    hipLaunchKernelGGL((coeff_chunks_kernel<T, VEC, NV, L, P>), dim3(grid), dim3(kWave), 0, s,       \
                       R->indptr, R->indices, R->values, U, GX, PU, GP, n_f, ld, ldm, lambda,   \
                       pR->n_chunks, pR->chunk_row, pR->chunk_begin, pR->chunk_len, part, pred)
        if (persist)
            ALS_COEF(true);
        else
            ALS_COEF(false);
#undef ALS_COEF
    }
    hipLaunchKernelGGL((coeff_itemreg_kernel<T, (NV * L * VEC + 15) / 16>), dim3(kItemBlocks), dim3(256), 0, s,
                       Rt->indptr, Rt->n_rows, M, PM, n_f, ld, lambda, part + 5 * pR->n_chunks,
                       pred);
    launch_sum_columns(part, rows, 5, coeffs, 0, part + rows * 5, s);
    return hipGetLastError() == hipSuccess ? ALS_OK : ALS_E_HIP;
}

// FP32 rows of length and stride divisible by 4 on 16-byte boundaries are
// gathered 4 elements per lane; everything else one element per lane.
static bool vec4_ok(int n_f, int ld, std::initializer_list<const void *> ptrs) {
    if (n_f % 4 != 0 || ld % 4 != 0) return false;
    for (const void *p : ptrs)
        if (p && ((uintptr_t)p % 16) != 0) return false;
    return true;
}

}  // namespace

// Lanes per rating and vectors per lane for n_f: FP32 rows in vectors of 4
// with 8 lanes per rating up to n_f = 128, else 16; single elements with 8
// lanes up to n_f = 64, else 16.
#define ALS_PASS_DISPATCH(dt, n_f, vec4, X)                            \
    do {                                                               \
        if ((dt) == ALS_F32 && (vec4)) {                               \
            switch (((n_f) + 31) / 32) {                               \
                case 1: X(float, 4, 1, 8);                             \
                case 2: X(float, 4, 2, 8);                             \
                case 3: X(float, 4, 3, 8);                             \
                case 4: X(float, 4, 4, 8);                             \
                case 5:                                                \
                case 6: X(float, 4, 3, 16);                            \
                default: return ALS_E_INVAL;                           \
            }                                                          \
        }                                                              \
        if ((dt) != ALS_F32 && (dt) != ALS_F64) return ALS_E_INVAL;    \
        if ((n_f) <= 64) {                                             \
            switch (((n_f) + 7) / 8) {                                 \
                case 1: ALS_PASS_T(dt, X, 1, 1, 8);                    \
                case 2: ALS_PASS_T(dt, X, 1, 2, 8);                    \
                case 3: ALS_PASS_T(dt, X, 1, 3, 8);                    \
                case 4: ALS_PASS_T(dt, X, 1, 4, 8);                    \
                case 5: ALS_PASS_T(dt, X, 1, 5, 8);                    \
                case 6: ALS_PASS_T(dt, X, 1, 6, 8);                    \
                case 7: ALS_PASS_T(dt, X, 1, 7, 8);                    \
                default: ALS_PASS_T(dt, X, 1, 8, 8);                   \
            }                                                          \
        }                                                              \
        switch (((n_f) + 15) / 16) {                                   \
            case 5: ALS_PASS_T(dt, X, 1, 5, 16);                       \
            case 6: ALS_PASS_T(dt, X, 1, 6, 16);                       \
            case 7: ALS_PASS_T(dt, X, 1, 7, 16);                       \
            case 8: ALS_PASS_T(dt, X, 1, 8, 16);                       \
            case 9: ALS_PASS_T(dt, X, 1, 9, 16);                       \
            default: return ALS_E_INVAL;                               \
        }                                                              \
    } while (0)
#define ALS_PASS_T(dt, X, VEC, NV, L) \
    if ((dt) == ALS_F32) X(float, VEC, NV, L); else X(double, VEC, NV, L)

int launch_gradient(Ctx *ctx, const Plan *pR, const als_csr *R, const Plan *pRt, const als_csr *Rt,
                    const void *U, const void *M, int n_f, int ld, double lambda, als_dtype dt,
                    void *gU, void *gM, double *out2, hipStream_t s) {
#define GA(T, VEC, NV, L)                                                                         \
    return run_gradient<T, VEC, NV, L>(ctx, pR, R, pRt, Rt, (const T *)U, (const T *)M, n_f, ld, \
                                       lambda, (T *)gU, (T *)gM, out2, s)
    ALS_PASS_DISPATCH(dt, n_f, vec4_ok(n_f, ld, {U, M, gU, gM}), GA);
#undef GA
}

int launch_coeffs(Ctx *ctx, const Plan *pR, const als_csr *R, const als_csr *Rt, const void *U,
                  const void *M, const void *pU, const void *pM, int n_f, int ld, double lambda,
                  als_dtype dt, double *coeffs, const double *pred, hipStream_t s, double *fixed,
                  size_t fixed_doubles) {
#define CA(T, VEC, NV, L)                                                                       \
    return run_coeffs<T, VEC, NV, L>(ctx, pR, R, Rt, (const T *)U, (const T *)M, (const T *)pU, \
                                     (const T *)pM, n_f, ld, lambda, coeffs, pred, s, fixed,     \
                                     fixed_doubles)
    ALS_PASS_DISPATCH(dt, n_f, vec4_ok(n_f, ld, {U, M, pU, pM}), CA);
#undef CA
}

}  // namespace alsncg
