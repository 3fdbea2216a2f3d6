// Streaming passes over the ratings: the gradient of Eq. (1) (Section III-A,
// Section V-C "Gradient Evaluation") and the coefficients of the line-search
// quartic Q(alpha) = f(x + alpha p) (Section V-C "Line Search & Loss
// Function Evaluation").
//
// Both walk the same row plan as the half-sweep: one wavefront per chunk,
// lane l = 16 g + c handles rating t + g of each group of 4 and factor
// columns c, c + 16, ... of it, so every gathered factor row is read as 16
// consecutive words per quarter-wave.  Dot products are formed in the factor
// type and reduced across the 16 lanes of a quarter-wave; everything that
// enters f, ||g||^2 or the quartic coefficients is accumulated in FP64 and
// stored as one partial per chunk (or per block), then summed in a fixed
// order, so results are bitwise reproducible.
#include "internal.h"

namespace alsncg {
namespace {

// ---------------------------------------------------------------- gradient

// Rows-side pass: for every row i of this orientation (users for R, items
// for R^T) with X the row-side factor and Y the gathered side:
//   G[i] = 2 lambda n_i X[i] + 2 sum_j Y[j] (X[i].Y[j] - r_ij).
// scal[2q] receives this chunk's share of f, scal[2q + 1] of ||G||^2 (rows
// that are whole in this chunk); split rows leave the regulariser and ||G||^2
// to grad_split_kernel.
template <typename T, int NBV>
__global__ __launch_bounds__(64) void grad_chunks_kernel(
    const int64_t *__restrict__ indptr, const int32_t *__restrict__ idx,
    const float *__restrict__ val, const T *__restrict__ X, const T *__restrict__ Y, int n_f,
    int ld, double lambda, int64_t n_chunks, const int32_t *__restrict__ chunk_row,
    const int64_t *__restrict__ chunk_begin, const int32_t *__restrict__ chunk_len,
    const int32_t *__restrict__ chunk_slot, T *__restrict__ G, T *__restrict__ partial,
    double *__restrict__ scal, int data_in_f, int want_g) {
    const int64_t q = blockIdx.x;
    if (q >= n_chunks) return;
    const int lane = threadIdx.x, g = lane >> 4, c = lane & 15;
    const int64_t row = chunk_row[q], b = chunk_begin[q], e = b + chunk_len[q];
    const int slot = chunk_slot[q];
    const T *xr = X + row * (int64_t)ld;
    T x[NBV], acc[NBV];
#pragma unroll
    for (int cb = 0; cb < NBV; ++cb) {
        const int col = 16 * cb + c;
        x[cb] = col < n_f ? xr[col] : T(0);
        acc[cb] = T(0);
    }
    double e2 = 0.0;
    for (int64_t t = b; t < e; t += 4) {
        const int64_t p = t + g;
        const bool ok = p < e;
        const int j = ok ? idx[p] : 0;
        const T r = ok ? (T)val[p] : T(0);
        const T *yr = Y + (int64_t)j * ld;
        T y[NBV];
        T d = T(0);
#pragma unroll
        for (int cb = 0; cb < NBV; ++cb) {
            const int col = 16 * cb + c;
            y[cb] = (ok && col < n_f) ? yr[col] : T(0);
            d += x[cb] * y[cb];
        }
        d = sum16(d);
        const T res = ok ? d - r : T(0);
#pragma unroll
        for (int cb = 0; cb < NBV; ++cb) acc[cb] += res * y[cb];
        if (c == 0) e2 += (double)res * (double)res;
    }
#pragma unroll
    for (int cb = 0; cb < NBV; ++cb) acc[cb] = sum4g(acc[cb]);
    e2 = sum64(e2);
    if (slot < 0) {
        const int64_t n_i = indptr[row + 1] - indptr[row];
        const T reg2 = T(2.0 * lambda * (double)n_i);
        double gn = 0.0, xn = 0.0;
#pragma unroll
        for (int cb = 0; cb < NBV; ++cb) {
            const int col = 16 * cb + c;
            const T gv = T(2) * acc[cb] + reg2 * x[cb];
            if (g == 0 && col < n_f) {
                if (G) G[row * (int64_t)ld + col] = gv;
                gn += (double)gv * (double)gv;
                xn += (double)x[cb] * (double)x[cb];
            }
        }
        gn = sum64(gn);
        xn = sum64(xn);
        if (lane == 0) {
            scal[2 * q] = (data_in_f ? e2 : 0.0) + lambda * (double)n_i * xn;
            scal[2 * q + 1] = want_g ? gn : 0.0;
        }
    } else {
        constexpr int NP = NBV * 16;
#pragma unroll
        for (int cb = 0; cb < NBV; ++cb)
            if (g == 0) partial[(int64_t)slot * NP + 16 * cb + c] = acc[cb];
        if (lane == 0) {
            scal[2 * q] = data_in_f ? e2 : 0.0;
            scal[2 * q + 1] = 0.0;
        }
    }
}

template <typename T, int NBV>
__global__ __launch_bounds__(64) void grad_split_kernel(
    const int64_t *__restrict__ indptr, const T *__restrict__ X, int n_f, int ld, double lambda,
    int64_t n_split, const int32_t *__restrict__ split_row, const int32_t *__restrict__ split_slot0,
    const int32_t *__restrict__ split_nslot, const T *__restrict__ partial, T *__restrict__ G,
    double *__restrict__ scal, int want_g) {
    constexpr int NP = NBV * 16;
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
template <typename T, int NBV>
__global__ __launch_bounds__(64) void coeff_chunks_kernel(
    const int64_t *__restrict__ indptr, const int32_t *__restrict__ idx,
    const float *__restrict__ val, const T *__restrict__ XU, const T *__restrict__ XM,
    const T *__restrict__ PU, const T *__restrict__ PM, int n_f, int ld, double lambda,
    int64_t n_chunks, const int32_t *__restrict__ chunk_row,
    const int64_t *__restrict__ chunk_begin, const int32_t *__restrict__ chunk_len,
    double *__restrict__ part) {
    const int64_t q = blockIdx.x;
    if (q >= n_chunks) return;
    const int lane = threadIdx.x, g = lane >> 4, c = lane & 15;
    const int64_t row = chunk_row[q], b = chunk_begin[q], e = b + chunk_len[q];
    T xu[NBV], pu[NBV];
#pragma unroll
    for (int cb = 0; cb < NBV; ++cb) {
        const int col = 16 * cb + c;
        xu[cb] = col < n_f ? XU[row * (int64_t)ld + col] : T(0);
        pu[cb] = col < n_f ? PU[row * (int64_t)ld + col] : T(0);
    }
    double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0, c4 = 0.0;
    for (int64_t t = b; t < e; t += 4) {
        const int64_t p = t + g;
        const bool ok = p < e;
        const int j = ok ? idx[p] : 0;
        const float r = ok ? val[p] : 0.0f;
        const T *xmr = XM + (int64_t)j * ld;
        const T *pmr = PM + (int64_t)j * ld;
        T a0 = T(0), a1 = T(0), a2 = T(0);
#pragma unroll
        for (int cb = 0; cb < NBV; ++cb) {
            const int col = 16 * cb + c;
            const bool in = ok && col < n_f;
            const T xm = in ? xmr[col] : T(0);
            const T pm = in ? pmr[col] : T(0);
            a0 += xu[cb] * xm;
            a1 += xu[cb] * pm + pu[cb] * xm;
            a2 += pu[cb] * pm;
        }
        a0 = sum16(a0);
        a1 = sum16(a1);
        a2 = sum16(a2);
        if (ok && c == 0) {
            const double d = (double)r - (double)a0, A1 = (double)a1, A2 = (double)a2;
            c0 += d * d;
            c1 += -2.0 * d * A1;
            c2 += A1 * A1 - 2.0 * d * A2;
            c3 += 2.0 * A1 * A2;
            c4 += A2 * A2;
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
        for (int cb = 0; cb < NBV; ++cb)
            if (g == 0) {
                xx += (double)xu[cb] * (double)xu[cb];
                xp += (double)xu[cb] * (double)pu[cb];
                pp += (double)pu[cb] * (double)pu[cb];
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

// Item regulariser lambda n_j ||xm_j + alpha pm_j||^2, n_j from the CSR of
// R^T.  Fixed grid; block k writes part[5k .. 5k + 4] (C3 = C4 = 0).
template <typename T, int NBV>
__global__ __launch_bounds__(256) void coeff_itemreg_kernel(const int64_t *__restrict__ indptr_t,
                                                            int64_t n_items,
                                                            const T *__restrict__ XM,
                                                            const T *__restrict__ PM, int n_f,
                                                            int ld, double lambda,
                                                            double *__restrict__ part) {
    __shared__ double red[4][3];
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

constexpr int kItemBlocks = 512;

template <typename T, int NBV>
int run_gradient(Ctx *ctx, const Plan *pR, const als_csr *R, const Plan *pRt, const als_csr *Rt,
                 const T *U, const T *M, int n_f, int ld, double lambda, T *gU, T *gM,
                 double *out2, hipStream_t s) {
    constexpr int NP = NBV * 16;
    const bool doR = (gU != nullptr) || (out2 != nullptr);
    const bool doRt = (gM != nullptr) || (out2 != nullptr);
    const int64_t rowsR = doR ? pR->n_chunks + pR->n_split_rows : 0;
    const int64_t rowsRt = doRt ? pRt->n_chunks + pRt->n_split_rows : 0;
    const size_t scal_bytes = align_up((size_t)(rowsR + rowsRt + 1) * 2 * sizeof(double), 256);
    const size_t pR_bytes = doR ? align_up((size_t)pR->n_slots * NP * sizeof(T) + 16, 256) : 0;
    const size_t pRt_bytes = doRt ? align_up((size_t)pRt->n_slots * NP * sizeof(T) + 16, 256) : 0;
    int err = ALS_OK;
    char *ws = (char *)ctx->workspace(scal_bytes + pR_bytes + pRt_bytes, s, &err);
    if (!ws) return err;
    double *scal = (double *)ws;
    T *partR = (T *)(ws + scal_bytes);
    T *partRt = (T *)(ws + scal_bytes + pR_bytes);
    if (doR) {
        if (pR->n_chunks)
            hipLaunchKernelGGL((grad_chunks_kernel<T, NBV>), dim3((unsigned)pR->n_chunks), dim3(kWave),
                               0, s, R->indptr, R->indices, R->values, U, M, n_f, ld, lambda,
                               pR->n_chunks, pR->chunk_row, pR->chunk_begin, pR->chunk_len,
                               pR->chunk_slot, gU, partR, scal, 1, gU != nullptr ? 1 : 0);
        if (pR->n_split_rows)
            hipLaunchKernelGGL((grad_split_kernel<T, NBV>), dim3((unsigned)pR->n_split_rows),
                               dim3(kWave), 0, s, R->indptr, U, n_f, ld, lambda, pR->n_split_rows,
                               pR->split_row, pR->split_slot0, pR->split_nslot, partR, gU,
                               scal + 2 * pR->n_chunks, gU != nullptr ? 1 : 0);
    }
    if (doRt) {
        double *sc = scal + 2 * rowsR;
        if (pRt->n_chunks)
            hipLaunchKernelGGL((grad_chunks_kernel<T, NBV>), dim3((unsigned)pRt->n_chunks),
                               dim3(kWave), 0, s, Rt->indptr, Rt->indices, Rt->values, M, U, n_f,
                               ld, lambda, pRt->n_chunks, pRt->chunk_row, pRt->chunk_begin,
                               pRt->chunk_len, pRt->chunk_slot, gM, partRt, sc, 0,
                               gM != nullptr ? 1 : 0);
        if (pRt->n_split_rows)
            hipLaunchKernelGGL((grad_split_kernel<T, NBV>), dim3((unsigned)pRt->n_split_rows),
                               dim3(kWave), 0, s, Rt->indptr, M, n_f, ld, lambda,
                               pRt->n_split_rows, pRt->split_row, pRt->split_slot0,
                               pRt->split_nslot, partRt, gM, sc + 2 * pRt->n_chunks,
                               gM != nullptr ? 1 : 0);
    }
    if (out2) {
        launch_sum_columns(scal, rowsR + rowsRt, 2, out2, 0, s);
    }
    return hipGetLastError() == hipSuccess ? ALS_OK : ALS_E_HIP;
}

template <typename T, int NBV>
int run_coeffs(Ctx *ctx, const Plan *pR, const als_csr *R, const als_csr *Rt, const T *U,
               const T *M, const T *PU, const T *PM, int n_f, int ld, double lambda,
               double *coeffs, hipStream_t s) {
    const int64_t rows = pR->n_chunks + kItemBlocks;
    int err = ALS_OK;
    double *part = (double *)ctx->workspace((size_t)rows * 5 * sizeof(double), s, &err);
    if (!part) return err;
    if (pR->n_chunks)
        hipLaunchKernelGGL((coeff_chunks_kernel<T, NBV>), dim3((unsigned)pR->n_chunks), dim3(kWave),
                           0, s, R->indptr, R->indices, R->values, U, M, PU, PM, n_f, ld, lambda,
                           pR->n_chunks, pR->chunk_row, pR->chunk_begin, pR->chunk_len, part);
    hipLaunchKernelGGL((coeff_itemreg_kernel<T, NBV>), dim3(kItemBlocks), dim3(256), 0, s,
                       Rt->indptr, Rt->n_rows, M, PM, n_f, ld, lambda, part + 5 * pR->n_chunks);
    launch_sum_columns(part, rows, 5, coeffs, 0, s);
    return hipGetLastError() == hipSuccess ? ALS_OK : ALS_E_HIP;
}

#define ALS_NBV_SWITCH(nbv, CALL) \
    switch (nbv) {                \
        case 1: CALL(1);          \
        case 2: CALL(2);          \
        case 3: CALL(3);          \
        case 4: CALL(4);          \
        case 5: CALL(5);          \
        case 6: CALL(6);          \
        case 7: CALL(7);          \
        case 8: CALL(8);          \
        case 9: CALL(9);          \
        default: return ALS_E_INVAL; \
    }

}  // namespace

int launch_gradient(Ctx *ctx, const Plan *pR, const als_csr *R, const Plan *pRt, const als_csr *Rt,
                    const void *U, const void *M, int n_f, int ld, double lambda, als_dtype dt,
                    void *gU, void *gM, double *out2, hipStream_t s) {
    const int nbv = (n_f + 15) / 16;
#define G32(N) return run_gradient<float, N>(ctx, pR, R, pRt, Rt, (const float *)U, (const float *)M, n_f, ld, lambda, (float *)gU, (float *)gM, out2, s)
#define G64(N) return run_gradient<double, N>(ctx, pR, R, pRt, Rt, (const double *)U, (const double *)M, n_f, ld, lambda, (double *)gU, (double *)gM, out2, s)
    if (dt == ALS_F32) { ALS_NBV_SWITCH(nbv, G32) }
    if (dt == ALS_F64) { ALS_NBV_SWITCH(nbv, G64) }
#undef G32
#undef G64
    return ALS_E_INVAL;
}

int launch_coeffs(Ctx *ctx, const Plan *pR, const als_csr *R, const als_csr *Rt, const void *U,
                  const void *M, const void *pU, const void *pM, int n_f, int ld, double lambda,
                  als_dtype dt, double *coeffs, hipStream_t s) {
    const int nbv = (n_f + 15) / 16;
#define C32(N) return run_coeffs<float, N>(ctx, pR, R, Rt, (const float *)U, (const float *)M, (const float *)pU, (const float *)pM, n_f, ld, lambda, coeffs, s)
#define C64(N) return run_coeffs<double, N>(ctx, pR, R, Rt, (const double *)U, (const double *)M, (const double *)pU, (const double *)pM, n_f, ld, lambda, coeffs, s)
    if (dt == ALS_F32) { ALS_NBV_SWITCH(nbv, C32) }
    if (dt == ALS_F64) { ALS_NBV_SWITCH(nbv, C64) }
#undef C32
#undef C64
    return ALS_E_INVAL;
}

}  // namespace alsncg
