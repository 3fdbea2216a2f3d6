// Per-row dense SPD solve on one wavefront, shared by the half-sweep kernels
// (Eq. (3)/(4): x_i = A_i^{-1} v_i with A_i the regularised Gram matrix;
// Cholesky as in Section V-B).
//
// The matrix lives in MFMA accumulator tiles: the upper-triangular 16x16
// tiles (a, b), a <= b, of an NB*16 square, tile id Tri<NB>::id(a, b); lane
// l = 16 g + c of tile (a, b) holds element (16 a + row(g, r), 16 b + c) in
// register r (row() of the MFMA traits).  Only the leading n_f x n_f block
// (the real unknowns) is factorised; rows and columns past n_f are ignored.
//
// After cholesky_blocked():
//   * tile (kb, b), b > kb, holds R(kb, b) of A = R^T R;
//   * tile (kb, kb) holds R_kk (upper triangle);
//   * Yinv + kb * TS holds R_kk^{-T} (lower triangular, row stride 17).
// forward_solve() and back_solve() then solve R^T z = w and R x = z with
// 16x16 mat-vecs against the stored inverses.
#pragma once

#include "internal.h"

namespace alsncg {

// LDS ordering between the steps of a row solve.  WS = false: a workgroup
// barrier (the solving wavefront is the whole workgroup).  WS = true: the
// solving wavefront shares its workgroup with a wavefront doing other work,
// so only the wavefront's own LDS accesses are ordered (a wavefront's LDS
// instructions complete in order; the fences keep the compiler from moving
// accesses across the step).
template <bool WS> __device__ __forceinline__ void row_sync() {
    if constexpr (WS) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

template <int NB> struct Tri {
    static constexpr int NT = NB * (NB + 1) / 2;
    __host__ __device__ static constexpr int id(int a, int b) { return a * NB - a * (a - 1) / 2 + (b - a); }
};

// LDS per wavefront: two vectors of NB*16, one 16x17 transpose tile and the
// NB inverted diagonal factors R_kk^{-T} (16x17 each).
template <typename T, int NB> struct Shared {
    static constexpr int NP = NB * 16;
    static constexpr int TS = 16 * 17;
    static constexpr int size = 2 * NP + TS + NB * TS;
};

// A += reg * I on the real diagonal (slots < n_f).
template <typename T, int NB>
__device__ __forceinline__ void regularize(typename Mfma<T>::acc4 (&A)[Tri<NB>::NT], T reg,
                                           int n_f) {
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (Mfma<T>::row(g, r) == c && 16 * a + c < n_f) A[Tri<NB>::id(a, a)][r] += reg;
}

// Blocked right-looking Cholesky of the leading n_f x n_f block, in place.
// Block row kb: the 16x16 diagonal tile is copied to LDS (Dt) and factored
// together with an identity block, 32 columns = 32 lanes, each lane owning
// one column in 16 registers; row kk of the pivot block is broadcast with
// readlane.  Lanes 0..15 end with the columns of R_kk, lanes 16..31 with
// those of R_kk^{-T}.  The other tiles of the block row then become
// R(kb, b) = R_kk^{-T} A(kb, b), 4 MFMAs each, and the trailing update
// A(a, b) -= R(kb, a)^T R(kb, b) 4 more (the contraction index of an MFMA
// is a free label, so accumulator registers are fed back as operands).
// Returns true when a pivot is not positive (the matrix is not SPD).
template <typename T, int NB, bool WS = false>
__device__ __forceinline__ bool cholesky_blocked(typename Mfma<T>::acc4 (&A)[Tri<NB>::NT],
                                                 int n_f, T *Dt, T *Yinv) {
    typedef Tri<NB> TR;
    typedef Mfma<T> MF;
    constexpr int TS = Shared<T, NB>::TS;
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
    bool bad = false;
#pragma unroll
    for (int kb = 0; kb < NB; ++kb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) Dt[MF::row(g, r) * 17 + c] = A[TR::id(kb, kb)][r];
        row_sync<WS>();
        T p[16];
#pragma unroll
        for (int i = 0; i < 16; ++i)
            p[i] = lane < 16 ? Dt[i * 17 + lane] : (i == (lane & 15) ? T(1) : T(0));
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            if (16 * kb + kk < n_f) {
                // a pivot that is not positive marks the row; the NaN or
                // infinity it leaves in the factor reaches only this row,
                // whose output is replaced by NaN
                const T d = readlane(p[kk], kk);
                bad |= !(d > T(0));
                p[kk] *= inv_sqrt(d);
                T rk[16];  // row kk of the factor, broadcast first, then used
#pragma unroll
                for (int i = kk + 1; i < 16; ++i) rk[i] = readlane(p[kk], i);
#pragma unroll
                for (int i = kk + 1; i < 16; ++i) p[i] -= rk[i] * p[kk];
            }
        }
        row_sync<WS>();
        if (lane < 16) {
#pragma unroll
            for (int i = 0; i < 16; ++i) Dt[i * 17 + lane] = p[i];
        } else if (lane < 32) {
#pragma unroll
            for (int i = 0; i < 16; ++i) Yinv[kb * TS + i * 17 + (lane - 16)] = p[i];
        }
        row_sync<WS>();
#pragma unroll
        for (int r = 0; r < 4; ++r) A[TR::id(kb, kb)][r] = Dt[MF::row(g, r) * 17 + c];
        if (kb + 1 < NB) {
            T aop[4];
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) aop[s4] = Yinv[kb * TS + c * 17 + MF::row(g, s4)];
#pragma unroll
            for (int bb = kb + 1; bb < NB; ++bb) {
                typename Mfma<T>::acc4 t = {T(0), T(0), T(0), T(0)};
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) t = Mfma<T>::mma(aop[s4], A[TR::id(kb, bb)][s4], t);
                A[TR::id(kb, bb)] = t;
            }
        }
#pragma unroll
        for (int a = kb + 1; a < NB; ++a)
#pragma unroll
            for (int bb = a; bb < NB; ++bb)
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4)
                    A[TR::id(a, bb)] = Mfma<T>::mma(-A[TR::id(kb, a)][s4], A[TR::id(kb, bb)][s4],
                                                    A[TR::id(a, bb)]);
        row_sync<WS>();
    }
    return bad;
}

// Back substitution R x = z on the factor left by cholesky_blocked(), block
// by block from the last: z_kb -= R(kb, b) x_b for b > kb, then
// x_kb = R_kk^{-1} z_kb = Y^T z_kb with the stored Y = R_kk^{-T}.
// z, x: LDS vectors of NB*16 in slot order (x must not alias z); slots past
// n_f of x come out zero.
template <typename T, int NB, bool WS = false>
__device__ __forceinline__ void back_solve(const typename Mfma<T>::acc4 (&A)[Tri<NB>::NT],
                                           int n_f, const T *z, T *x, const T *Yinv) {
    typedef Tri<NB> TR;
    typedef Mfma<T> MF;
    constexpr int NP = NB * 16;
    constexpr int TS = Shared<T, NB>::TS;
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
    for (int k = lane; k < NP; k += kWave) x[k] = T(0);
    row_sync<WS>();
#pragma unroll
    for (int kb = NB - 1; kb >= 0; --kb) {
        if (16 * kb < n_f) {
            T part[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int bb = kb + 1; bb < NB; ++bb) {
                const T xv = x[16 * bb + c];
#pragma unroll
                for (int r = 0; r < 4; ++r) part[r] += A[TR::id(kb, bb)][r] * xv;
            }
            T xp = T(0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = MF::row(g, r);
                const T zi = (16 * kb + i < n_f) ? z[16 * kb + i] - sum16(part[r]) : T(0);
                xp += Yinv[kb * TS + i * 17 + c] * zi;
            }
            xp = sum4g(xp);
            if (g == 0 && 16 * kb + c < n_f) x[16 * kb + c] = xp;
            row_sync<WS>();
        }
    }
}

// Forward substitution R^T z = w on the factor left by cholesky_blocked():
// for kb = 0, 1, ...: t = w_kb - sum_{a < kb} R(a, kb)^T z_a, z_kb = R_kk^{-T} t.
// w, z: LDS vectors of NB*16 in slot order (z must not alias w); tmp: 16
// elements of LDS scratch.  Slots past n_f of z come out zero.
template <typename T, int NB, bool WS = false>
__device__ __forceinline__ void forward_solve(const typename Mfma<T>::acc4 (&A)[Tri<NB>::NT],
                                              int n_f, const T *w, T *z, const T *Yinv, T *tmp) {
    typedef Tri<NB> TR;
    typedef Mfma<T> MF;
    constexpr int TS = Shared<T, NB>::TS;
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
#pragma unroll
    for (int kb = 0; kb < NB; ++kb) {
        if (16 * kb < n_f) {
            T t = T(0);
#pragma unroll
            for (int a = 0; a < kb; ++a)
#pragma unroll
                for (int r = 0; r < 4; ++r) t += A[TR::id(a, kb)][r] * z[16 * a + MF::row(g, r)];
            t = sum4g(t);
            if (g == 0) tmp[c] = (16 * kb + c < n_f) ? w[16 * kb + c] - t : T(0);
            row_sync<WS>();
            T zp = T(0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = MF::row(g, r);
                zp += Yinv[kb * TS + c * 17 + j] * tmp[j];
            }
            zp = sum4g(zp);
            if (g == 0) z[16 * kb + c] = (16 * kb + c < n_f) ? zp : T(0);
            row_sync<WS>();
        } else if (g == 0) {
            z[16 * kb + c] = T(0);
        }
    }
    row_sync<WS>();
}

}  // namespace alsncg
