// Reduced-precision half-sweep (the row solve of Eq. (3)/(4) with BF16
// factor copies):
//   * the fixed side is gathered from a BF16 copy and the Gram matrix
//     A~_i = sum y~_j y~_j^T + lambda n_i I (y~ = bf16(y)) is built on
//     v_mfma_f32_16x16x32_bf16 with FP32 accumulation, 32 ratings per MFMA;
//   * the augmented column carries bf16(r_ij), so factorising A~ also gives
//     the forward substitution for v~_i = sum bf16(r_ij) y~_j;
//   * the blocked Cholesky and both substitutions run in FP32 (rowsolve.h);
//   * optionally one step of iterative refinement with the residual taken
//     from the FP32 factors and ratings:
//         x0 = A~^{-1} v~,  res = sum_j (r_ij - y_j . x0) y_j - lambda n_i x0
//         x1 = x0 + A~^{-1} res
//     (res = v - A x0 for the FP32 normal equations; one step contracts the
//     BF16 perturbation of the solution by roughly its own relative size).
// The solution is written in FP32 and, optionally, as a BF16 copy.
//
// Lanes: l = 16 g + c.  For a group of 32 ratings, lane group g owns ratings
// 8 g .. 8 g + 7 and lane c column c of every 16-wide block of the slot
// order (Slots16); the operand of block a is the 8 BF16 values of those
// ratings at that column, which is exactly the A[c][8g..8g+7] (and
// B[8g..8g+7][c]) operand layout of the 16x16x32 MFMA.
//
// Rows split over several chunks run in four stages: partial Gram tiles per
// chunk; fixed-order sum, factorisation and x0 per row (factors kept in the
// workspace); residual partials per chunk at x0; fixed-order sum of the
// residual and the correction per row.
#include <math.h>

#include <climits>

#include "internal.h"
#include "rowsolve.h"

namespace alsncg {
namespace {

typedef float acc4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

__device__ __forceinline__ acc4 mma_bf16(u32x4 a, u32x4 b, acc4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// FP32 -> BF16, round to nearest even (inputs are finite).
__device__ __forceinline__ unsigned bf16_bits(float x) {
    const unsigned u = __float_as_uint(x);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// Slot order of the BF16 Gram.  Slot s = 16 cb + c holds factor column
//   blocks 0 .. 8O-1            : 128 (cb / 8) + 8 c + cb % 8   (one 16-byte load per lane)
//   blocks 8O .. 8O+4Q-1        : 128 O + 4 c + (cb - 8O)       (one 8-byte load)
//   blocks 8O+4Q .. VB-1        : 128 O + 64 Q + 2 c + ...      (one 4-byte load)
//   blocks VB .. NB-1           : s                              (2-byte loads)
// O = (NB-1) / 8, Q and P mark a remaining group of 4 and of 2 blocks.  The
// vector groups cover columns 0 .. 16 VB - 1 <= 16 (NB-1) - 1 < n_f, so every
// column they load is real; block a < VB sits in half (a & 1) of dword a / 2
// of a lane's loaded data.  Slot n_f (last block) is the rating.
template <int NB> struct Slots16 {
    static constexpr int O = (NB - 1) / 8;
    static constexpr int Q = ((NB - 1) - 8 * O) >= 4 ? 1 : 0;
    static constexpr int P = ((NB - 1) - 8 * O - 4 * Q) >= 2 ? 1 : 0;
    static constexpr int VB = 8 * O + 4 * Q + 2 * P;
    static constexpr int DW = VB / 2;     // loaded dwords per rating (vector groups)
    static constexpr int NS = NB - VB;    // 2-byte loads per rating
    __host__ __device__ static constexpr int col(int s) {
        return (s >> 4) < 8 * O ? 128 * ((s >> 4) >> 3) + 8 * (s & 15) + ((s >> 4) & 7)
               : (s >> 4) < 8 * O + 4 * Q ? 128 * O + 4 * (s & 15) + ((s >> 4) - 8 * O)
               : (s >> 4) < VB ? 128 * O + 64 * Q + 2 * (s & 15) + ((s >> 4) - 8 * O - 4 * Q)
                               : s;
    }
};

// Loaded data of one rating for one lane.
template <int NB> struct Raw {
    unsigned d[Slots16<NB>::DW > 0 ? Slots16<NB>::DW : 1];
    unsigned s[Slots16<NB>::NS];
};

// VEC (16-byte aligned rows of a multiple of 8 elements) is a template
// parameter: a run-time choice would put a branch around every load, across
// which the compiler waits for all loads in flight.
template <int NB, bool VEC>
__device__ __forceinline__ void gather16(Raw<NB> &w, const u16 *__restrict__ Y, int j, int ld,
                                         int n_f, int c) {
    typedef Slots16<NB> SL;
    const u16 *row = Y + (int64_t)j * ld;
    if constexpr (VEC) {
#pragma unroll
        for (int q = 0; q < SL::O; ++q) {
            const u32x4 v = *(const u32x4 *)(row + 128 * q + 8 * c);
#pragma unroll
            for (int e = 0; e < 4; ++e) w.d[4 * q + e] = v[e];
        }
        if constexpr (SL::Q == 1) {
            const u32x2 v = *(const u32x2 *)(row + 128 * SL::O + 4 * c);
            w.d[4 * SL::O] = v[0];
            w.d[4 * SL::O + 1] = v[1];
        }
        if constexpr (SL::P == 1) w.d[4 * SL::O + 2 * SL::Q] = *(const unsigned *)(row + 128 * SL::O + 64 * SL::Q + 2 * c);
    } else {
#pragma unroll
        for (int m = 0; m < SL::DW; ++m) {
            const unsigned lo = row[SL::col(16 * (2 * m) + c)];
            const unsigned hi = row[SL::col(16 * (2 * m + 1) + c)];
            w.d[m] = lo | (hi << 16);
        }
    }
#pragma unroll
    for (int k = 0; k < SL::NS; ++k) {
        const int col = 16 * (SL::VB + k) + c;
        w.s[k] = row[col < n_f ? col : n_f - 1];
    }
}

// Operands of one group (8 ratings x NB blocks) from the loaded data, with the
// masks: ratings past the end -> 0, slot n_f -> bf16(r), padding slots -> 0.
// Then one MFMA per upper-triangular tile.
template <int NB>
__device__ __forceinline__ void gram_group(acc4 (&A)[Tri<NB>::NT], const Raw<NB> (&w)[8],
                                           const unsigned (&rb)[8], int s, int g, int c, int last,
                                           int n_f) {
    typedef Slots16<NB> SL;
    unsigned mask[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int t = 32 * s + 8 * g + 2 * m;
        mask[m] = (t <= last ? 0xffffu : 0u) | (t + 1 <= last ? 0xffff0000u : 0u);
    }
    u32x4 op[NB];
#pragma unroll
    for (int a = 0; a < SL::VB; ++a) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const unsigned x0 = w[2 * m].d[a >> 1], x1 = w[2 * m + 1].d[a >> 1];
            const unsigned v = (a & 1) ? ((x0 >> 16) | (x1 & 0xffff0000u))
                                       : ((x0 & 0xffffu) | (x1 << 16));
            op[a][m] = v & mask[m];
        }
    }
#pragma unroll
    for (int k = 0; k < SL::NS; ++k) {
        const int a = SL::VB + k;
        const int col = 16 * a + c;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            unsigned v = (w[2 * m].s[k] & 0xffffu) | (w[2 * m + 1].s[k] << 16);
            if (a == NB - 1) {
                const unsigned rv = rb[2 * m] | (rb[2 * m + 1] << 16);
                v = col < n_f ? v : (col == n_f ? rv : 0u);
            }
            op[a][m] = v & mask[m];
        }
    }
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int bb = a; bb < NB; ++bb) A[Tri<NB>::id(a, bb)] = mma_bf16(op[a], op[bb], A[Tri<NB>::id(a, bb)]);
}

// Gram accumulation over ratings [b, e): group s holds ratings 32 s + 8 g +
// k (clamped to the last rating; masked at use).  Two register buffers
// alternate (the rows of group s + 1 in flight while group s is consumed);
// the ids and values of a group are loaded two steps before its gather
// (rings jq, rq) and the values turned into BF16 bits when the gather is
// issued, so that no wait for an id or a value drains the gathers in flight
// (the wait counter completes loads in issue order).  Single exit; loads
// past the end read valid clamped addresses.
template <int NB, bool VEC>
__device__ __forceinline__ void gram_accumulate16(acc4 (&A)[Tri<NB>::NT],
                                                  const int32_t *__restrict__ idx,
                                                  const float *__restrict__ val, int64_t b,
                                                  int64_t e, const u16 *__restrict__ Y, int ld,
                                                  int n_f, int g, int c) {
    if (b >= e) return;
    const int last = (int)(e - 1 - b);
    const int ng = (last >> 5) + 1;
    const int32_t *ix = idx + b;
    const float *vx = val + b;
    auto pos = [&](int s, int k) { return min(32 * s + 8 * g + k, last); };
    Raw<NB> w[2][8];
    unsigned rb[2][8];
    int jq[2][8];
    float rq[2][8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        gather16<NB, VEC>(w[0][k], Y, ix[pos(0, k)], ld, n_f, c);
        rb[0][k] = bf16_bits(vx[pos(0, k)]);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        jq[1][k] = ix[pos(1, k)];
        rq[1][k] = vx[pos(1, k)];
        jq[0][k] = ix[pos(2, k)];
        rq[0][k] = vx[pos(2, k)];
    }
    for (int s = 0; s < ng; s += 2) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            // group s + h is in w[h]; gather group s + h + 1, then load the
            // ids of group s + h + 3 into the slot that freed
            const int slot = 1 - h;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                gather16<NB, VEC>(w[slot][k], Y, jq[slot][k], ld, n_f, c);
                rb[slot][k] = bf16_bits(rq[slot][k]);
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                jq[slot][k] = ix[pos(s + h + 3, k)];
                rq[slot][k] = vx[pos(s + h + 3, k)];
            }
            // keep the loads above the MFMAs of group s + h (the scheduler
            // would sink them below and serialise the pipeline); not for the
            // widest rows, whose tiles leave no registers for two buffers
            if constexpr (NB <= 7) __builtin_amdgcn_sched_barrier(0);
            if (s + h < ng) gram_group<NB>(A, w[h], rb[h], s + h, g, c, last, n_f);
        }
    }
}

// LDS of the mixed finish (floats).
template <int NB> struct SharedMx {
    static constexpr int NP = NB * 16;
    static constexpr int NV = (NP + 63) / 64;   // float4 column groups per lane in the residual
    static constexpr int NPV = 64 * NV;
    static constexpr int TS = Shared<float, NB>::TS;
    // xs, ys, wsl, z2, dl [NP]; Dt [TS]; Yinv [NB TS]; xn, wn [NPV]; tmp [16]
    static constexpr int size = 5 * NP + TS + NB * TS + 2 * NPV + 16;
};

// One FP32 factor row for the residual: lane c takes columns 64 v + 4 c ..
// + 3.  Loads are unconditional: columns past n_f are clamped into the row
// (their x0 is zero, so they add nothing to the dot product, and
// write_residual drops their sums).  VEC: 16-byte loads (rows of a multiple
// of 4 floats, 16-byte aligned, n_f a multiple of 4 so a vector never
// straddles n_f).
template <int NV, bool VEC>
__device__ __forceinline__ void load_res_row(float (&y)[NV][4], const float *__restrict__ Y32,
                                             int j, int ld, int n_f, int c) {
    const float *row = Y32 + (int64_t)j * ld;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int col = 64 * v + 4 * c;
        if constexpr (VEC) {
            const f4 q4 = *(const f4 *)(row + min(col, n_f - 4));
#pragma unroll
            for (int q = 0; q < 4; ++q) y[v][q] = q4[q];
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) y[v][q] = row[min(col + q, n_f - 1)];
        }
    }
}

// Partial residual sum_j (r_ij - y_j . x0) y_j over ratings [b, e) with FP32
// factors; x0 (natural column order) in xn.  Lane (g, c) takes columns
// 64 v + 4 c .. + 3 of ratings b + g + 4 k; ratings go in blocks of RU per
// lane group.  Two register buffers alternate (the rows of block s + 1 in
// flight while block s is consumed); ids and values are loaded two steps
// before their gather (rings jq, rq), so that no wait drains the gathers in
// flight.  Returns the lane's column sums reduced over the 4 lane groups
// (valid in every group).
template <int NB> struct ResU {
    static constexpr int U = NB <= 5 ? 4 : NB <= 7 ? 1 : 2;
};

template <int NB, bool VEC>
__device__ __forceinline__ void residual_stream(float (&res)[SharedMx<NB>::NV][4],
                                                const int32_t *__restrict__ idx,
                                                const float *__restrict__ val, int64_t b,
                                                int64_t e, const float *__restrict__ Y32, int ld,
                                                int n_f, const float *xn, int g, int c) {
    constexpr int NV = SharedMx<NB>::NV;
    constexpr int U = ResU<NB>::U;
    float xv[NV][4];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int col = 64 * v + 4 * c + q;
            xv[v][q] = col < n_f ? xn[col] : 0.0f;  // zero past n_f masks padding columns
            res[v][q] = 0.0f;
        }
    if (b >= e) return;
    const int64_t last = e - 1;
    // rating of lane group g, block s, slot u: b + g + 4 (U s + u), clamped
    auto at = [&](int64_t s, int u) { return min(b + g + 4 * (U * s + u), last); };
    auto okr = [&](int64_t s, int u) { return b + g + 4 * (U * s + u) <= last; };
    const int64_t nblk = (e - b + 4 * U - 1) / (4 * U);
    float y[2][U][NV][4];
    float rv[2][U], rq[2][U];
    int jq[2][U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        load_res_row<NV, VEC>(y[0][u], Y32, idx[at(0, u)], ld, n_f, c);
        rv[0][u] = val[at(0, u)];
        jq[1][u] = idx[at(1, u)];
        rq[1][u] = val[at(1, u)];
        jq[0][u] = idx[at(2, u)];
        rq[0][u] = val[at(2, u)];
    }
    for (int64_t s0 = 0; s0 < nblk; s0 += 2) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int slot = 1 - h;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                load_res_row<NV, VEC>(y[slot][u], Y32, jq[slot][u], ld, n_f, c);
                rv[slot][u] = rq[slot][u];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                jq[slot][u] = idx[at(s0 + h + 3, u)];
                rq[slot][u] = val[at(s0 + h + 3, u)];
            }
            __builtin_amdgcn_sched_barrier(0);  // keep the loads above the block's FMAs
            if (s0 + h < nblk) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    float dot = 0.0f;
#pragma unroll
                    for (int v = 0; v < NV; ++v)
#pragma unroll
                        for (int q = 0; q < 4; ++q) dot += y[h][u][v][q] * xv[v][q];
                    const float err = okr(s0 + h, u) ? rv[h][u] - sum16(dot) : 0.0f;
#pragma unroll
                    for (int v = 0; v < NV; ++v)
#pragma unroll
                        for (int q = 0; q < 4; ++q) res[v][q] += err * y[h][u][v][q];
                }
            }
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int q = 0; q < 4; ++q) res[v][q] = sum4g(res[v][q]);
}

// Correction x1 = x0 + A~^{-1} (res - lambda n_i x0) on the factor in A /
// Yinv.  resn: residual sums (natural order, without the regulariser) in
// LDS; xs: x0 in slot order; the result replaces xs.
template <int NB>
__device__ __forceinline__ void refine_solve(const acc4 (&A)[Tri<NB>::NT], int n_f, float reg,
                                             float *xs, const float *resn, float *sm) {
    typedef SharedMx<NB> SM;
    typedef Slots16<NB> SL;
    constexpr int NP = SM::NP;
    const int lane = threadIdx.x;
    float *wsl = sm + 2 * NP;
    float *z2 = sm + 3 * NP;
    float *dl = sm + 4 * NP;
    float *Yinv = sm + 5 * NP + SM::TS;
    float *tmp = sm + 5 * NP + SM::TS + NB * SM::TS + 2 * SM::NPV;
    for (int k = lane; k < NP; k += kWave) wsl[k] = k < n_f ? resn[SL::col(k)] - reg * xs[k] : 0.0f;
    __syncthreads();
    forward_solve<float, NB>(A, n_f, wsl, z2, Yinv, tmp);
    back_solve<float, NB>(A, n_f, z2, dl, Yinv);
    for (int k = lane; k < NP; k += kWave) xs[k] += dl[k];
    __syncthreads();
}

template <int NB>
__device__ __forceinline__ void store_row(const float *xs, int64_t row, int n_f, int ld,
                                          float *__restrict__ X32, u16 *__restrict__ X16, bool bad) {
    const int lane = threadIdx.x;
    for (int k = lane; k < n_f; k += kWave) {
        const int col = Slots16<NB>::col(k);
        const float x = bad ? NAN : xs[k];
        X32[row * (int64_t)ld + col] = x;
        if (X16) X16[row * (int64_t)ld + col] = (u16)bf16_bits(x);
    }
}

// Factorise the regularised Gram in A and solve for x0 (slot order, xs).
template <int NB>
__device__ __forceinline__ bool factor_and_solve(acc4 (&A)[Tri<NB>::NT], int n_f, float reg,
                                                 float *sm) {
    typedef SharedMx<NB> SM;
    constexpr int NP = SM::NP;
    const int lane = threadIdx.x, g = lane >> 4, c = lane & 15;
    float *xs = sm, *ys = sm + NP;
    float *Dt = sm + 5 * NP;
    float *Yinv = Dt + SM::TS;
    regularize<float, NB>(A, reg, n_f);
    const bool bad = cholesky_blocked<float, NB>(A, n_f, Dt, Yinv);
    const int caug = n_f - 16 * (NB - 1);
    if (c == caug) {
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int r = 0; r < 4; ++r) ys[16 * a + Mfma<float>::row(g, r)] = A[Tri<NB>::id(a, NB - 1)][r];
    }
    back_solve<float, NB>(A, n_f, ys, xs, Yinv);
    return bad;
}

// x0 (slot order, xs) into natural order (xn).
template <int NB> __device__ __forceinline__ void to_natural(const float *xs, float *xn, int n_f) {
    const int lane = threadIdx.x;
    for (int k = lane; k < SharedMx<NB>::NPV; k += kWave) xn[k] = 0.0f;
    __syncthreads();
    for (int k = lane; k < n_f; k += kWave) xn[Slots16<NB>::col(k)] = xs[k];
    __syncthreads();
}

template <int NB>
__device__ __forceinline__ void write_residual(const float (&res)[SharedMx<NB>::NV][4], float *dst,
                                               int n_f) {
    const int lane = threadIdx.x, g = lane >> 4, c = lane & 15;
    if (g == 0) {
#pragma unroll
        for (int v = 0; v < SharedMx<NB>::NV; ++v)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int col = 64 * v + 4 * c + q;
                dst[col] = col < n_f ? res[v][q] : 0.0f;  // clamped columns carry no data
            }
    }
}

template <int NB> struct OccMx {
    static constexpr int waves = NB <= 4 ? 3 : NB <= 7 ? 2 : 1;
};

struct MixArgs {
    const int64_t *indptr;
    const int32_t *idx;
    const float *val;
    const u16 *Y16;
    const float *Y32;
    float *X32;
    u16 *X16;
    int n_f, ld;
    float lambda;
    int refine, vec16, vec32;
    int64_t *bad_row;
};

template <int NB, bool VEC16>
__global__ __launch_bounds__(64, (OccMx<NB>::waves)) void sweep_mixed_chunks_kernel(
    MixArgs a, int64_t n_chunks, const int32_t *__restrict__ chunk_row,
    const int64_t *__restrict__ chunk_begin, const int32_t *__restrict__ chunk_len,
    const int32_t *__restrict__ chunk_slot, acc4 *__restrict__ partial) {
    typedef Tri<NB> TR;
    typedef SharedMx<NB> SM;
    __shared__ float sm[SM::size];
    const int64_t q = blockIdx.x;
    if (q >= n_chunks) return;
    const int lane = threadIdx.x, g = lane >> 4, c = lane & 15;
    const int64_t row = chunk_row[q];
    const int64_t b = chunk_begin[q];
    const int64_t len = chunk_len[q];
    const int slot = chunk_slot[q];
    acc4 A[TR::NT];
#pragma unroll
    for (int t = 0; t < TR::NT; ++t) A[t] = acc4{0.0f, 0.0f, 0.0f, 0.0f};
    gram_accumulate16<NB, VEC16>(A, a.idx, a.val, b, b + len, a.Y16, a.ld, a.n_f, g, c);
    if (slot >= 0) {
        acc4 *dst = partial + (int64_t)slot * TR::NT * kWave;
#pragma unroll
        for (int t = 0; t < TR::NT; ++t) dst[t * kWave + lane] = A[t];
        return;
    }
    const int n_f = a.n_f;
    const int64_t n_i = len;  // a whole row
    if (n_i == 0) {
        float *xs = sm;
        for (int k = lane; k < n_f; k += kWave) xs[k] = 0.0f;
        __syncthreads();
        store_row<NB>(xs, row, n_f, a.ld, a.X32, a.X16, false);
        return;
    }
    const float reg = a.lambda * (float)n_i;
    const bool bad = factor_and_solve<NB>(A, n_f, reg, sm);
    if (a.refine && !bad) {
        float *xs = sm;
        float *xn = sm + 5 * SM::NP + SM::TS + NB * SM::TS;
        float *wn = xn + SM::NPV;
        to_natural<NB>(xs, xn, n_f);
        float res[SM::NV][4];
        if (a.vec32)
            residual_stream<NB, true>(res, a.idx, a.val, b, b + len, a.Y32, a.ld, n_f, xn, g, c);
        else
            residual_stream<NB, false>(res, a.idx, a.val, b, b + len, a.Y32, a.ld, n_f, xn, g, c);
        write_residual<NB>(res, wn, n_f);
        __syncthreads();
        refine_solve<NB>(A, n_f, reg, xs, wn, sm);
    }
    store_row<NB>(sm, row, n_f, a.ld, a.X32, a.X16, bad);
    if (lane == 0 && bad && a.bad_row) atomicMin((unsigned long long *)a.bad_row, (unsigned long long)row);
}

// Factor store of one split row: the NT factor tiles (lane-major), the NB
// inverted diagonal blocks and a flag.
template <int NB> struct FStore {
    static constexpr size_t tiles = (size_t)Tri<NB>::NT * kWave * 4;  // floats
    static constexpr size_t yinv = (size_t)NB * Shared<float, NB>::TS;
    static constexpr size_t floats = tiles + yinv + 4;
};

// Split rows, stage 2: fixed-order sum of the partial tiles, factorisation,
// x0 (written to X32, and to X16 when there is no refinement); with
// refinement the factor is kept for stage 4.
template <int NB>
__global__ __launch_bounds__(64, (OccMx<NB>::waves)) void sweep_mixed_split_kernel(
    MixArgs a, int64_t n_split, const int32_t *__restrict__ split_row,
    const int32_t *__restrict__ split_slot0, const int32_t *__restrict__ split_nslot,
    const acc4 *__restrict__ partial, float *__restrict__ fstore) {
    typedef Tri<NB> TR;
    typedef SharedMx<NB> SM;
    __shared__ float sm[SM::size];
    const int64_t s = blockIdx.x;
    if (s >= n_split) return;
    const int lane = threadIdx.x;
    const int64_t row = split_row[s];
    const int64_t s0 = split_slot0[s];
    const int ns = split_nslot[s];
    acc4 A[TR::NT];
#pragma unroll
    for (int t = 0; t < TR::NT; ++t) A[t] = acc4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int u = 0; u < ns; ++u) {
        const acc4 *src = partial + (s0 + u) * TR::NT * kWave;
#pragma unroll
        for (int t = 0; t < TR::NT; ++t) A[t] += src[t * kWave + lane];
    }
    const int64_t n_i = a.indptr[row + 1] - a.indptr[row];
    const bool bad = factor_and_solve<NB>(A, a.n_f, a.lambda * (float)n_i, sm);
    store_row<NB>(sm, row, a.n_f, a.ld, a.X32, a.refine ? nullptr : a.X16, bad);
    if (lane == 0 && bad && a.bad_row) atomicMin((unsigned long long *)a.bad_row, (unsigned long long)row);
    if (a.refine) {
        float *fs = fstore + (size_t)s * FStore<NB>::floats;
        acc4 *ft = (acc4 *)fs;
#pragma unroll
        for (int t = 0; t < TR::NT; ++t) ft[t * kWave + lane] = A[t];
        const float *Yinv = sm + 5 * SM::NP + SM::TS;
        for (int k = lane; k < (int)FStore<NB>::yinv; k += kWave) fs[FStore<NB>::tiles + k] = Yinv[k];
        if (lane == 0) fs[FStore<NB>::tiles + FStore<NB>::yinv] = bad ? 1.0f : 0.0f;
    }
}

// Split rows, stage 3: residual partials at x0.  Each split chunk is cut
// into kResPieces pieces of at most ceil(len / kResPieces) ratings, one
// wavefront each (piece p of slot k writes rpart[k * kResPieces + p]), so the
// longest chunk does not leave a latency-bound tail.
constexpr int kResPieces = 8;

template <int NB>
__global__ __launch_bounds__(64) void mixed_residual_kernel(
    MixArgs a, int64_t n_slots, const int32_t *__restrict__ slot_chunk,
    const int32_t *__restrict__ chunk_row, const int64_t *__restrict__ chunk_begin,
    const int32_t *__restrict__ chunk_len, float *__restrict__ rpart) {
    typedef SharedMx<NB> SM;
    __shared__ float xn[SM::NPV];
    const int64_t w = blockIdx.x;
    const int64_t k = w / kResPieces;
    const int piece = (int)(w % kResPieces);
    if (k >= n_slots) return;
    const int lane = threadIdx.x, g = lane >> 4, c = lane & 15;
    const int32_t q = slot_chunk[k];
    const int64_t row = chunk_row[q];
    const int64_t len = chunk_len[q];
    const int64_t per = (len + kResPieces - 1) / kResPieces;
    const int64_t b = chunk_begin[q] + min(len, piece * per);
    const int64_t e = chunk_begin[q] + min(len, (piece + 1) * per);
    for (int i = lane; i < SM::NPV; i += kWave) xn[i] = i < a.n_f ? a.X32[row * (int64_t)a.ld + i] : 0.0f;
    __syncthreads();
    float res[SM::NV][4];
    if (a.vec32)
        residual_stream<NB, true>(res, a.idx, a.val, b, e, a.Y32, a.ld, a.n_f, xn, g, c);
    else
        residual_stream<NB, false>(res, a.idx, a.val, b, e, a.Y32, a.ld, a.n_f, xn, g, c);
    write_residual<NB>(res, rpart + w * (int64_t)SM::NPV, a.n_f);
}

// Split rows, stage 4: fixed-order sum of the residual partials and the
// correction on the stored factor.
template <int NB>
__global__ __launch_bounds__(64, (OccMx<NB>::waves)) void mixed_correct_kernel(
    MixArgs a, int64_t n_split, const int32_t *__restrict__ split_row,
    const int32_t *__restrict__ split_slot0, const int32_t *__restrict__ split_nslot,
    const float *__restrict__ fstore, const float *__restrict__ rpart) {
    typedef Tri<NB> TR;
    typedef SharedMx<NB> SM;
    __shared__ float sm[SM::size];
    const int64_t s = blockIdx.x;
    if (s >= n_split) return;
    const int lane = threadIdx.x;
    const float *fs = fstore + (size_t)s * FStore<NB>::floats;
    if (fs[FStore<NB>::tiles + FStore<NB>::yinv] != 0.0f) return;  // not SPD: x0 = NaN already
    const int64_t row = split_row[s];
    const int64_t s0 = split_slot0[s];
    const int ns = split_nslot[s];
    const int n_f = a.n_f;
    acc4 A[TR::NT];
    const acc4 *ft = (const acc4 *)fs;
#pragma unroll
    for (int t = 0; t < TR::NT; ++t) A[t] = ft[t * kWave + lane];
    float *xs = sm;
    float *Yinv = sm + 5 * SM::NP + SM::TS;
    float *wn = Yinv + NB * SM::TS + SM::NPV;
    for (int k = lane; k < (int)FStore<NB>::yinv; k += kWave) Yinv[k] = fs[FStore<NB>::tiles + k];
    for (int k = lane; k < SM::NP; k += kWave)
        xs[k] = k < n_f ? a.X32[row * (int64_t)a.ld + Slots16<NB>::col(k)] : 0.0f;
    for (int i = lane; i < SM::NPV; i += kWave) {
        float acc = 0.0f;
        for (int u = 0; u < ns * kResPieces; ++u) acc += rpart[(s0 * kResPieces + u) * (int64_t)SM::NPV + i];
        wn[i] = acc;
    }
    __syncthreads();
    const int64_t n_i = a.indptr[row + 1] - a.indptr[row];
    refine_solve<NB>(A, n_f, a.lambda * (float)n_i, xs, wn, sm);
    store_row<NB>(xs, row, n_f, a.ld, a.X32, a.X16, false);
}

__global__ void set_i64_kernel(int64_t *p, int64_t v) { *p = v; }

template <int NB>
int run_mixed(Ctx *ctx, const Plan *plan, const als_csr *R, const MixArgs &a, hipStream_t s) {
    typedef Tri<NB> TR;
    if (a.bad_row) hipLaunchKernelGGL(set_i64_kernel, dim3(1), dim3(1), 0, s, a.bad_row, (int64_t)LLONG_MAX);
    acc4 *partial = nullptr;
    float *fstore = nullptr, *rpart = nullptr;
    if (plan->n_slots > 0) {
        const size_t p_bytes = align_up((size_t)plan->n_slots * TR::NT * kWave * sizeof(acc4), 256);
        const size_t f_bytes = a.refine ? align_up((size_t)plan->n_split_rows * FStore<NB>::floats * 4, 256) : 0;
        const size_t r_bytes = a.refine ? (size_t)plan->n_slots * kResPieces * SharedMx<NB>::NPV * 4 : 0;
        int err = ALS_OK;
        char *ws = (char *)ctx->workspace(p_bytes + f_bytes + r_bytes, s, &err);
        if (!ws) return err;
        partial = (acc4 *)ws;
        fstore = (float *)(ws + p_bytes);
        rpart = (float *)(ws + p_bytes + f_bytes);
    }
    if (plan->n_chunks > 0) {
        if (a.vec16)
            hipLaunchKernelGGL((sweep_mixed_chunks_kernel<NB, true>), dim3((unsigned)plan->n_chunks),
                               dim3(kWave), 0, s, a, plan->n_chunks, plan->chunk_row,
                               plan->chunk_begin, plan->chunk_len, plan->chunk_slot, partial);
        else
            hipLaunchKernelGGL((sweep_mixed_chunks_kernel<NB, false>), dim3((unsigned)plan->n_chunks),
                               dim3(kWave), 0, s, a, plan->n_chunks, plan->chunk_row,
                               plan->chunk_begin, plan->chunk_len, plan->chunk_slot, partial);
    }
    if (plan->n_split_rows > 0) {
        hipLaunchKernelGGL((sweep_mixed_split_kernel<NB>), dim3((unsigned)plan->n_split_rows),
                           dim3(kWave), 0, s, a, plan->n_split_rows, plan->split_row,
                           plan->split_slot0, plan->split_nslot, (const acc4 *)partial, fstore);
        if (a.refine) {
            hipLaunchKernelGGL((mixed_residual_kernel<NB>), dim3((unsigned)(plan->n_slots * kResPieces)), dim3(kWave),
                               0, s, a, plan->n_slots, plan->slot_chunk, plan->chunk_row,
                               plan->chunk_begin, plan->chunk_len, rpart);
            hipLaunchKernelGGL((mixed_correct_kernel<NB>), dim3((unsigned)plan->n_split_rows),
                               dim3(kWave), 0, s, a, plan->n_split_rows, plan->split_row,
                               plan->split_slot0, plan->split_nslot, (const float *)fstore,
                               (const float *)rpart);
        }
    }
    return hipGetLastError() == hipSuccess ? ALS_OK : ALS_E_HIP;
}

__global__ void to_bf16_kernel(int64_t n, const float *__restrict__ x, u16 *__restrict__ y) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        y[i] = (u16)bf16_bits(x[i]);
}

}  // namespace

int launch_sweep_mixed(Ctx *ctx, const Plan *plan, const als_csr *R, const void *Y16,
                       const float *Y32, float *X32, void *X16, int n_f, int ld, double lambda,
                       int refine, int64_t *bad_row, hipStream_t s) {
    MixArgs a;
    a.indptr = R->indptr;
    a.idx = R->indices;
    a.val = (const float *)R->values;
    a.Y16 = (const u16 *)Y16;
    a.Y32 = Y32;
    a.X32 = X32;
    a.X16 = (u16 *)X16;
    a.n_f = n_f;
    a.ld = ld;
    a.lambda = (float)lambda;
    a.refine = refine ? 1 : 0;
    a.vec16 = (ld % 8 == 0 && ((uintptr_t)Y16 % 16) == 0) ? 1 : 0;
    a.vec32 = (!Y32 || (n_f % 4 == 0 && ld % 4 == 0 && ((uintptr_t)Y32 % 16) == 0)) ? 1 : 0;
    a.bad_row = bad_row;
    const int nb = (n_f + 1 + 15) / 16;
    switch (nb) {
        case 1: return run_mixed<1>(ctx, plan, R, a, s);
        case 2: return run_mixed<2>(ctx, plan, R, a, s);
        case 3: return run_mixed<3>(ctx, plan, R, a, s);
        case 4: return run_mixed<4>(ctx, plan, R, a, s);
        case 5: return run_mixed<5>(ctx, plan, R, a, s);
        case 6: return run_mixed<6>(ctx, plan, R, a, s);
        case 7: return run_mixed<7>(ctx, plan, R, a, s);
        case 8: return run_mixed<8>(ctx, plan, R, a, s);
        case 9: return run_mixed<9>(ctx, plan, R, a, s);
        default: return ALS_E_INVAL;
    }
}

int launch_to_bf16(int64_t n, const float *x, void *y, hipStream_t s) {
    if (n <= 0) return ALS_OK;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, s, n, x, (u16 *)y);
    return hipGetLastError() == hipSuccess ? ALS_OK : ALS_E_HIP;
}

}  // namespace alsncg
