// ALS half-sweep and fold-in kernels (Eq. (3)/(4) of the paper, Section III-A;
// Cholesky solve as in Section V-B).
//
// One wavefront owns one chunk of one row.  The wave gathers the fixed-side
// factor rows of the chunk's ratings straight into registers and
// accumulates the upper-triangular 16x16 tiles of the Gram matrix on the
// MFMA: FP32 in groups of 32 ratings on v_mfma_f32_16x16x32_f16 from
// two-term FP16 splits (gram_split), FP64 in groups of 4 on the FP64
// 16x16x4 MFMA (gram_accumulate).  The gathered row is AUGMENTED with the
// rating value in column n_f, so the same tiles also accumulate
// v_i = sum r_ij y_j (column n_f) and sum r_ij^2; factorising the augmented
// matrix performs the forward substitution R^T z = v for free (z ends up in
// column n_f of the factor).
//
// Register layout of an accumulator tile (a, b) (rows of block a, columns of
// block b, a <= b): lane l = 16 g + c holds element (16 a + row(g, r),
// 16 b + c) in register r (row() of the MFMA traits: 4 g + r for FP32,
// g + 4 r for FP64).  The blocked right-looking Cholesky A = R^T R
// works on that layout directly:
//   * the 16 pivots of block row kb are processed on the VALU, one row of R
//     at a time, the pivot row being broadcast with readlane;
//   * the trailing update A(a, b) -= R(kb, a)^T R(kb, b) is 4 MFMAs per tile,
//     again feeding accumulator registers as MFMA operands (the sum over the
//     16 rows of block kb is order-free).
// Rows longer than the plan's chunk size are split: each chunk stores its
// partial Gram tiles, and a second kernel sums them in chunk order (fixed,
// so results do not depend on scheduling) before the solve.
#include <math.h>

#include <algorithm>
#include <climits>

#include "internal.h"
#include "rowsolve.h"

namespace alsncg {
namespace {

// Slot order of the Gram matrix.  Slot s = 16 cb + c (tile block cb, lane
// column c) holds factor column pi(s):
//   blocks 0 .. 4Q-1      : pi = 64 q + 4 c + e   (cb = 4 q + e)  -- one 16-byte load per lane
//   blocks 4Q .. 4Q+2P-1  : pi = 64 Q + 2 c + e  (cb = 4 Q + e)  -- one 8-byte load
//   remaining blocks      : pi = s                                 -- one 4-byte load each
// with Q = floor((NB-1)/4) and P = 1 when 64 Q + 32 <= 16 (NB-1).  For
// NB = ceil((n_f+1)/16) every column of the first two groups is a real factor
// column, so slots 0..n_f-1 are the n_f factor columns (in permuted order),
// slot n_f is the rating (the augmented column) and the rest is zero padding:
// a symmetric permutation of the real block, which the factorisation does not
// care about; only the row's input and output go through pi.
template <int NB> struct Slots {
    static constexpr int Q = (NB - 1) / 4;
    static constexpr int P = (64 * Q + 32 <= 16 * (NB - 1)) ? 1 : 0;
    __host__ __device__ static constexpr int col(int s) {
        return (s >> 4) < 4 * Q ? 64 * ((s >> 4) >> 2) + 4 * (s & 15) + ((s >> 4) & 3)
               : (s >> 4) < 4 * Q + 2 * P ? 64 * Q + 2 * (s & 15) + ((s >> 4) - 4 * Q)
                                          : s;
    }
};

// Raw gathered operand of one group of 4 ratings: lane (g, c) loads slot
// 16 cb + c of the factor row j of rating t + g.  The load is unconditional
// (j is 0 for ratings past the end of the chunk and columns past n_f are
// clamped into the row) so that no branch or mask sits between a load and its
// use; finish_operand() applies the masks when the MFMAs consume the values.
// VEC: the row is read with 16- and 8-byte loads (FP32, 16-byte aligned
// rows).  It is a template parameter: a run-time choice puts a branch around
// every load, and across such branches the compiler waits for all loads in
// flight right after issuing one, which serialises the gather pipeline.
template <typename T, int NB, bool VEC>
__device__ __forceinline__ void gather_row(T (&gv)[NB], const T *__restrict__ Y, int j, int ld,
                                           int n_f, int c) {
    typedef Slots<NB> SL;
    const T *row = Y + (int64_t)j * ld;
#pragma unroll
    for (int q = 0; q < SL::Q; ++q) {
        const T *p4 = row + 64 * q + 4 * c;
        if constexpr (VEC) {
            static_assert(sizeof(T) == 4, "vector loads of FP32 rows");
            {
                typedef float f4 __attribute__((ext_vector_type(4)));
                const f4 v = *(const f4 *)p4;
#pragma unroll
                for (int e = 0; e < 4; ++e) gv[4 * q + e] = v[e];
                continue;
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) gv[4 * q + e] = p4[e];
    }
    if constexpr (SL::P == 1) {
        const T *p2 = row + 64 * SL::Q + 2 * c;
        if constexpr (VEC) {
            typedef float f2 __attribute__((ext_vector_type(2)));
            const f2 v = *(const f2 *)p2;
            gv[4 * SL::Q] = v[0];
            gv[4 * SL::Q + 1] = v[1];
        } else {
            gv[4 * SL::Q] = p2[0];
            gv[4 * SL::Q + 1] = p2[1];
        }
    }
#pragma unroll
    for (int cb = 4 * SL::Q + 2 * SL::P; cb < NB; ++cb) {
        const int col = cb * 16 + c;
        gv[cb] = row[col < n_f ? col : n_f - 1];
    }
}

// Masks of a gathered operand: zero for ratings past the chunk end, the
// rating value in slot n_f, zero in padding slots.
template <typename T, int NB>
__device__ __forceinline__ void finish_operand(T (&gv)[NB], bool ok, T r, int n_f, int c) {
    typedef Slots<NB> SL;
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
        if (cb < 4 * SL::Q + 2 * SL::P) {
            gv[cb] = ok ? gv[cb] : T(0);
        } else {
            const int col = cb * 16 + c;
            gv[cb] = (col < n_f) ? (ok ? gv[cb] : T(0)) : (col == n_f ? r : T(0));
        }
    }
}

// One MFMA per upper-triangular tile.
template <typename T, int NB>
__device__ __forceinline__ void gram_update(typename Mfma<T>::acc4 (&A)[Tri<NB>::NT],
                                            const T (&gv)[NB]) {
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int bb = a; bb < NB; ++bb)
            A[Tri<NB>::id(a, bb)] = Mfma<T>::mma(gv[a], gv[bb], A[Tri<NB>::id(a, bb)]);
}

// Gram accumulation over ratings [b, e) of one row.  kGramDepth register
// buffers rotate: while the MFMAs consume group s, the factor rows of groups
// s + 1 .. s + kGramDepth - 1 are in flight.  The gather of a group comes
// from L2, the Infinity Cache or HBM and takes several times as long as its
// 4 ratings' MFMAs, so one group in flight per wavefront leaves the matrix
// cores idle most of the time.
//
// Loads complete in issue order as far as the wait counter is concerned:
// waiting for one load waits for every load issued before it.  The rating
// ids (and values) of a group are therefore loaded kGramDepth steps before
// its gather is issued (a ring of ids), so that waiting for an id only
// waits for gathers of groups already consumed, never for those in flight.
// The loop body covers kGramDepth groups with every buffer and ring index
// fixed in each copy, so no register is copied between a load and its use,
// and has a single exit (exits in the middle make the allocator duplicate
// the accumulators); groups past the end are skipped by a uniform branch.
// Loads for groups past the end read valid addresses and are discarded.
constexpr int kGramDepth = 3;

template <typename T, int NB, bool VEC>
__device__ __forceinline__ void gram_accumulate(typename Mfma<T>::acc4 (&A)[Tri<NB>::NT],
                                                const int32_t *__restrict__ idx,
                                                const float *__restrict__ val, int64_t b, int64_t e,
                                                const T *__restrict__ Y, int ld, int n_f, int g,
                                                int c) {
    constexpr int D = kGramDepth;
    if (b >= e) return;
    const int last = (int)(e - 1 - b);
    const int ng = (last >> 2) + 1;
    const int32_t *ix = idx + b;
    const float *vx = val + b;
    T buf[D][NB];
    float rv[D];      // rating of the group in buf[k]
    int jq[D];        // id ring: group X's id in jq[X % D] until its gather is issued
    float rq[D];
#pragma unroll
    for (int k = 0; k < D - 1; ++k) {  // groups 0 .. D - 2: gathered now
        const int p = min(4 * k + g, last);
        rv[k] = vx[p];
        gather_row<T, NB, VEC>(buf[k], Y, ix[p], ld, n_f, c);
    }
#pragma unroll
    for (int x = D - 1; x < 2 * D - 1; ++x) {  // ids of groups D - 1 .. 2 D - 2
        const int p = min(4 * x + g, last);
        jq[x % D] = ix[p];
        rq[x % D] = vx[p];
    }
    for (int s = 0; s < ng; s += D) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            // group s + k is in buf[k]; gather group s + k + D - 1, then load
            // the id of group s + k + 2 D - 1 into the slot that freed
            const int slot = (k + D - 1) % D;
            gather_row<T, NB, VEC>(buf[slot], Y, jq[slot], ld, n_f, c);
            rv[slot] = rq[slot];
            const int p = min(4 * (s + k + 2 * D - 1) + g, last);
            jq[slot] = ix[p];
            rq[slot] = vx[p];
            if (s + k < ng) {
                finish_operand<T, NB>(buf[k], 4 * (s + k) + g <= last, (T)rv[k], n_f, c);
                gram_update<T, NB>(A, buf[k]);
            }
        }
    }
}

// ---------------------------------------------------------------- FP32 Gram on FP16 MFMAs
//
// The FP32 half-sweep accumulates its Gram tiles from two-term FP16 splits
// of the gathered rows on v_mfma_f32_16x16x32_f16 (32 ratings per
// instruction, about 16 cycles; the same 32 ratings take 8 x 32 cycles of
// v_mfma_f32_16x16x4f32).  With x = 2^s y (s = sy for the factor slots from
// max |Y|, s = sr for the rating slot from the chunk's largest rating, so
// that every |x| < 2^14: the FP16 range holds x and its low part stays
// normal for every |x| above 2^-17 of the largest), x = h + m + d where h = fp16(x) and
// m = fp16(x - h), both rounded to nearest: x - h is exact in FP32 and
// |d| <= 2^-22 |x|.  Then
//     x_a x_b ~ h_a h_b + h_a m_b + m_a h_b
// drops m_a m_b (at most 2^-22 |x_a x_b|, unbiased off the diagonal since
// m has either sign); the three products are exact in FP32 and the MFMA
// adds them into FP32 accumulators.  The tiles are scaled back by the
// exact powers of two at the end, so per rating the Gram carries about the
// error of FP32 rounding.
//
// Lanes: l = 16 g + c.  For a group of 32 ratings lane group g owns
// ratings 8 g .. 8 g + 7 and lane c slot 16 a + c of every block a; the
// operand of block a is the 8 FP16 values of those ratings at that slot,
// which is the A[c][8g..8g+7] (and B[8g..8g+7][c]) operand layout of the
// 16x16x32 MFMA.  The slots are those of Slots<NB> (same loads as the
// 16x16x4 path, 8 rows per lane instead of 1), and the rating rides in
// slot n_f: lane c = n_f - 16 (NB - 1) loads it in place of a factor
// element, so no separate value register is kept per rating.
// Largest |r| over the ratings vx[p0 .. p0 + 16 kWave - 1] (clamped at
// last) seen by this lane: 16 loads in flight.
__device__ __forceinline__ float abs_max_step(const float *__restrict__ vx, int p0, int last,
                                              int lane) {
    float v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = vx[min(p0 + kWave * u + lane, last)];
    float m = 0.0f;
#pragma unroll
    for (int u = 0; u < 16; ++u) m = fmaxf(m, fabsf(v[u]));
    return m;
}

// One factor row (slot order of Slots<NB>) for lane c; in the last block the
// lane of slot n_f reads the rating at rp instead.  Loads are unconditional
// (clamped columns; the masks are applied when the operands are built).
template <int NB, bool VEC>
__device__ __forceinline__ void gather_aug(float (&gv)[NB], const float *__restrict__ Y, int j,
                                           int ld, int n_f, int c, const float *rp) {
    typedef Slots<NB> SL;
    static_assert(4 * SL::Q + 2 * SL::P < NB, "the last block is loaded per element");
    const float *row = Y + (int64_t)j * ld;
#pragma unroll
    for (int q = 0; q < SL::Q; ++q) {
        const float *p4 = row + 64 * q + 4 * c;
        if constexpr (VEC) {
            typedef float f4 __attribute__((ext_vector_type(4)));
            const f4 v = *(const f4 *)p4;
#pragma unroll
            for (int e = 0; e < 4; ++e) gv[4 * q + e] = v[e];
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) gv[4 * q + e] = p4[e];
        }
    }
    if constexpr (SL::P == 1) {
        const float *p2 = row + 64 * SL::Q + 2 * c;
        if constexpr (VEC) {
            const float2_t v = *(const float2_t *)p2;
            gv[4 * SL::Q] = v[0];
            gv[4 * SL::Q + 1] = v[1];
        } else {
            gv[4 * SL::Q] = p2[0];
            gv[4 * SL::Q + 1] = p2[1];
        }
    }
#pragma unroll
    for (int cb = 4 * SL::Q + 2 * SL::P; cb < NB - 1; ++cb) gv[cb] = row[cb * 16 + c];
    const int col = (NB - 1) * 16 + c;
    gv[NB - 1] = *(col == n_f ? rp : row + min(col, n_f - 1));
}

// Gram of ratings [b, e) into A (FP32 tiles, unscaled).  One register
// buffer of gathered rows: group t is split into its FP16 operands first,
// which frees the buffer, then the rows of group t + 1 are gathered into it
// and stay in flight while group t's MFMAs run; the ids of group t + 2 are
// loaded after that gather, so waiting for them later never waits for a
// gather issued after them (the wait counter completes loads in issue
// order).  Scheduling barriers keep the three phases in this order (left to
// itself the scheduler sinks the gathers among the MFMAs, and the
// registers of two groups then spill).  Loads past the end of the chunk
// read clamped (valid) positions and are zeroed by the scale.
template <int NB, bool VEC>
__device__ __forceinline__ void gram_split(Mfma<float>::acc4 (&A)[Tri<NB>::NT],
                                           const int32_t *__restrict__ idx,
                                           const float *__restrict__ val, int64_t b, int64_t e,
                                           const float *__restrict__ Y, int ld, int n_f,
                                           unsigned ybits, int g, int c) {
    typedef Tri<NB> TR;
    if (b >= e) return;
    const int last = (int)(e - 1 - b);
    const int ng = (last >> 5) + 1;
    const int32_t *ix = idx + b;
    const float *vx = val + b;
    auto pos = [&](int t, int k) { return min(32 * t + 8 * g + k, last); };
    float buf[8][NB];
    int jq[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) jq[k] = ix[pos(0, k)];
    // the scale needs the largest rating of the chunk: its first loads go
    // out before the first gather, so waiting for them leaves the gather in
    // flight
    float rmax = abs_max_step(vx, 0, last, 16 * g + c);
#pragma unroll
    for (int k = 0; k < 8; ++k)
        gather_aug<NB, VEC>(buf[k], Y, jq[k], ld, n_f, c, vx + pos(0, k));
#pragma unroll
    for (int k = 0; k < 8; ++k) jq[k] = ix[pos(1, k)];
    for (int p0 = 16 * kWave; p0 <= last; p0 += 16 * kWave)
        rmax = fmaxf(rmax, abs_max_step(vx, p0, last, 16 * g + c));
    // factor slots scale by 2^sy (max |Y|), the rating slot by 2^sr (the
    // chunk's largest rating), so that neither magnitude costs the other
    // its low parts; padding slots by 0
    const int sy = split_shift(ybits, 0u);
    const int sr = split_shift(0u, __float_as_uint(wave_max(rmax)));
    const int caug = n_f - 16 * (NB - 1);  // lane of slot n_f in the last block
    const float Sy = exp2i(sy);
    const float Sl = c < caug ? Sy : c == caug ? exp2i(sr) : 0.0f;
    for (int t = 0; t < ng; ++t) {
        const int rem = last - (32 * t + 8 * g);  // ratings k <= rem are real
        u32x4_t hp[NB], lp[NB];
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float sa = a == NB - 1 ? Sl : Sy;
                const float s0 = 2 * i <= rem ? sa : 0.0f, s1 = 2 * i + 1 <= rem ? sa : 0.0f;
                unsigned hi, lo;
                split2(buf[2 * i][a] * s0, buf[2 * i + 1][a] * s1, hi, lo);
                hp[a][i] = hi;
                lp[a][i] = lo;
            }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            gather_aug<NB, VEC>(buf[k], Y, jq[k], ld, n_f, c, vx + pos(t + 1, k));
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int bb = a; bb < NB; ++bb) A[TR::id(a, bb)] = mma_f16(hp[a], hp[bb], A[TR::id(a, bb)]);
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int bb = a; bb < NB; ++bb) A[TR::id(a, bb)] = mma_f16(hp[a], lp[bb], A[TR::id(a, bb)]);
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int bb = a; bb < NB; ++bb) A[TR::id(a, bb)] = mma_f16(lp[a], hp[bb], A[TR::id(a, bb)]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < 8; ++k) jq[k] = ix[pos(t + 2, k)];
    }
    // scale back: 2^-2sy (factor x factor), 2^-(sy+sr) (factor x rating),
    // 2^-2sr (rating x rating); the rating is row and column n_f
    const float Fyy = exp2i(-2 * sy), Fyr = exp2i(-sy - sr), Frr = exp2i(-2 * sr);
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int bb = a; bb < NB; ++bb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float f = Fyy;
                if (bb == NB - 1) {
                    const bool rrow = a == NB - 1 && Mfma<float>::row(g, r) == caug;
                    const bool rcol = c == caug;
                    f = rrow ? (rcol ? Frr : Fyr) : (rcol ? Fyr : Fyy);
                }
                A[TR::id(a, bb)][r] *= f;
            }
}

// ---------------------------------------------------------------- split copy of the fixed side
//
// A planned FP32 half-sweep splits the fixed side once per call instead of
// once per gathered rating.  Row j of the copy holds, for lane c of a 16-lane
// group and block a < NB, the dword (h, m) of x = 2^sy Y[j][col(16 a + c)]
// (h = fp16(x) in the low half, m = fp16(x - h) in the high half: the values
// the split in the Gram loop forms), and zero for slots at or past n_f.  A
// lane's part is LW dwords (NB rounded up to whole 16-byte vectors), a row
// 16 LW dwords; one more row of zeros (row n) stands in for the positions
// past the end of a chunk.
template <int NB> struct SplitRow {
    static constexpr int LW = (NB + 3) / 4 * 4;
    static constexpr int W = 16 * LW;
};

template <int NB>
__global__ __launch_bounds__(256) void presplit_kernel(const float *__restrict__ Y, int64_t n,
                                                       int n_f, int ld,
                                                       const unsigned *__restrict__ ybits,
                                                       unsigned *__restrict__ Yp) {
    typedef SplitRow<NB> SR;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (n + 1) * 16) return;
    const int64_t j = t >> 4;
    const int c = (int)(t & 15);
    const float Sy = exp2i(split_shift(*ybits, 0u));
    const float *row = Y + j * ld;
    unsigned d[SR::LW];
#pragma unroll
    for (int a = 0; a < SR::LW; ++a) {
        const int k = 16 * a + c;
        const float x = (j < n && a < NB && k < n_f) ? row[Slots<NB>::col(k)] * Sy : 0.0f;
        unsigned hi, lo;
        split2(x, 0.0f, hi, lo);
        d[a] = (hi & 0xffffu) | (lo << 16);
    }
    u32x4_t *dst = (u32x4_t *)(Yp + j * SR::W + c * SR::LW);
#pragma unroll
    for (int q = 0; q < SR::LW / 4; ++q) dst[q] = u32x4_t{d[4 * q], d[4 * q + 1], d[4 * q + 2], d[4 * q + 3]};
}

typedef unsigned u32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned u32x3_t __attribute__((ext_vector_type(3)));

// The NB dwords of a lane's part of a row at byte offset `off` of Yp (the
// copy is smaller than 4 GiB: a 32-bit offset from a uniform base).
template <int NB>
__device__ __forceinline__ void gather_split(unsigned (&d)[NB], const unsigned *__restrict__ Yp,
                                             unsigned off) {
    const unsigned *p = (const unsigned *)((const char *)Yp + off);
#pragma unroll
    for (int q = 0; q < NB / 4; ++q) {
        const u32x4_t v = *(const u32x4_t *)(p + 4 * q);
#pragma unroll
        for (int e = 0; e < 4; ++e) d[4 * q + e] = v[e];
    }
    constexpr int o = NB / 4 * 4;
    if constexpr (NB % 4 == 3) {
        const u32x3_t v = *(const u32x3_t *)(p + o);
        d[o] = v[0];
        d[o + 1] = v[1];
        d[o + 2] = v[2];
    } else if constexpr (NB % 4 == 2) {
        const u32x2_t v = *(const u32x2_t *)(p + o);
        d[o] = v[0];
        d[o + 1] = v[1];
    } else if constexpr (NB % 4 == 1) {
        d[o] = p[o];
    }
}

// gram_split over the split copy Yp (n_y rows and the zero row n_y): the
// same lanes, scales, MFMAs and unscaling, with the operands of a group of 32
// ratings formed from the 8 gathered rows of a lane by byte permutes (the h
// halves of ratings 2 i and 2 i + 1 at one slot into one dword, the m halves
// into another) instead of three instructions of split per value.  The
// rating slot (lane n_f - 16 (NB - 1) of the last block, zero in the copy) is
// split in the loop with the chunk's scale.  Positions past the end of the
// chunk gather the zero row and a zero rating.  Yields the same Gram, bit for
// bit, as gram_split.
template <int NB>
__device__ __forceinline__ void gram_split_pre(Mfma<float>::acc4 (&A)[Tri<NB>::NT],
                                               const int32_t *__restrict__ idx,
                                               const float *__restrict__ val, int64_t b, int64_t e,
                                               const unsigned *__restrict__ Yp, int n_y, int n_f,
                                               unsigned ybits, int g, int c) {
    typedef Tri<NB> TR;
    typedef SplitRow<NB> SR;
    if (b >= e) return;
    const int last = (int)(e - 1 - b);
    const int ng = (last >> 5) + 1;
    const int32_t *ix = idx + b;
    const float *vx = val + b;
    auto at = [&](int t, int k) { return 32 * t + 8 * g + k; };
    auto pos = [&](int t, int k) { return (unsigned)min(at(t, k), last); };
    const unsigned lane_off = (unsigned)c * SR::LW * 4u;
    // byte offset of the gathered part of position (t, k) holding id j
    auto offset = [&](int t, int k, int j) {
        return (unsigned)(at(t, k) <= last ? j : n_y) * (unsigned)(SR::W * 4) + lane_off;
    };
    unsigned raw[8][NB];
    float rv[8];
    int jq[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) jq[k] = ix[pos(0, k)];
    float rmax = abs_max_step(vx, 0, last, 16 * g + c);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        gather_split<NB>(raw[k], Yp, offset(0, k, jq[k]));
        rv[k] = vx[pos(0, k)];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) jq[k] = ix[pos(1, k)];
    for (int p0 = 16 * kWave; p0 <= last; p0 += 16 * kWave)
        rmax = fmaxf(rmax, abs_max_step(vx, p0, last, 16 * g + c));
    const int sy = split_shift(ybits, 0u);
    const int sr = split_shift(0u, __float_as_uint(wave_max(rmax)));
    const int caug = n_f - 16 * (NB - 1);  // lane of slot n_f in the last block
    const bool rlane = c == caug;
    const float Sr = exp2i(sr);
    for (int t = 0; t < ng; ++t) {
        u32x4_t hp[NB], lp[NB];
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                hp[a][i] = __builtin_amdgcn_perm(raw[2 * i + 1][a], raw[2 * i][a], 0x05040100u);
                lp[a][i] = __builtin_amdgcn_perm(raw[2 * i + 1][a], raw[2 * i][a], 0x07060302u);
            }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float r0 = at(t, 2 * i) <= last ? rv[2 * i] : 0.0f;
            const float r1 = at(t, 2 * i + 1) <= last ? rv[2 * i + 1] : 0.0f;
            unsigned rh, rl;
            split2(r0 * Sr, r1 * Sr, rh, rl);
            hp[NB - 1][i] = rlane ? rh : hp[NB - 1][i];
            lp[NB - 1][i] = rlane ? rl : lp[NB - 1][i];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            gather_split<NB>(raw[k], Yp, offset(t + 1, k, jq[k]));
            rv[k] = vx[pos(t + 1, k)];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int bb = a; bb < NB; ++bb) A[TR::id(a, bb)] = mma_f16(hp[a], hp[bb], A[TR::id(a, bb)]);
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int bb = a; bb < NB; ++bb) A[TR::id(a, bb)] = mma_f16(hp[a], lp[bb], A[TR::id(a, bb)]);
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int bb = a; bb < NB; ++bb) A[TR::id(a, bb)] = mma_f16(lp[a], hp[bb], A[TR::id(a, bb)]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < 8; ++k) jq[k] = ix[pos(t + 2, k)];
    }
    const float Fyy = exp2i(-2 * sy), Fyr = exp2i(-sy - sr), Frr = exp2i(-2 * sr);
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int bb = a; bb < NB; ++bb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float f = Fyy;
                if (bb == NB - 1) {
                    const bool rrow = a == NB - 1 && Mfma<float>::row(g, r) == caug;
                    const bool rcol = c == caug;
                    f = rrow ? (rcol ? Frr : Fyr) : (rcol ? Fyr : Fyy);
                }
                A[TR::id(a, bb)][r] *= f;
            }
}

// Regularise, optionally form the gradient 2 (A x_in - v), factorise, solve
// and store one row.  `sm` is Shared<T, NB>::size elements of LDS.
template <typename T, int NB, bool WS = false>
__device__ __forceinline__ void finish_row(typename Mfma<T>::acc4 (&A)[Tri<NB>::NT], int64_t row,
                                           int64_t n_i, T *__restrict__ X, int n_f, int ld,
                                           T lambda, const T *__restrict__ X_at,
                                           T *__restrict__ grad_out,
                                           int64_t *__restrict__ bad_row,
                                           int32_t *__restrict__ status, int empty_status, T *sm) {
    typedef Tri<NB> TR;
    typedef Mfma<T> MF;
    constexpr int NP = NB * 16;
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
    T *xs = sm;
    T *ys = sm + NP;
    T *w = sm + 2 * NP;  // v during the gradient (shares space with the factor scratch)
    T *xrow = X + row * (int64_t)ld;

    if (n_i == 0) {
        for (int k = lane; k < n_f; k += kWave) {
            xrow[k] = T(0);
            if (grad_out) grad_out[row * (int64_t)ld + k] = T(0);
        }
        if (status && lane == 0) status[row] = empty_status;
        return;
    }
    regularize<T, NB>(A, lambda * (T)n_i, n_f);

    const int caug = n_f - 16 * (NB - 1);  // lane column of the augmented column

    if (grad_out) {
        // y = A x_in (A symmetric, upper tiles only), then g = 2 (y - v).
        const T *xin = X_at ? X_at + row * (int64_t)ld : xrow;
        for (int k = lane; k < NP; k += kWave) xs[k] = (k < n_f) ? xin[Slots<NB>::col(k)] : T(0);
        row_sync<WS>();
        // row-block a of A x: tiles (a, b >= a) times x_b, reduced over the 16
        // lanes of a quarter-wave as soon as the block row is done; the
        // transposed contributions of the upper tiles to block b collect in cacc
        T cacc[NB];
#pragma unroll
        for (int a = 0; a < NB; ++a) cacc[a] = T(0);
#pragma unroll
        for (int a = 0; a < NB; ++a) {
            T racc[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int bb = a; bb < NB; ++bb) {
                const T xv = xs[16 * bb + c];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    racc[r] += A[TR::id(a, bb)][r] * xv;
                    if (a < bb) cacc[bb] += A[TR::id(a, bb)][r] * xs[16 * a + MF::row(g, r)];
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const T v = sum16(racc[r]);
                if (c == 0) ys[16 * a + MF::row(g, r)] = v;
            }
        }
#pragma unroll
        for (int a = 0; a < NB; ++a) cacc[a] = sum4g(cacc[a]);
        if (c == caug) {
#pragma unroll
            for (int a = 0; a < NB; ++a)
#pragma unroll
                for (int r = 0; r < 4; ++r) w[16 * a + MF::row(g, r)] = A[TR::id(a, NB - 1)][r];
        }
        row_sync<WS>();
        if (g == 0) {
#pragma unroll
            for (int a = 0; a < NB; ++a) ys[16 * a + c] += cacc[a];
        }
        row_sync<WS>();
        for (int k = lane; k < n_f; k += kWave)
            grad_out[row * (int64_t)ld + Slots<NB>::col(k)] = T(2) * (ys[k] - w[k]);
        row_sync<WS>();
    }

    // ---- blocked Cholesky A = R^T R of the augmented matrix (pivots 0 .. n_f-1);
    // column n_f of the factor is then z with R^T z = v.
    T *Dt = sm + 2 * NP;
    T *Yinv = Dt + Shared<T, NB>::TS;
    const bool bad = cholesky_blocked<T, NB, WS>(A, n_f, Dt, Yinv);

    // ---- back substitution R x = z
    if (c == caug) {
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int r = 0; r < 4; ++r) ys[16 * a + MF::row(g, r)] = A[TR::id(a, NB - 1)][r];
    }
    back_solve<T, NB, WS>(A, n_f, ys, xs, Yinv);
    for (int k = lane; k < n_f; k += kWave) xrow[Slots<NB>::col(k)] = bad ? T(NAN) : xs[k];
    if (lane == 0) {
        if (bad && bad_row) atomicMin((unsigned long long *)bad_row, (unsigned long long)row);
        if (status) status[row] = bad ? (int32_t)ALS_E_NOT_SPD : 0;
    }
}

// One chunk per 64-lane workgroup.  chunk_row == nullptr: chunk q is row q
// in full (fold-in and unplanned use).
// Two resident wavefronts per SIMD where the tiles fit in 256 registers
// (one runs its MFMA Gram while the other factorises).
template <typename T, int NB> struct Occ {
    static constexpr int waves = (sizeof(T) == 4 ? NB <= 7 : NB <= 4) ? 2 : 1;
};

// One chunk: Gram of its ratings, then either the partial tiles (split row)
// or the row solve.
template <typename T, int NB, bool VEC, bool PRE>
__device__ __forceinline__ void sweep_chunk(
    int64_t q, const int64_t *__restrict__ indptr, const int32_t *__restrict__ idx,
    const float *__restrict__ val, const T *__restrict__ Y, const unsigned *__restrict__ ybits,
    const unsigned *__restrict__ Yp, int n_y,
    T *__restrict__ X, int n_f, int ld,
    T lambda, const int32_t *__restrict__ chunk_row, const int64_t *__restrict__ chunk_begin,
    const int32_t *__restrict__ chunk_len, const int32_t *__restrict__ chunk_slot,
    typename Mfma<T>::acc4 *__restrict__ partial, const T *__restrict__ X_at,
    T *__restrict__ grad_out, int64_t *__restrict__ bad_row, int32_t *__restrict__ status,
    int empty_status, T *sm) {
    typedef typename Mfma<T>::acc4 acc4;
    typedef Tri<NB> TR;
    const int lane = threadIdx.x, g = lane >> 4, c = lane & 15;
    int64_t row, b, len;
    int slot;
    if (chunk_row) {
        row = chunk_row[q];
        b = chunk_begin[q];
        len = chunk_len[q];
        slot = chunk_slot[q];
    } else {
        row = q;
        b = indptr[q];
        len = indptr[q + 1] - b;
        slot = -1;
    }
    acc4 A[TR::NT];
#pragma unroll
    for (int t = 0; t < TR::NT; ++t) A[t] = acc4{T(0), T(0), T(0), T(0)};
    if constexpr (sizeof(T) == 4 && PRE)
        gram_split_pre<NB>(A, idx, val, b, b + len, Yp, n_y, n_f, *ybits, g, c);
    else if constexpr (sizeof(T) == 4)
        gram_split<NB, VEC>(A, idx, val, b, b + len, Y, ld, n_f, *ybits, g, c);
    else
        gram_accumulate<T, NB, VEC>(A, idx, val, b, b + len, Y, ld, n_f, g, c);
    if (slot >= 0) {
        acc4 *dst = partial + (int64_t)slot * TR::NT * kWave;
#pragma unroll
        for (int t = 0; t < TR::NT; ++t) dst[t * kWave + lane] = A[t];
        return;
    }
    const int64_t n_i = indptr[row + 1] - indptr[row];
    finish_row<T, NB>(A, row, n_i, X, n_f, ld, lambda, X_at, grad_out, bad_row, status,
                      empty_status, sm);
}

// One chunk per 64-lane workgroup (PERSIST = false), or a persistent grid
// striding over the chunks (PERSIST = true; chunks are ordered longest
// first, so the stride deals them out like a greedy schedule).
// chunk_row == nullptr: chunk q is row q in full (fold-in and unplanned use).
// PRE (FP32): the Gram reads the split copy Yp of Y instead of Y.
template <typename T, int NB, bool PERSIST, bool VEC, bool PRE = false>
__global__ __launch_bounds__(64, (Occ<T, NB>::waves)) void sweep_chunks_kernel(
    const int64_t *__restrict__ indptr, const int32_t *__restrict__ idx,
    const float *__restrict__ val, const T *__restrict__ Y, const unsigned *__restrict__ ybits,
    const unsigned *__restrict__ Yp, int n_y,
    T *__restrict__ X, int n_f, int ld,
    T lambda, int64_t n_chunks, const int32_t *__restrict__ chunk_row,
    const int64_t *__restrict__ chunk_begin, const int32_t *__restrict__ chunk_len,
    const int32_t *__restrict__ chunk_slot, typename Mfma<T>::acc4 *__restrict__ partial,
    const T *__restrict__ X_at, T *__restrict__ grad_out, int64_t *__restrict__ bad_row,
    int32_t *__restrict__ status, int empty_status) {
    __shared__ T sm[Shared<T, NB>::size];
    if constexpr (PERSIST) {
        for (int64_t q = blockIdx.x; q < n_chunks; q += gridDim.x)
            sweep_chunk<T, NB, VEC, PRE>(q, indptr, idx, val, Y, ybits, Yp, n_y, X, n_f, ld, lambda, chunk_row,
                                    chunk_begin, chunk_len, chunk_slot, partial, X_at, grad_out,
                                    bad_row, status, empty_status, sm);
    } else {
        const int64_t q = blockIdx.x;
        if (q >= n_chunks) return;
        sweep_chunk<T, NB, VEC, PRE>(q, indptr, idx, val, Y, ybits, Yp, n_y, X, n_f, ld, lambda, chunk_row,
                                chunk_begin, chunk_len, chunk_slot, partial, X_at, grad_out,
                                bad_row, status, empty_status, sm);
    }
}

// Second stage for rows split over several chunks: fixed-order sum of the
// partial Gram tiles, then the row solve.
template <typename T, int NB>
__global__ __launch_bounds__(64, (Occ<T, NB>::waves)) void sweep_split_kernel(
    const int64_t *__restrict__ indptr, T *__restrict__ X, int n_f, int ld, T lambda,
    int64_t n_split, const int32_t *__restrict__ split_row, const int32_t *__restrict__ split_slot0,
    const int32_t *__restrict__ split_nslot, const typename Mfma<T>::acc4 *__restrict__ partial,
    const T *__restrict__ X_at, T *__restrict__ grad_out, int64_t *__restrict__ bad_row,
    int32_t *__restrict__ status) {
    typedef typename Mfma<T>::acc4 acc4;
    typedef Tri<NB> TR;
    __shared__ T sm[Shared<T, NB>::size];
    const int64_t s = blockIdx.x;
    if (s >= n_split) return;
    const int lane = threadIdx.x;
    const int64_t row = split_row[s];
    const int64_t s0 = split_slot0[s];
    const int ns = split_nslot[s];
    acc4 A[TR::NT];
#pragma unroll
    for (int t = 0; t < TR::NT; ++t) A[t] = acc4{T(0), T(0), T(0), T(0)};
    for (int u = 0; u < ns; ++u) {
        const acc4 *src = partial + (s0 + u) * TR::NT * kWave;
#pragma unroll
        for (int t = 0; t < TR::NT; ++t) A[t] += src[t * kWave + lane];
    }
    const int64_t n_i = indptr[row + 1] - indptr[row];
    finish_row<T, NB>(A, row, n_i, X, n_f, ld, lambda, X_at, grad_out, bad_row, status, 0, sm);
}

__global__ void set_i64_kernel(int64_t *p, int64_t v) { *p = v; }
__global__ void set_u32_kernel(unsigned *p, unsigned v) { *p = v; }

// Bit pattern of the largest finite |y| over the n x n_f block of Y (row
// stride ld): the integer order of the bit patterns of non-negative finite
// floats is their numeric order, so the maximum is exact and independent of
// the schedule (a non-finite entry poisons only the rows that rate it, not
// the scale of every row).  A wavefront takes 8 rows per step, lanes over the columns
// (n_f <= 192), loads clamped into the block; each workgroup writes its
// maximum to part[blockIdx.x] and one more workgroup reduces the parts (no
// atomics: thousands of them on one address serialise at L2).
constexpr int kAbsMaxRows = 8;
__global__ __launch_bounds__(256) void abs_max_bits_kernel(const float *__restrict__ Y, int64_t n,
                                                           int n_f, int ld,
                                                           unsigned *__restrict__ part) {
    __shared__ unsigned red[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int nq = (n_f + kWave - 1) / kWave;
    unsigned m = 0u;
    for (int64_t r0 = w0 * kAbsMaxRows; r0 < n; r0 += nw * kAbsMaxRows) {
        unsigned v[kAbsMaxRows][3];
#pragma unroll
        for (int u = 0; u < kAbsMaxRows; ++u)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int64_t r = min(r0 + u, n - 1);
                const int col = min(lane + kWave * min(q, nq - 1), n_f - 1);
                const unsigned a = __float_as_uint(Y[r * ld + col]) & 0x7fffffffu;
                v[u][q] = a < 0x7f800000u ? a : 0u;  // non-finite entries do not set the scale
            }
#pragma unroll
        for (int u = 0; u < kAbsMaxRows; ++u)
#pragma unroll
            for (int q = 0; q < 3; ++q) m = max(m, v[u][q]);
    }
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) m = max(m, (unsigned)__shfl_xor((int)m, o));
    if (lane == 0) red[wv] = m;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = max(max(red[0], red[1]), max(red[2], red[3]));
}

__global__ __launch_bounds__(256) void abs_max_final_kernel(const unsigned *__restrict__ part,
                                                            int n_part, unsigned *out) {
    __shared__ unsigned red[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    unsigned m = 0u;
    for (int k = threadIdx.x; k < n_part; k += blockDim.x) m = max(m, part[k]);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) m = max(m, (unsigned)__shfl_xor((int)m, o));
    if (lane == 0) red[wv] = m;
    __syncthreads();
    if (threadIdx.x == 0) *out = max(max(red[0], red[1]), max(red[2], red[3]));
}

// FP32: ybits holds the bits of max |Y| (abs_max_bits_kernel); null: it is
// computed here into the context's word first (over the R->n_cols rows of Y).
template <typename T, int NB, bool VEC>
int run_sweep_v(Ctx *ctx, const Plan *plan, const als_csr *R, const T *Y, const unsigned *ybits,
                T *X, int n_f, int ld, T lambda, const T *X_at, T *grad_out, int64_t *bad_row,
                int32_t *status, int empty_status, int64_t n_rows_unplanned, void *partial_ext,
                hipStream_t s) {
    typedef typename Mfma<T>::acc4 acc4;
    typedef Tri<NB> TR;
    if constexpr (sizeof(T) == 4) {
        if (!ybits) {
            if (!ctx || !ctx->ybits) return ALS_E_INVAL;
            const int rc = launch_abs_max_bits((const float *)Y, R->n_cols, n_f, ld, ctx->ybits, s);
            if (rc != ALS_OK) return rc;
            ybits = ctx->ybits;
        }
    }
    if (bad_row) hipLaunchKernelGGL(set_i64_kernel, dim3(1), dim3(1), 0, s, bad_row, (int64_t)LLONG_MAX);
    if (!plan) {
        if (n_rows_unplanned > 0)
            hipLaunchKernelGGL((sweep_chunks_kernel<T, NB, false, VEC>), dim3((unsigned)n_rows_unplanned),
                               dim3(kWave), 0, s, R->indptr, R->indices, R->values, Y, ybits,
                               (const unsigned *)nullptr, 0, X,
                               n_f, ld, lambda, n_rows_unplanned, nullptr, nullptr, nullptr,
                               nullptr, (acc4 *)nullptr, X_at, grad_out, bad_row, status,
                               empty_status);
        return hipGetLastError() == hipSuccess ? ALS_OK : ALS_E_HIP;
    }
    acc4 *partial = (acc4 *)partial_ext;
    if (plan->n_slots > 0 && !partial) {
        int err = ALS_OK;
        partial = (acc4 *)ctx->workspace((size_t)plan->n_slots * TR::NT * kWave * sizeof(acc4), s, &err);
        if (!partial) return err;
    }
    // the plan's dual-form bins (the last n_dual chunks) go to their own
    // kernels; with lambda = 0 every row keeps the n_f x n_f form
    const bool dual = plan->n_dual > 0 && lambda > T(0) && !status;
    const int64_t n_main = dual ? plan->n_chunks - plan->n_dual : plan->n_chunks;
    // FP32 with a context: split the fixed side once into the context's copy
    const unsigned *Yp = nullptr;
    if constexpr (sizeof(T) == 4) {
        const size_t bytes = (size_t)(R->n_cols + 1) * SplitRow<NB>::W * sizeof(unsigned);
        const bool want = plan->split_copy > 0 || (plan->split_copy < 0 && SplitRow<NB>::W <= ld);
        if (want && ctx && n_main > 0 && bytes <= (size_t(1) << 32)) {
            int err = ALS_OK;
            unsigned *cp = (unsigned *)ctx->split_buffer(bytes, s, &err);
            if (!cp) return err;
            const int64_t nt = (R->n_cols + 1) * 16;
            hipLaunchKernelGGL((presplit_kernel<NB>), dim3((unsigned)((nt + 255) / 256)), dim3(256), 0,
                               s, (const float *)Y, R->n_cols, n_f, ld, ybits, cp);
            Yp = cp;
        }
    }
#define ALS_MAIN(P, V, PR)                                                                         \
    hipLaunchKernelGGL((sweep_chunks_kernel<T, NB, P, V, PR>),                                     \
                       dim3((unsigned)(P ? std::min<int64_t>(plan->grid, n_main) : n_main)),        \
                       dim3(kWave), 0, s, R->indptr, R->indices, R->values, Y, ybits, Yp,          \
                       (int)R->n_cols, X, n_f,                                                     \
                       ld, lambda, n_main, plan->chunk_row, plan->chunk_begin, plan->chunk_len,     \
                       plan->chunk_slot, partial, X_at, grad_out, bad_row, status, empty_status)
    bool launched = false;
    if constexpr (sizeof(T) == 4) {
        if (n_main > 0 && Yp) {
            if (plan->grid > 0)
                ALS_MAIN(true, false, true);
            else
                ALS_MAIN(false, false, true);
            launched = true;
        }
    }
    if (n_main > 0 && !launched) {
        if (plan->grid > 0) {
            ALS_MAIN(true, VEC, false);
        } else {
            ALS_MAIN(false, VEC, false);
        }
    }
#undef ALS_MAIN
    if (dual) {
        const int rc = launch_sweep_dual(plan, R, Y, X, n_f, ld, (double)lambda, Mfma<T>::kDtype,
                                         X_at, grad_out, bad_row, s);
        if (rc != ALS_OK) return rc;
    }
    if (plan->n_split_rows > 0)
        hipLaunchKernelGGL((sweep_split_kernel<T, NB>), dim3((unsigned)plan->n_split_rows),
                           dim3(kWave), 0, s, R->indptr, X, n_f, ld, lambda, plan->n_split_rows,
                           plan->split_row, plan->split_slot0, plan->split_nslot, partial, X_at,
                           grad_out, bad_row, status);
    return hipGetLastError() == hipSuccess ? ALS_OK : ALS_E_HIP;
}

template <typename T, int NB>
int run_sweep(Ctx *ctx, const Plan *plan, const als_csr *R, const T *Y, const unsigned *ybits,
              T *X, int n_f, int ld, T lambda, const T *X_at, T *grad_out, int64_t *bad_row,
              int32_t *status, int empty_status, int64_t n_rows_unplanned, void *partial_ext,
              hipStream_t s) {
    if constexpr (sizeof(T) == 4) {
        if (ld % 4 == 0 && ((uintptr_t)Y % 16) == 0)
            return run_sweep_v<T, NB, true>(ctx, plan, R, Y, ybits, X, n_f, ld, lambda, X_at,
                                            grad_out, bad_row, status, empty_status,
                                            n_rows_unplanned, partial_ext, s);
    }
    return run_sweep_v<T, NB, false>(ctx, plan, R, Y, ybits, X, n_f, ld, lambda, X_at, grad_out,
                                     bad_row, status, empty_status, n_rows_unplanned, partial_ext,
                                     s);
}

template <typename T>
int dispatch_sweep(Ctx *ctx, const Plan *plan, const als_csr *R, const void *Y,
                   const unsigned *ybits, void *X, int n_f, int ld, double lambda,
                   const void *X_at, void *grad_out, int64_t *bad_row, int32_t *status,
                   int empty_status, int64_t n_rows_unplanned, void *partial_ext, hipStream_t s) {
    const int nb = (n_f + 1 + 15) / 16;
#define ALS_SWEEP_CASE(NBV)                                                                      \
    case NBV:                                                                                    \
        return run_sweep<T, NBV>(ctx, plan, R, (const T *)Y, ybits, (T *)X, n_f, ld, (T)lambda,  \
                                 (const T *)X_at, (T *)grad_out, bad_row, status, empty_status,  \
                                 n_rows_unplanned, partial_ext, s);
    if constexpr (sizeof(T) == 4) {
        switch (nb) {
            ALS_SWEEP_CASE(1)
            ALS_SWEEP_CASE(2)
            ALS_SWEEP_CASE(3)
            ALS_SWEEP_CASE(4)
            ALS_SWEEP_CASE(5)
            ALS_SWEEP_CASE(6)
            ALS_SWEEP_CASE(7)
            ALS_SWEEP_CASE(8)
            ALS_SWEEP_CASE(9)
            default: return ALS_E_INVAL;
        }
    } else {
        switch (nb) {
            ALS_SWEEP_CASE(1)
            ALS_SWEEP_CASE(2)
            ALS_SWEEP_CASE(3)
            ALS_SWEEP_CASE(4)
            ALS_SWEEP_CASE(5)
            ALS_SWEEP_CASE(6)
            default: return ALS_E_INVAL;
        }
    }
#undef ALS_SWEEP_CASE
}

}  // namespace

int launch_abs_max_bits(const float *Y, int64_t n, int n_f, int ld, unsigned *out, hipStream_t s) {
    if (!Y || n <= 0 || n_f <= 0) {
        hipLaunchKernelGGL(set_u32_kernel, dim3(1), dim3(1), 0, s, out, 0u);
    } else {
        const int64_t per_block = 4 * kAbsMaxRows;
        const unsigned blocks =
            (unsigned)std::min<int64_t>((n + per_block - 1) / per_block, kAbsMaxParts);
        hipLaunchKernelGGL(abs_max_bits_kernel, dim3(blocks), dim3(256), 0, s, Y, n, n_f, ld,
                           out + 1);
        hipLaunchKernelGGL(abs_max_final_kernel, dim3(1), dim3(256), 0, s, out + 1, (int)blocks,
                           out);
    }
    return hipGetLastError() == hipSuccess ? ALS_OK : ALS_E_HIP;
}

int launch_sweep(Ctx *ctx, const Plan *plan, const als_csr *R, const void *Y, void *X, int n_f,
                 int ld, double lambda, als_dtype dt, const void *X_at, void *grad_out,
                 int64_t *bad_row, hipStream_t s) {
    if (dt == ALS_F32)
        return dispatch_sweep<float>(ctx, plan, R, Y, nullptr, X, n_f, ld, lambda, X_at, grad_out,
                                     bad_row, nullptr, 0, 0, nullptr, s);
    if (dt == ALS_F64)
        return dispatch_sweep<double>(ctx, plan, R, Y, nullptr, X, n_f, ld, lambda, X_at,
                                      grad_out, bad_row, nullptr, 0, 0, nullptr, s);
    return ALS_E_INVAL;
}

int launch_fold_in(Ctx *ctx, const void *M, int64_t n_items, int n_f, int ld, double lambda,
                   als_dtype dt, int64_t n_req, const int64_t *indptr, const int32_t *items,
                   const float *vals, void *U_out, int32_t *status, hipStream_t s) {
    als_csr R;
    R.n_rows = n_req;
    R.n_cols = n_items;
    R.nnz = 0;
    R.indptr = indptr;
    R.indices = items;
    R.values = vals;
    if (dt == ALS_F32)
        return dispatch_sweep<float>(ctx, nullptr, &R, M, nullptr, U_out, n_f, ld, lambda, nullptr,
                                     nullptr, nullptr, status, ALS_E_INVAL, n_req, nullptr, s);
    if (dt == ALS_F64)
        return dispatch_sweep<double>(ctx, nullptr, &R, M, nullptr, U_out, n_f, ld, lambda,
                                      nullptr, nullptr, nullptr, status, ALS_E_INVAL, n_req,
                                      nullptr, s);
    return ALS_E_INVAL;
}

size_t sweep_partial_bytes(int n_f, als_dtype dt) {
    const size_t nb = (size_t)(n_f + 1 + 15) / 16;
    const size_t nt = nb * (nb + 1) / 2;
    return nt * kWave * 4 * (dt == ALS_F64 ? sizeof(double) : sizeof(float));
}

int launch_sweep_batch(const Plan *plan, const als_csr *R, const void *Y, const unsigned *ybits,
                       void *X, int n_f, int ld, double lambda, als_dtype dt, void *partial,
                       int32_t *status, hipStream_t s) {
    if (dt == ALS_F32) {
        if (!ybits) return ALS_E_INVAL;
        return dispatch_sweep<float>(nullptr, plan, R, Y, ybits, X, n_f, ld, lambda, nullptr,
                                     nullptr, nullptr, status, ALS_E_INVAL, 0, partial, s);
    }
    if (dt == ALS_F64)
        return dispatch_sweep<double>(nullptr, plan, R, Y, nullptr, X, n_f, ld, lambda, nullptr,
                                      nullptr, nullptr, status, ALS_E_INVAL, 0, partial, s);
    return ALS_E_INVAL;
}

}  // namespace alsncg
