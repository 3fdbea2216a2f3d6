// Top-t rankings and the ranking accuracy of Section IV (a modified Kendall
// tau distance restricted to the top t items of each user).
//
// A user's ranking orders all items by the predicted rating u_i . m_j,
// largest first, equal ratings by increasing item id.  Predicted ratings are
// formed in FP64 on the FP64 MFMA (v_mfma_f64_16x16x4): a wavefront owns 16
// users (the tile's rows) and sweeps the items in tiles of 64 (four 16-column
// MFMA blocks), reading the item factors straight from L2 (every wavefront of
// a workgroup streams the same rows, so the workgroup's four wavefronts share
// them through L1).  The contraction index is a free label, so lane group g
// supplies the contiguous factor range [g*NS, g*NS + NS) over the NS MFMA
// steps (vector loads of 4 floats when rows allow it).  The 16x64 block of
// ratings goes through LDS to a layout with four lanes per user.
//
// rank_top_kernel: every lane keeps a sorted list (best first) of the best
// items among those it has seen (items 16q .. 16q + 15 of each tile for
// lane q of its user).  An item is inserted only if it is ahead of the t-th
// entry of every one of the user's four lists (taken at the start of the
// tile): a list holds t items ahead of anything behind its t-th entry.
// At the end the four lists are merged through LDS.
//
// rank_accuracy_kernel: for the reference items a_1..a_t of a user, the
// swap count of Section IV is s = sum_k (r_k - #{j < k : r_j < r_k}) where
// r_k is the number of items ranked ahead of a_k by the current factors
// (moving a_1..a_{k-1} to the front leaves the others in order, so a_k
// passes exactly the items ahead of it that were not moved yet).  r_k is
// counted against the rating of a_k taken from the diagonal of an MFMA block
// whose column c holds a_k of user c, i.e. the same dot-product arithmetic
// as the tiles, so equal ratings compare equal on both sides; a_k itself is
// excluded by id.  The swap counts are summed exactly in int64.
#include <math.h>

#include "internal.h"

namespace alsncg {
namespace {

constexpr int kRankUsers = 16;                 // users per wavefront (MFMA rows)
constexpr int kRankWaves = 4;                  // wavefronts per workgroup
constexpr int kRankItems = 64;                 // items per tile (4 MFMA column blocks)
constexpr int kRankPitch = kRankItems + 2;     // LDS row pitch (16-byte rows, no bank conflicts)
constexpr int kRankMaxT = 32;                  // largest t (list capacity)
constexpr int kRankTQ = kRankMaxT / 4;         // reference items per lane (accuracy)

typedef Mfma<double>::acc4 dacc4;

// Order of a ranking: (s, x) comes before (s2, x2).
__device__ inline bool ahead(double s, int x, double s2, int x2) {
    return s > s2 || (s == s2 && x < x2);
}

// Orders a wavefront's own LDS accesses (LDS instructions of a wavefront
// complete in order; the fences keep the compiler from moving accesses).
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A operand: lane (g, c) holds U[user0 + c][g*NS + s] for s < NS, zero past
// n_f and for users past n_u, in type AT (T: widened to FP64 at each MFMA).
template <typename T, typename AT, int NS>
__device__ inline void load_users(AT (&a)[NS], const T *U, int64_t n_u, int n_f, int ld,
                                  int64_t user0) {
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
    const int64_t u = user0 + c;
    const T *row = U + (u < n_u ? u : n_u - 1) * (int64_t)ld;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int k = g * NS + s;
        const T v = row[k < n_f ? k : n_f - 1];
        a[s] = (u < n_u && k < n_f) ? (AT)v : AT(0);
    }
}

// B operand of one 16x16 MFMA block: lane (g, c) loads M[item][g*NS + s],
// s < NS, for the item of its column c (0 <= item < n_m).  Factors past n_f
// are read clamped and cancelled by the zeros of the A operand.  VEC = 4:
// 16-byte loads (float rows with n_f and ld multiples of 4, aligned base).
template <typename T, int NS, int VEC>
__device__ inline void load_items(T (&b)[NS], const T *M, int item, int n_f, int ld) {
    const int g = (threadIdx.x & 63) >> 4;
    const T *row = M + (int64_t)item * ld;
    if constexpr (VEC == 4) {
        static_assert(NS % 4 == 0, "vector loads need NS % 4 == 0");
#pragma unroll
        for (int v = 0; v < NS / 4; ++v) {
            const int k = g * NS + 4 * v;
            const float4 x = *reinterpret_cast<const float4 *>(row + (k < n_f ? k : n_f - 4));
            b[4 * v] = x.x;
            b[4 * v + 1] = x.y;
            b[4 * v + 2] = x.z;
            b[4 * v + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int k = g * NS + s;
            b[s] = row[k < n_f ? k : n_f - 1];
        }
    }
}

// D[u][c] = U[user0 + u] . M[item of column c], accumulated over the NS
// steps in FP64.
template <typename T, typename AT, int NS>
__device__ inline dacc4 rating_mma(const AT (&a)[NS], const T (&b)[NS]) {
    dacc4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < NS; ++s) d = Mfma<double>::mma((double)a[s], (double)b[s], d);
    return d;
}

template <typename T, typename AT, int NS, int VEC>
__device__ inline dacc4 rating_block(const AT (&a)[NS], const T *M, int item, int n_f, int ld) {
    T b[NS];
    load_items<T, NS, VEC>(b, M, item, n_f, ld);
    return rating_mma<T, AT, NS>(a, b);
}

__device__ inline int tile_item(int tile, int b, int n_m) {
    return min(tile + 16 * b + (threadIdx.x & 15), n_m - 1);
}

__device__ inline void store_block(double *S, int b, const dacc4 &d) {
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
#pragma unroll
    for (int r = 0; r < 4; ++r) S[Mfma<double>::row(g, r) * kRankPitch + 16 * b + c] = d[r];
}

// Ratings of the wavefront's 16 users against items tile .. tile + 63 into
// the LDS tile S[u * kRankPitch + x] (items past n_m repeat the last item;
// readers skip them).  Each block's loads are in flight while the previous
// block's MFMAs run.  NEXT: b0 holds the B operand of the tile's first block
// on entry and that of the next tile's first block on exit (loads in flight
// across the caller's scan of the tile); else b0 is loaded here.
template <typename T, typename AT, int NS, int VEC, bool NEXT>
__device__ inline void rating_tile(const AT (&a)[NS], T (&b0)[NS], const T *M, int n_m, int n_f,
                                   int ld, int tile, double *S) {
    if constexpr (!NEXT) load_items<T, NS, VEC>(b0, M, tile_item(tile, 0, n_m), n_f, ld);
    T b1[NS];
    load_items<T, NS, VEC>(b1, M, tile_item(tile, 1, n_m), n_f, ld);
    store_block(S, 0, rating_mma<T, AT, NS>(a, b0));
    load_items<T, NS, VEC>(b0, M, tile_item(tile, 2, n_m), n_f, ld);
    store_block(S, 1, rating_mma<T, AT, NS>(a, b1));
    load_items<T, NS, VEC>(b1, M, tile_item(tile, 3, n_m), n_f, ld);
    store_block(S, 2, rating_mma<T, AT, NS>(a, b0));
    if constexpr (NEXT) load_items<T, NS, VEC>(b0, M, tile_item(tile + kRankItems, 0, n_m), n_f, ld);
    store_block(S, 3, rating_mma<T, AT, NS>(a, b1));
}

// Insert (s, x) into the sorted list (ls, li) of capacity TT, dropping the
// last entry; requires ahead(s, x, ls[TT-1], li[TT-1]).
template <int TT>
__device__ inline void list_insert(double (&ls)[TT], int (&li)[TT], double s, int x) {
    bool here = true;  // (s, x) is ahead of entry q (true for q = TT - 1)
#pragma unroll
    for (int q = TT - 1; q > 0; --q) {
        const bool prev = ahead(s, x, ls[q - 1], li[q - 1]);
        if (here) {
            ls[q] = prev ? ls[q - 1] : s;
            li[q] = prev ? li[q - 1] : x;
        }
        here = prev;
    }
    if (here) {
        ls[0] = s;
        li[0] = x;
    }
}

// LDS per wavefront of the top-t kernel: the 16x64 rating tile, reused at
// the end for the lists handed over in the merge (32 lists of t entries).
constexpr int kTopLdsBytes = 32 * kRankMaxT * (8 + 4);
static_assert(kTopLdsBytes >= kRankUsers * kRankPitch * 8, "merge buffer covers the tile");

// Wavefronts per SIMD the top-t kernel is compiled for: two where the
// register budget of two (256 per lane) holds the lists and the operands
// without spills, else one.
template <typename T, int NS, int VEC, int TT>
constexpr int kTopOccupancy =
    (NS < 28 || (sizeof(T) == 4 && VEC == 4 && (NS == 28 || TT <= 20))) ? 2 : 1;

// TT: list capacity (>= t; 20, the paper's t, or kRankMaxT).
template <typename T, int NS, int VEC, int TT>
__global__ __launch_bounds__(kRankWaves * 64, (kTopOccupancy<T, NS, VEC, TT>)) void rank_top_kernel(
    const T *U, const T *M, int64_t n_u, int n_m, int n_f, int ld, int t, int32_t *top) {
    static_assert(TT <= kRankMaxT, "merge buffer holds kRankMaxT entries per list");
    __shared__ __align__(16) double lds_all[kRankWaves][kTopLdsBytes / 8];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t user0 = ((int64_t)blockIdx.x * kRankWaves + w) * kRankUsers;
    if (user0 >= n_u) return;  // whole wavefront; no workgroup barrier below
    double *S = lds_all[w];
    T a[NS];
    load_users<T, T, NS>(a, U, n_u, n_f, ld, user0);

    const int u = lane >> 2, q = lane & 3;
    double ls[TT];
    int li[TT];
#pragma unroll
    for (int e = 0; e < TT; ++e) {
        ls[e] = -INFINITY;
        li[e] = INT32_MAX;
    }
    for (int tile = 0; tile < n_m; tile += kRankItems) {
        // the user's bar: the best t-th entry of its four lists
        double bs = ls[0];
        int bi = li[0];
#pragma unroll
        for (int e = 1; e < TT; ++e)
            if (e == t - 1) {
                bs = ls[e];
                bi = li[e];
            }
#pragma unroll
        for (int m = 1; m <= 2; m <<= 1) {
            const double os = __shfl_xor(bs, m);
            const int oi = __shfl_xor(bi, m);
            if (ahead(os, oi, bs, bi)) {
                bs = os;
                bi = oi;
            }
        }
        T b0[NS];
        rating_tile<T, T, NS, VEC, false>(a, b0, M, n_m, n_f, ld, tile, S);
        wave_lds_sync();
        // lane q takes items 16q .. 16q + 15 of the tile: candidates first
        // (16-byte reads), then the few insertions
        const int n_x = min(kRankItems, n_m - tile);
        const double *row = S + u * kRankPitch + 16 * q;
        unsigned cand = 0;
        {
            double v[16];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const double2 p = reinterpret_cast<const double2 *>(row)[i];
                v[2 * i] = p.x;
                v[2 * i + 1] = p.y;
            }
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (16 * q + i < n_x && ahead(v[i], tile + 16 * q + i, bs, bi)) cand |= 1u << i;
        }
        while (cand) {
            const int i = __builtin_ctz(cand);
            cand &= cand - 1;
            const double s = row[i];
            const int x = tile + 16 * q + i;
            if (ahead(s, x, ls[TT - 1], li[TT - 1])) list_insert<TT>(ls, li, s, x);
        }
        wave_lds_sync();
    }
    // merge the user's four lists through LDS: lane q receives the first t
    // entries of lane q + 1 (q even), then lane 0 those of lane 2
    double *Ms = S;
    int *Mi = reinterpret_cast<int *>(S + 32 * TT);
#pragma unroll 1
    for (int m = 1; m <= 2; m <<= 1) {
        const bool sender = (q & (2 * m - 1)) == m, receiver = (q & (2 * m - 1)) == 0;
        const int slot = lane / (2 * m);
        if (sender) {
#pragma unroll
            for (int e = 0; e < TT; ++e)
                if (e < t) {
                    Ms[slot * TT + e] = ls[e];
                    Mi[slot * TT + e] = li[e];
                }
        }
        wave_lds_sync();
        if (receiver) {
#pragma unroll 1
            for (int e = 0; e < t; ++e) {
                const double s = Ms[slot * TT + e];
                const int x = Mi[slot * TT + e];
                if (ahead(s, x, ls[TT - 1], li[TT - 1])) list_insert<TT>(ls, li, s, x);
            }
        }
        wave_lds_sync();
    }
    const int64_t user = user0 + u;
    if (q == 0 && user < n_u) {
#pragma unroll
        for (int e = 0; e < TT; ++e)
            if (e < t) top[user * t + e] = li[e] == INT32_MAX ? -1 : li[e];
    }
}

// Wavefronts per SIMD of the accuracy kernel (one where n_f > 64 and the
// factors are FP64 or take element loads: no room for two without spills).
template <typename T, int NS, int VEC>
constexpr int kAccOccupancy = (NS >= 28 && (sizeof(T) == 8 || VEC == 1)) ? 1 : 2;

template <typename T, int NS, int VEC>
__global__ __launch_bounds__(kRankWaves * 64, (kAccOccupancy<T, NS, VEC>)) void rank_accuracy_kernel(
    const T *U, const T *M, int64_t n_u, int n_m, int n_f, int ld, int t, const int32_t *top,
    int64_t *swaps, unsigned long long *total) {
    constexpr int TQ = kRankTQ;
    __shared__ __align__(16) double S_all[kRankWaves][kRankUsers * kRankPitch];
    __shared__ double Th_all[kRankWaves][kRankUsers * kRankMaxT];
    __shared__ int Rk_all[kRankWaves][kRankUsers * kRankMaxT];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
    const int64_t user0 = ((int64_t)blockIdx.x * kRankWaves + w) * kRankUsers;
    if (user0 >= n_u) return;  // whole wavefront; no workgroup barrier below
    double *S = S_all[w], *Th = Th_all[w];
    int *Rk = Rk_all[w];
    double a[NS];
    load_users<T, double, NS>(a, U, n_u, n_f, ld, user0);

    // ratings of the reference items: column c of block k holds a_k of user c
    {
        const int64_t uc = min(user0 + c, n_u - 1);
        for (int k = 0; k < t; ++k) {
            const int item = min(max(top[uc * t + k], 0), n_m - 1);
            const dacc4 d = rating_block<T, double, NS, VEC>(a, M, item, n_f, ld);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (Mfma<double>::row(g, r) == c) Th[c * kRankMaxT + k] = d[r];
        }
    }
    wave_lds_sync();

    const int u = lane >> 2, q = lane & 3;
    const int64_t user = user0 + u;
    const int64_t uu = user < n_u ? user : n_u - 1;
    double th[TQ];
    int ak[TQ], cnt[TQ];
    double th_min = INFINITY;
#pragma unroll
    for (int j = 0; j < TQ; ++j) {
        const int k = q + 4 * j;
        th[j] = k < t ? Th[u * kRankMaxT + k] : INFINITY;  // never passed
        ak[j] = k < t ? top[uu * t + k] : -1;
        cnt[j] = 0;
        th_min = fmin(th_min, th[j]);
    }
    // lowest reference rating of the user (over its four lanes)
    th_min = fmin(th_min, __shfl_xor(th_min, 1));
    th_min = fmin(th_min, __shfl_xor(th_min, 2));
    T b0[NS];
    load_items<T, NS, VEC>(b0, M, tile_item(0, 0, n_m), n_f, ld);
    for (int tile = 0; tile < n_m; tile += kRankItems) {
        rating_tile<T, double, NS, VEC, true>(a, b0, M, n_m, n_f, ld, tile, S);
        wave_lds_sync();
        // items at or above the user's lowest reference rating: lane q scans
        // items 16q .. 16q + 15 (16-byte reads), the four masks are combined,
        // and every lane counts those few against its own reference items
        const int n_x = min(kRankItems, n_m - tile);
        const double *row = S + u * kRankPitch;
        unsigned long long cand;
        {
            double v[16];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const double2 p = reinterpret_cast<const double2 *>(row + 16 * q)[i];
                v[2 * i] = p.x;
                v[2 * i + 1] = p.y;
            }
            unsigned m = 0;
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (16 * q + i < n_x && v[i] >= th_min) m |= 1u << i;
            cand = (unsigned long long)m << (16 * q);
            cand |= __shfl_xor(cand, 1);
            cand |= __shfl_xor(cand, 2);
        }
        while (cand) {
            const int xl = __builtin_ctzll(cand);
            cand &= cand - 1;
            const double s = row[xl];
            const int x = tile + xl;
#pragma unroll
            for (int j = 0; j < TQ; ++j) cnt[j] += (x != ak[j] && ahead(s, x, th[j], ak[j])) ? 1 : 0;
        }
        wave_lds_sync();
    }
    // s = sum_k (r_k - #{j < k : r_j < r_k})
#pragma unroll
    for (int j = 0; j < TQ; ++j)
        if (q + 4 * j < t) Rk[u * kRankMaxT + q + 4 * j] = cnt[j];
    wave_lds_sync();
    long long part = 0;
#pragma unroll
    for (int j = 0; j < TQ; ++j) {
        const int k = q + 4 * j;
        if (k < t) {
            int below = 0;
            for (int i = 0; i < k; ++i) below += Rk[u * kRankMaxT + i] < cnt[j] ? 1 : 0;
            part += cnt[j] - below;
        }
    }
    part += __shfl_xor(part, 1);
    part += __shfl_xor(part, 2);
    const bool own = q == 0 && user < n_u;
    if (own && swaps) swaps[user] = part;
    long long wsum = own ? part : 0;
#pragma unroll
    for (int m = 4; m < 64; m <<= 1) wsum += __shfl_xor(wsum, m);
    if (lane == 0) atomicAdd(total, (unsigned long long)wsum);
}

__global__ void rank_total_zero(unsigned long long *total) {
    if (threadIdx.x == 0) total[0] = 0ull;
}

// mean q = 1 - total / (n_u s_max)
__global__ void rank_mean_q(const unsigned long long *total, int64_t n_u, double s_max,
                            double *mean_q) {
    if (threadIdx.x == 0) mean_q[0] = 1.0 - (double)total[0] / ((double)n_u * s_max);
}

// NS buckets: 4 * ceil(n_f / 16) rounded to {4, 8, 16, 28, 32}
template <template <typename, int, int> class Launch, typename T, int VEC, typename... A>
int dispatch_ns(int n_f, A... args) {
    if (n_f <= 16) return Launch<T, 4, VEC>::run(args...);
    if (n_f <= 32) return Launch<T, 8, VEC>::run(args...);
    if (n_f <= 64) return Launch<T, 16, VEC>::run(args...);
    if (n_f <= 112) return Launch<T, 28, VEC>::run(args...);
    return Launch<T, 32, VEC>::run(args...);
}

inline int64_t rank_blocks(int64_t n_u) {
    const int64_t per = (int64_t)kRankWaves * kRankUsers;
    return (n_u + per - 1) / per;
}

template <int TT> struct TopLaunch {
    template <typename T, int NS, int VEC> struct L {
        static int run(const void *U, const void *M, int64_t n_u, int n_m, int n_f, int ld, int t,
                       int32_t *top, hipStream_t s) {
            hipLaunchKernelGGL((rank_top_kernel<T, NS, VEC, TT>), dim3((unsigned)rank_blocks(n_u)),
                               dim3(kRankWaves * 64), 0, s, (const T *)U, (const T *)M, n_u, n_m,
                               n_f, ld, t, top);
            return hipGetLastError() == hipSuccess ? ALS_OK : ALS_E_HIP;
        }
    };
};

template <typename T, int NS, int VEC> struct AccLaunch {
    static int run(const void *U, const void *M, int64_t n_u, int n_m, int n_f, int ld, int t,
                   const int32_t *top, int64_t *swaps, unsigned long long *total, hipStream_t s) {
        hipLaunchKernelGGL((rank_accuracy_kernel<T, NS, VEC>), dim3((unsigned)rank_blocks(n_u)),
                           dim3(kRankWaves * 64), 0, s, (const T *)U, (const T *)M, n_u, n_m, n_f,
                           ld, t, top, swaps, total);
        return hipGetLastError() == hipSuccess ? ALS_OK : ALS_E_HIP;
    }
};

// 16-byte loads of M rows: float rows, n_f and ld multiples of 4, aligned base.
bool rank_vec4(const void *M, int n_f, int ld, als_dtype dt) {
    return dt == ALS_F32 && n_f % 4 == 0 && ld % 4 == 0 && ((uintptr_t)M & 15) == 0;
}

template <int TT>
int launch_rank_top_tt(const void *U, const void *M, int64_t n_u, int n_m, int n_f, int ld,
                       als_dtype dt, int t, int32_t *top, hipStream_t s) {
    if (dt == ALS_F64)
        return dispatch_ns<TopLaunch<TT>::template L, double, 1>(n_f, U, M, n_u, n_m, n_f, ld, t, top, s);
    if (rank_vec4(M, n_f, ld, dt))
        return dispatch_ns<TopLaunch<TT>::template L, float, 4>(n_f, U, M, n_u, n_m, n_f, ld, t, top, s);
    return dispatch_ns<TopLaunch<TT>::template L, float, 1>(n_f, U, M, n_u, n_m, n_f, ld, t, top, s);
}

}  // namespace

int launch_rank_top(const void *U, const void *M, int64_t n_u, int n_m, int n_f, int ld,
                    als_dtype dt, int t, int32_t *top, hipStream_t s) {
    if (n_u == 0) return ALS_OK;
    if (t <= 20) return launch_rank_top_tt<20>(U, M, n_u, n_m, n_f, ld, dt, t, top, s);
    return launch_rank_top_tt<kRankMaxT>(U, M, n_u, n_m, n_f, ld, dt, t, top, s);
}

int launch_rank_accuracy(Ctx *ctx, const void *U, const void *M, int64_t n_u, int n_m, int n_f,
                         int ld, als_dtype dt, int t, const int32_t *top, int64_t *swaps,
                         double *mean_q, hipStream_t s) {
    int err = ALS_OK;
    auto *total = (unsigned long long *)ctx->workspace(sizeof(unsigned long long), s, &err);
    if (!total) return err;
    hipLaunchKernelGGL(rank_total_zero, dim3(1), dim3(64), 0, s, total);
    ALS_HIP_CHECK(hipGetLastError());
    if (dt == ALS_F64)
        err = dispatch_ns<AccLaunch, double, 1>(n_f, U, M, n_u, n_m, n_f, ld, t, top, swaps, total, s);
    else if (rank_vec4(M, n_f, ld, dt))
        err = dispatch_ns<AccLaunch, float, 4>(n_f, U, M, n_u, n_m, n_f, ld, t, top, swaps, total, s);
    else
        err = dispatch_ns<AccLaunch, float, 1>(n_f, U, M, n_u, n_m, n_f, ld, t, top, swaps, total, s);
    if (err != ALS_OK) return err;
    if (mean_q) {
        const double smax = 0.5 * (double)t * (2.0 * (double)n_m - (double)t - 1.0);
        hipLaunchKernelGGL(rank_mean_q, dim3(1), dim3(64), 0, s, total, n_u, smax, mean_q);
        ALS_HIP_CHECK(hipGetLastError());
    }
    return ALS_OK;
}

}  // namespace alsncg
