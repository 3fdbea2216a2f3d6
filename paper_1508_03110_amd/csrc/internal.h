// Internal declarations shared by the HIP translation units of libalsncg.
// gfx950 (CDNA4) only: 64-lane wavefronts, 16x16 MFMA tiles.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>
#include <vector>

#include "../../include/alsncg.h"

namespace alsncg {

constexpr int kWave = 64;

// ---------------------------------------------------------------- MFMA tiles
//
// v_mfma_{f32,f64}_16x16x4: D[16x16] += A[16x4] B[4x16].  Lane l = 16 g + c
// (g = l / 16, c = l % 16) supplies A[c][g] and B[g][c]; accumulator
// register r of lane l holds D[row(g, r)][c], where
//     f32: row(g, r) = 4 g + r      (each lane group owns 4 consecutive rows)
//     f64: row(g, r) = g + 4 r      (rows interleaved across lane groups).
// The contraction index of a Gram update is a free label, so a lane may feed
// the same register as A and B.  pivot_g / pivot_r invert row().
template <typename T> struct Mfma;

template <> struct Mfma<float> {
    static constexpr als_dtype kDtype = ALS_F32;
    typedef float acc4 __attribute__((ext_vector_type(4)));
    __device__ static inline acc4 mma(float a, float b, acc4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __host__ __device__ static constexpr int row(int g, int r) { return 4 * g + r; }
    __host__ __device__ static constexpr int pivot_g(int k) { return k >> 2; }
    __host__ __device__ static constexpr int pivot_r(int k) { return k & 3; }
};

template <> struct Mfma<double> {
    static constexpr als_dtype kDtype = ALS_F64;
    typedef double acc4 __attribute__((ext_vector_type(4)));
    __device__ static inline acc4 mma(double a, double b, acc4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __host__ __device__ static constexpr int row(int g, int r) { return g + 4 * r; }
    __host__ __device__ static constexpr int pivot_g(int k) { return k & 3; }
    __host__ __device__ static constexpr int pivot_r(int k) { return k >> 2; }
};

__device__ inline float readlane(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ inline double readlane(double v, int lane) {
    long long x = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), lane);
    int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 1/sqrt(d) for d > 0 on the Cholesky pivots, avoiding the long IEEE sqrt
// and divide sequences.  FP32: the hardware reciprocal square root
// (v_rsq_f32, about 1 ulp).  FP64: the FP32 estimate refined by three Newton
// steps y <- y (3 - d y^2) / 2, accurate to a few units in the last place.
// d <= 0 gives a NaN or an infinity (the caller reports the pivot).
__device__ inline float inv_sqrt(float d) { return __builtin_amdgcn_rsqf(d); }
__device__ inline double inv_sqrt(double d) {
    double y = (double)__builtin_amdgcn_rsqf((float)d);
    y = y * (1.5 - 0.5 * d * y * y);
    y = y * (1.5 - 0.5 * d * y * y);
    return y * (1.5 - 0.5 * d * y * y);
}

// Sum over the 16 lanes that share l / 16 (result in all 16 lanes), as the
// butterfly v += v[l ^ 1], v[l ^ 2], v[l ^ 4], v[l ^ 8].
template <typename T> __device__ inline T sum16(T v) {
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    return v;
}
// FP32: the same additions through DPP lane moves instead of LDS permutes.
// quad_perm [1,0,3,2] and [2,3,0,1] are l ^ 1 and l ^ 2; after them every lane
// of a quad holds the quad's sum, so row_half_mirror (l -> 7 - l within 8)
// adds the same value as l ^ 4, and row_mirror (l -> 15 - l within 16) the
// same value as l ^ 8.  Same pairs, same order: bit-identical results.
template <int CTRL> __device__ inline float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <> __device__ inline float sum16<float>(float v) {
    v += dpp_f32<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f32<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_f32<0x141>(v);  // row_half_mirror
    v += dpp_f32<0x140>(v);  // row_mirror
    return v;
}
// Sum over the 4 lanes that share l % 16 (result in all 4 lanes), as the
// butterfly v += v[l ^ 16], v[l ^ 32].
template <typename T> __device__ inline T sum4g(T v) {
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}
// FP32: the same additions through the lane-swap instructions.  With both
// operands v, permlane16_swap returns the even rows of 16 lanes duplicated
// and the odd rows duplicated, whose sum is v[l] + v[l ^ 16] in every lane;
// permlane32_swap does the same for the two halves of the wave (l ^ 32).
template <> __device__ inline float sum4g<float>(float v) {
    auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(a[0]) + __uint_as_float(a[1]);
    auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}
template <typename T> __device__ inline T sum64(T v) { return sum4g(sum16(v)); }
// Maximum over the wavefront (result in every lane).
__device__ inline float wave_max(float m) {
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) m = fmaxf(m, __shfl_xor(m, o));
    return m;
}

// ---------------------------------------------------------------- FP16-split products
//
// FP32 products on FP16 MFMAs: a value x (already scaled by a power of two
// into the FP16 range) is split into h = fp16(x) and m = fp16(x - h), both
// rounded to nearest (x - h is exact in FP32, so x = h + m + d with
// |d| <= 2^-22 |x|), and x_a x_b is taken as h_a h_b + h_a m_b + m_a h_b,
// three exact FP16 products accumulated in FP32 by
// v_mfma_f32_16x16x32_f16 (lane l = 16 g + c supplies A[c][8g..8g+7] and
// B[8g..8g+7][c]; the accumulator layout is that of Mfma<float>).
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef float float2_t __attribute__((ext_vector_type(2)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ Mfma<float>::acc4 mma_f16(u32x4_t a, u32x4_t b, Mfma<float>::acc4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(half8_t, a),
                                                  __builtin_bit_cast(half8_t, b), c, 0, 0, 0);
}

// Two scaled values -> packed FP16 high parts and packed FP16 low parts.
__device__ __forceinline__ void split2(float x0, float x1, unsigned &hi, unsigned &lo) {
    const float2_t x = {x0, x1};
    const half2_t h = __builtin_convertvector(x, half2_t);
    const half2_t m = __builtin_convertvector(x - __builtin_convertvector(h, float2_t), half2_t);
    hi = __builtin_bit_cast(unsigned, h);
    lo = __builtin_bit_cast(unsigned, m);
}

// 2^e as an FP32 number, -126 <= e <= 127.
__device__ __forceinline__ float exp2i(int e) { return __int_as_float((127 + e) << 23); }

// s with 2^s M < 2^14 for M = max(a, b) given as the bits of two
// non-negative floats; clamped to [-60, 60] so that 2^s and 2^-2s are normal
// FP32 numbers (a Gram of entries above 2^74 overflows FP32 anyway).
// Non-finite or zero M: s = 0.
__device__ __forceinline__ int split_shift(unsigned ybits, unsigned rbits) {
    const unsigned mb = max(ybits, rbits);
    if (mb == 0u || mb >= 0x7f800000u) return 0;
    const int e = (int)(mb >> 23) - 126;  // M < 2^e
    return min(max(14 - e, -60), 60);
}


// ---------------------------------------------------------------- host objects

struct Plan {
    int64_t n_rows = 0, nnz = 0, n_chunks = 0, n_split_rows = 0, n_slots = 0, chunk = 0,
            max_row = 0;
    // persistent grids (workgroups striding over the chunks) of the
    // half-sweep and of the streaming passes; 0: one workgroup per chunk
    int64_t grid = 0, grid_pass = 0;
    // device arrays, chunk order = longest first
    int32_t *chunk_row = nullptr;
    int64_t *chunk_begin = nullptr;
    int32_t *chunk_len = nullptr;
    int32_t *chunk_slot = nullptr;  // -1: the chunk is the whole row
    // split rows (more than one chunk): slots slot0 .. slot0 + nslot - 1
    int32_t *split_row = nullptr;
    int32_t *split_slot0 = nullptr;
    int32_t *split_nslot = nullptr;
    // split chunks: slot -> index of its chunk in chunk order (may be null
    // for plans that are only used by the FP32/FP64 half-sweep)
    int32_t *slot_chunk = nullptr;
    // dual-form bins of the half-sweep (als_plan_set_dual): whole rows of
    // 1 <= n_i <= dual_max ratings are the last n_dual chunks, longest first;
    // bin b (1 <= b <= kDualMaxBlocks) holds the rows with n_i >= 2 and
    // ceil((n_i + 2) / 16) = b, bin 0 the rows with one rating (closed
    // form), chunks dual_first[b] .. + dual_count[b] - 1
    int64_t dual_max = 0, n_dual = 0;
    int64_t dual_first[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t dual_count[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    // host copies of the chunk arrays (in chunk order), kept to re-bin
    std::vector<int32_t> h_row, h_len, h_slot;
    std::vector<int64_t> h_beg;
    // > 0: rows cut at column-slice boundaries (als_plan_create_sliced); such
    // a plan serves the gradient pass only
    int64_t col_slices = 0;
    // FP32 half-sweep over a split copy of the fixed side: 1 on, 0 off, -1
    // (default) on when the copy's rows are no wider than the factor rows
    int split_copy = -1;
};

// Accelerator dies (XCDs) of the device, each with its own L2: the
// workgroups of a one-dimensional launch are handed to them in turn, so
// workgroup b runs on die b mod kXcds.
constexpr int64_t kXcds = 8;

// Largest dual system: kDualMaxBlocks tiles of 16 (rows of at most
// 16 kDualMaxBlocks - 2 ratings: one slot for the right-hand side, one for
// the gradient point).
constexpr int kDualMaxBlocks = 6;
constexpr int64_t kDualMaxLen = 16 * kDualMaxBlocks - 2;

struct Ctx {
    int device = 0;
    int num_cu = 256;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    // device address of the library's fixed scratch array on this context's
    // device (looked up once at creation) and its size in doubles
    double *scratch = nullptr;
    size_t scratch_doubles = 0;
    // device words for the FP32 half-sweep's scale (ybits[0]: bits of max
    // |Y|; kAbsMaxWords in all), rewritten before every FP32 half-sweep on
    // this context
    unsigned *ybits = nullptr;
    // FP16 split copy of the fixed side of the FP32 half-sweep (rewritten by
    // every planned FP32 half-sweep on this context) and its size
    void *ysplit = nullptr;
    size_t ysplit_bytes = 0;
    // Returns workspace of at least `bytes` (grows; synchronises before freeing).
    void *workspace(size_t bytes, hipStream_t stream, int *err);
    // The split copy's buffer, grown the same way.
    void *split_buffer(size_t bytes, hipStream_t stream, int *err);
};

}  // namespace alsncg

struct als_ctx : alsncg::Ctx {};
struct als_plan : alsncg::Plan {};

namespace alsncg {

// Kernel launchers (sweep.hip, passes.hip, vec.hip).  Return an als_status.
int launch_sweep(Ctx *ctx, const Plan *plan, const als_csr *R, const void *Y, void *X, int n_f,
                 int ld, double lambda, als_dtype dt, const void *X_at, void *grad_out,
                 int64_t *bad_row, hipStream_t s);
// Dual-form half-sweep over the plan's dual bins (sweep_dual.hip): for each
// row u = Y_I^T (Y_I Y_I^T + lambda n_i I)^{-1} r_i, the same solution as
// Eq. (3) when lambda > 0.  Optional fused gradient as launch_sweep.
int launch_sweep_dual(const Plan *plan, const als_csr *R, const void *Y, void *X, int n_f, int ld,
                      double lambda, als_dtype dt, const void *X_at, void *grad_out,
                      int64_t *bad_row, hipStream_t s);
int launch_fold_in(Ctx *ctx, const void *M, int64_t n_items, int n_f, int ld, double lambda,
                   als_dtype dt, int64_t n_req, const int64_t *indptr, const int32_t *items,
                   const float *vals, void *U_out, int32_t *status, hipStream_t s);
// out[0] = bit pattern of max |Y| over the n x n_f block of Y (row stride
// ld): the scale of the FP32 half-sweep's FP16-split Gram.  out holds
// kAbsMaxWords words (out[1..] per-workgroup maxima); two launches,
// stream-ordered, no memset.
constexpr int kAbsMaxParts = 2048;
constexpr int kAbsMaxWords = 1 + kAbsMaxParts;
int launch_abs_max_bits(const float *Y, int64_t n, int n_f, int ld, unsigned *out, hipStream_t s);
// Planned half-sweep over a caller-built plan with caller-provided split-K
// workspace (sweep_partial_bytes per split chunk) and per-row status (empty
// row: ALS_E_INVAL, not SPD: ALS_E_NOT_SPD, else 0).  Used by the fold-in
// server, which builds one plan per batch.
size_t sweep_partial_bytes(int n_f, als_dtype dt);
// ybits: launch_abs_max_bits of Y (FP32; ignored for FP64).
int launch_sweep_batch(const Plan *plan, const als_csr *R, const void *Y, const unsigned *ybits,
                       void *X, int n_f, int ld, double lambda, als_dtype dt, void *partial,
                       int32_t *status, hipStream_t s);
// Reduced-precision half-sweep (BF16 copies, BF16 MFMA Gram, FP32 solve,
// optional refinement against the FP32 factors); planned only.
int launch_sweep_mixed(Ctx *ctx, const Plan *plan, const als_csr *R, const void *Y16,
                       const float *Y32, float *X32, void *X16, int n_f, int ld, double lambda,
                       int refine, int64_t *bad_row, hipStream_t s);
int launch_to_bf16(int64_t n, const float *x, void *y, hipStream_t s);
int launch_gradient(Ctx *ctx, const Plan *pR, const als_csr *R, const Plan *pRt, const als_csr *Rt,
                    const void *U, const void *M, int n_f, int ld, double lambda, als_dtype dt,
                    void *gU, void *gM, double *out2, hipStream_t s);
// Blocks of the item-regulariser kernel of the coefficient pass (one
// partial each, after the per-chunk partials).
constexpr int kCoeffItemBlocks = 512;
// fixed != nullptr: use these fixed_doubles doubles of device memory for the
// per-chunk partial sums instead of the context's workspace (ALS_E_BUDGET
// when they do not fit; nothing is allocated).
int launch_coeffs(Ctx *ctx, const Plan *pR, const als_csr *R, const als_csr *Rt, const void *U,
                  const void *M, const void *pU, const void *pM, int n_f, int ld, double lambda,
                  als_dtype dt, double *coeffs, const double *pred, hipStream_t s,
                  double *fixed = nullptr, size_t fixed_doubles = 0);
int launch_backtrack(const double *coeffs, double alpha0, double tau, double c, int max_trials,
                     double *alpha_out, int32_t *trials_out, double *q_out, hipStream_t s);
int launch_axpy(int64_t n, void *x, const void *p, const double *alpha, als_dtype dt,
                hipStream_t s);
int launch_axpby(int64_t n, double a, const void *x, double b, void *y, als_dtype dt,
                 hipStream_t s);
int launch_direction(Ctx *ctx, int64_t n, const void *x, void *xbar, const void *g_new,
                     const void *g_old, void *p, double *scal, int restart,
                     const double *restart_dev, int pr_plus, als_dtype dt, hipStream_t s);
// Device-side line-search control (Algorithm 4 with the safeguards), see
// ncg_linesearch_step in the header for the state layout.
constexpr int kLsState = 32;
int launch_ls_first(double *state, int exact, double alpha0, double tau, double c, int max_trials,
                    hipStream_t s);
int launch_ls_restart_dir(int64_t n, void *p, const void *gbar, const double *state, als_dtype dt,
                          hipStream_t s);
int launch_ls_final(double *state, int exact, double alpha0, double tau, double c, int max_trials,
                    hipStream_t s);
int launch_quartic_min(const double *coeffs, double c, double *alpha_out, int32_t *trials_out,
                       double *q_out, hipStream_t s);

// Top-t rankings and ranking accuracy (rank.hip).
int launch_rank_top(const void *U, const void *M, int64_t n_u, int n_m, int n_f, int ld,
                    als_dtype dt, int t, int32_t *top, hipStream_t s);
int launch_rank_accuracy(Ctx *ctx, const void *U, const void *M, int64_t n_u, int n_m, int n_f,
                         int ld, als_dtype dt, int t, const int32_t *top, int64_t *swaps,
                         double *mean_q, hipStream_t s);

// Deterministic FP64 column sums of a row-major [rows, cols] array, cols <= 8
// (two launches, fixed order).  out[k] = sum_r parts[r * cols + k] (+ out[k]
// when accumulate != 0).  stage: device scratch of kSumStageDoubles doubles.
constexpr int kSumStageDoubles = 256 * 8;
void launch_sum_columns(const double *parts, int64_t rows, int cols, double *out, int accumulate,
                        double *stage, hipStream_t s);

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace alsncg

#define ALS_HIP_CHECK(expr)                                   \
    do {                                                      \
        hipError_t e_ = (expr);                               \
        if (e_ != hipSuccess) return ALS_E_HIP;               \
    } while (0)
