// C ABI of libalsncg: context, workspace, row plans and the argument checks
// in front of every kernel launch.  The declarations and their contracts are
// in include/alsncg.h.
#include <math.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "internal.h"

namespace alsncg {

// Fixed device scratch of linesearch_coeffs_noalloc: 2^22 doubles (32 MiB)
// per device, alive until the process ends.  Host code never uses this name
// as an address: als_ctx_create looks up its device address once, with the
// device current, and keeps it in the context.
constexpr size_t kScratchDoubles = size_t(1) << 22;
static __device__ __align__(256) double scratch[kScratchDoubles];

void *Ctx::workspace(size_t bytes, hipStream_t stream, int *err) {
    if (bytes == 0) bytes = 256;
    if (bytes <= ws_bytes) return ws;
    if (ws) {
        // earlier launches on this stream may still read the old buffer
        if (hipStreamSynchronize(stream) != hipSuccess) {
            *err = ALS_E_HIP;
            return nullptr;
        }
        (void)hipFree(ws);
        ws = nullptr;
        ws_bytes = 0;
    }
    const size_t want = align_up(bytes + bytes / 4, 1 << 20);
    if (hipMalloc(&ws, want) != hipSuccess) {
        ws = nullptr;
        *err = ALS_E_NOMEM;
        return nullptr;
    }
    ws_bytes = want;
    return ws;
}

void *Ctx::split_buffer(size_t bytes, hipStream_t stream, int *err) {
    if (bytes == 0) bytes = 256;
    if (bytes <= ysplit_bytes) return ysplit;
    if (ysplit) {
        if (hipStreamSynchronize(stream) != hipSuccess) {
            *err = ALS_E_HIP;
            return nullptr;
        }
        (void)hipFree(ysplit);
        ysplit = nullptr;
        ysplit_bytes = 0;
    }
    const size_t want = align_up(bytes, 1 << 20);
    if (hipMalloc(&ysplit, want) != hipSuccess) {
        ysplit = nullptr;
        *err = ALS_E_NOMEM;
        return nullptr;
    }
    ysplit_bytes = want;
    return ysplit;
}

static bool dtype_ok(als_dtype dt, int n_f, bool sweep) {
    if (n_f < 1) return false;
    if (dt == ALS_F32) return sweep ? n_f <= 143 : n_f <= 144;
    if (dt == ALS_F64) return sweep ? n_f <= 95 : n_f <= 144;
    return false;
}

static bool csr_ok(const als_csr *R) {
    if (!R || R->n_rows < 0 || R->n_cols < 0 || R->nnz < 0) return false;
    if (R->n_rows > INT32_MAX || R->n_cols > INT32_MAX) return false;
    if (!R->indptr) return false;
    if (R->nnz > 0 && (!R->indices || !R->values)) return false;
    return true;
}

// Any plan of R's shape (the gradient pass); plan_matches: one that is not
// cut at column slices (every other call).
static bool grad_plan_matches(const Plan *p, const als_csr *R) {
    return p && p->n_rows == R->n_rows && p->nnz == R->nnz;
}

static bool plan_matches(const Plan *p, const als_csr *R) {
    return grad_plan_matches(p, R) && p->col_slices == 0;
}

static bool lambda_ok(double lambda) { return lambda >= 0.0 && isfinite(lambda); }

template <typename V>
static int copy_in(V *dst, const std::vector<V> &src) {
    if (src.empty()) return ALS_OK;
    return hipMemcpy(dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice) == hipSuccess
               ? ALS_OK
               : ALS_E_HIP;
}

template <typename V>
static int upload(V **dst, const std::vector<V> &src) {
    *dst = nullptr;
    const size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(V);
    if (hipMalloc((void **)dst, bytes) != hipSuccess) {
        *dst = nullptr;
        return ALS_E_NOMEM;
    }
    if (!src.empty() && hipMemcpy(*dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice) != hipSuccess)
        return ALS_E_HIP;
    return ALS_OK;
}

}  // namespace alsncg

using namespace alsncg;

extern "C" {

const char *als_strerror(int status) {
    switch (status) {
        case ALS_OK: return "ok";
        case ALS_E_INVAL: return "invalid argument";
        case ALS_E_HIP: return "HIP runtime error";
        case ALS_E_NOT_SPD: return "normal equations not positive definite";
        case ALS_E_NONFINITE: return "non-finite value";
        case ALS_E_NOMEM: return "device allocation failed";
        case ALS_E_BUDGET: return "request exceeds the stated limit";
        default: return "unknown status";
    }
}

int als_ctx_create(als_ctx **out, int device) {
    if (!out) return ALS_E_INVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return ALS_E_HIP;
    if (device < 0 || device >= n) return ALS_E_INVAL;
    if (hipSetDevice(device) != hipSuccess) return ALS_E_HIP;
    als_ctx *c = new (std::nothrow) als_ctx();
    if (!c) return ALS_E_NOMEM;
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->num_cu = prop.multiProcessorCount;
    void *sp = nullptr;
    if (hipGetSymbolAddress(&sp, HIP_SYMBOL(alsncg::scratch)) != hipSuccess || !sp) {
        delete c;
        return ALS_E_HIP;
    }
    c->scratch = (double *)sp;
    c->scratch_doubles = alsncg::kScratchDoubles;
    if (hipMalloc((void **)&c->ybits, alsncg::kAbsMaxWords * sizeof(unsigned)) != hipSuccess) {
        delete c;
        return ALS_E_NOMEM;
    }
    *out = c;
    return ALS_OK;
}

void als_ctx_destroy(als_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->ybits) (void)hipFree(ctx->ybits);
    if (ctx->ysplit) (void)hipFree(ctx->ysplit);
    delete ctx;
}

size_t als_ctx_workspace_bytes(const als_ctx *ctx) { return ctx ? ctx->ws_bytes : 0; }

void als_plan_destroy(als_plan *p) {
    if (!p) return;
    void *bufs[] = {p->chunk_row, p->chunk_begin, p->chunk_len, p->chunk_slot,
                    p->split_row, p->split_slot0, p->split_nslot, p->slot_chunk};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    delete p;
}

int als_plan_set_grid(als_plan *p, int64_t sweep_grid, int64_t pass_grid) {
    if (!p || sweep_grid < 0 || sweep_grid > INT32_MAX || pass_grid < 0 || pass_grid > INT32_MAX)
        return ALS_E_INVAL;
    p->grid = sweep_grid;
    p->grid_pass = pass_grid;
    return ALS_OK;
}

int als_plan_set_split_copy(als_plan *p, int mode) {
    if (!p || mode < -1 || mode > 1 || p->col_slices) return ALS_E_INVAL;
    p->split_copy = mode;
    return ALS_OK;
}

int als_plan_info(const als_plan *p, int64_t out[8]) {
    if (!p || !out) return ALS_E_INVAL;
    out[0] = p->n_rows;
    out[1] = p->nnz;
    out[2] = p->n_chunks;
    out[3] = p->n_split_rows;
    out[4] = p->n_slots;
    out[5] = p->chunk;
    out[6] = p->max_row;
    out[7] = p->n_dual;
    return ALS_OK;
}

int als_plan_set_dual(als_plan *p, int64_t max_len) {
    if (!p || max_len < 0 || max_len > alsncg::kDualMaxLen || p->col_slices) return ALS_E_INVAL;
    max_len = std::min<int64_t>(max_len, p->chunk);  // dual rows are whole rows
    const size_t nc = p->h_row.size();
    auto is_dual = [&](size_t k) {
        return p->h_slot[k] < 0 && p->h_len[k] >= 1 && p->h_len[k] <= max_len;
    };
    // current order is (non-dual, then dual rows) each longest first; rebuild
    // it as all chunks longest first, then move the new dual rows last
    std::vector<size_t> order(nc);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t b) { return p->h_len[a] > p->h_len[b]; });
    std::stable_partition(order.begin(), order.end(), [&](size_t k) { return !is_dual(k); });
    std::vector<int32_t> row(nc), len(nc), slot(nc);
    std::vector<int64_t> beg(nc);
    int64_t n_dual = 0;
    for (size_t k = 0; k < nc; ++k) {
        row[k] = p->h_row[order[k]];
        len[k] = p->h_len[order[k]];
        slot[k] = p->h_slot[order[k]];
        beg[k] = p->h_beg[order[k]];
        n_dual += is_dual(order[k]) ? 1 : 0;
    }
    if (hipDeviceSynchronize() != hipSuccess) return ALS_E_HIP;  // no launch may read the old order
    int rc = copy_in(p->chunk_row, row);
    if (rc == ALS_OK) rc = copy_in(p->chunk_begin, beg);
    if (rc == ALS_OK) rc = copy_in(p->chunk_len, len);
    if (rc == ALS_OK) rc = copy_in(p->chunk_slot, slot);
    if (rc == ALS_OK && p->n_slots > 0) {
        std::vector<int32_t> slot_chunk((size_t)p->n_slots, 0);
        for (size_t k = 0; k < nc; ++k)
            if (slot[k] >= 0) slot_chunk[(size_t)slot[k]] = (int32_t)k;
        rc = copy_in(p->slot_chunk, slot_chunk);
    }
    if (rc != ALS_OK) return rc;
    p->h_row.swap(row);
    p->h_len.swap(len);
    p->h_slot.swap(slot);
    p->h_beg.swap(beg);
    p->dual_max = max_len;
    p->n_dual = n_dual;
    for (int b = 0; b < 8; ++b) p->dual_first[b] = p->dual_count[b] = 0;
    for (int64_t k = (int64_t)nc - n_dual; k < (int64_t)nc; ++k) {
        const int64_t n = p->h_len[(size_t)k];
        const int b = n == 1 ? 0 : (int)((n + 2 + 15) / 16);  // bin 0: one rating
        if (p->dual_count[b] == 0) p->dual_first[b] = k;
        ++p->dual_count[b];
    }
    return ALS_OK;
}

// Longest chunk the automatic plan uses (ratings per wavefront).
static constexpr int64_t kMaxAutoChunk = 8192;

int als_plan_create(als_ctx *ctx, const als_csr *R, int64_t chunk, als_plan **out) {
    if (!out) return ALS_E_INVAL;
    *out = nullptr;
    if (!ctx || !csr_ok(R) || chunk < 0) return ALS_E_INVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return ALS_E_HIP;
    const int64_t n = R->n_rows;
    std::vector<int64_t> ip((size_t)n + 1);
    if (hipDeviceSynchronize() != hipSuccess) return ALS_E_HIP;
    if (hipMemcpy(ip.data(), R->indptr, ip.size() * sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess)
        return ALS_E_HIP;
    if (ip[0] != 0 || ip[(size_t)n] != R->nnz) return ALS_E_INVAL;
    int64_t max_row = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t len = ip[i + 1] - ip[i];
        if (len < 0 || len > R->n_cols) return ALS_E_INVAL;
        max_row = std::max(max_row, len);
    }
    if (chunk == 0) {
        // at most the average work of one resident wavefront slot (8 per CU):
        // longer rows are split so that no single wave dominates the launch.
        // Capped at kMaxAutoChunk: an FP32 MFMA accumulator then sums at most
        // kMaxAutoChunk / 4 steps; longer rows are reduced by the fixed-order
        // second stage (VALU adds, rounded to nearest), which keeps the Gram
        // of rows with millions of ratings accurate.
        const int64_t slots = (int64_t)ctx->num_cu * 8;
        chunk = std::max<int64_t>(256, (R->nnz + slots - 1) / slots);
        chunk = std::min<int64_t>(chunk, kMaxAutoChunk);
        chunk = (chunk + 3) / 4 * 4;
    }
    chunk = std::min<int64_t>(chunk, INT32_MAX / 2);
    std::vector<int32_t> crow, clen, cslot, srow, sslot0, snslot;
    std::vector<int64_t> cbeg;
    int64_t slots = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t len = ip[i + 1] - ip[i];
        const int64_t nck = len <= chunk ? 1 : (len + chunk - 1) / chunk;
        if (nck == 1) {
            crow.push_back((int32_t)i);
            cbeg.push_back(ip[i]);
            clen.push_back((int32_t)len);
            cslot.push_back(-1);
            continue;
        }
        int64_t per = (len + nck - 1) / nck;
        per = (per + 3) / 4 * 4;
        const int64_t s0 = slots;
        int32_t ns = 0;
        for (int64_t o = 0; o < len; o += per) {
            crow.push_back((int32_t)i);
            cbeg.push_back(ip[i] + o);
            clen.push_back((int32_t)std::min(per, len - o));
            cslot.push_back((int32_t)(slots++));
            ++ns;
        }
        srow.push_back((int32_t)i);
        sslot0.push_back((int32_t)s0);
        snslot.push_back(ns);
    }
    if (slots > INT32_MAX) return ALS_E_INVAL;
    // longest chunks first: the hardware dispatcher then schedules greedily
    std::vector<int64_t> order(crow.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return clen[a] > clen[b]; });
    std::vector<int32_t> crow2(order.size()), clen2(order.size()), cslot2(order.size());
    std::vector<int64_t> cbeg2(order.size());
    for (size_t k = 0; k < order.size(); ++k) {
        crow2[k] = crow[order[k]];
        cbeg2[k] = cbeg[order[k]];
        clen2[k] = clen[order[k]];
        cslot2[k] = cslot[order[k]];
    }
    als_plan *p = new (std::nothrow) als_plan();
    if (!p) return ALS_E_NOMEM;
    p->n_rows = n;
    p->nnz = R->nnz;
    p->n_chunks = (int64_t)crow2.size();
    p->n_split_rows = (int64_t)srow.size();
    p->n_slots = slots;
    p->chunk = chunk;
    p->max_row = max_row;
    int rc = ALS_OK;
    if (rc == ALS_OK) rc = upload(&p->chunk_row, crow2);
    if (rc == ALS_OK) rc = upload(&p->chunk_begin, cbeg2);
    if (rc == ALS_OK) rc = upload(&p->chunk_len, clen2);
    if (rc == ALS_OK) rc = upload(&p->chunk_slot, cslot2);
    if (rc == ALS_OK) {
        p->h_row = crow2;
        p->h_len = clen2;
        p->h_slot = cslot2;
        p->h_beg = cbeg2;
    }
    if (rc == ALS_OK) rc = upload(&p->split_row, srow);
    if (rc == ALS_OK) rc = upload(&p->split_slot0, sslot0);
    if (rc == ALS_OK) rc = upload(&p->split_nslot, snslot);
    if (rc == ALS_OK) {
        std::vector<int32_t> slot_chunk((size_t)slots, 0);
        for (size_t k = 0; k < cslot2.size(); ++k)
            if (cslot2[k] >= 0) slot_chunk[(size_t)cslot2[k]] = (int32_t)k;
        rc = upload(&p->slot_chunk, slot_chunk);
    }
    if (rc != ALS_OK) {
        als_plan_destroy(p);
        return rc;
    }
    *out = p;
    return ALS_OK;
}

// Column slices of a sliced plan: at most this many.
static constexpr int64_t kMaxColSlices = 4096;

int als_plan_create_sliced(als_ctx *ctx, const als_csr *R, int64_t chunk, int64_t n_slices,
                           als_plan **out) {
    if (!out) return ALS_E_INVAL;
    *out = nullptr;
    if (!ctx || !csr_ok(R) || chunk < 0 || n_slices < 1 || n_slices > kMaxColSlices)
        return ALS_E_INVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return ALS_E_HIP;
    const int64_t n = R->n_rows, nnz = R->nnz, n_cols = R->n_cols;
    std::vector<int64_t> ip((size_t)n + 1);
    std::vector<int32_t> ix((size_t)nnz);
    if (hipDeviceSynchronize() != hipSuccess) return ALS_E_HIP;
    if (hipMemcpy(ip.data(), R->indptr, ip.size() * sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess)
        return ALS_E_HIP;
    if (nnz > 0 &&
        hipMemcpy(ix.data(), R->indices, ix.size() * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
        return ALS_E_HIP;
    if (ip[0] != 0 || ip[(size_t)n] != nnz) return ALS_E_INVAL;
    // rows must hold ascending column ids: a slice is then one contiguous
    // segment of every row
    int64_t max_row = 0;
    std::vector<int64_t> col_count((size_t)n_cols + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t b = ip[(size_t)i], e = ip[(size_t)i + 1];
        if (e < b || e - b > n_cols) return ALS_E_INVAL;
        max_row = std::max(max_row, e - b);
        for (int64_t k = b; k < e; ++k) {
            if (ix[(size_t)k] < 0 || ix[(size_t)k] >= n_cols) return ALS_E_INVAL;
            if (k > b && ix[(size_t)k] <= ix[(size_t)k - 1]) return ALS_E_INVAL;
            ++col_count[(size_t)ix[(size_t)k] + 1];
        }
    }
    if (chunk == 0) {
        const int64_t slots = (int64_t)ctx->num_cu * 8;
        chunk = std::max<int64_t>(256, (nnz + slots - 1) / slots);
        chunk = std::min<int64_t>(chunk, kMaxAutoChunk);
        chunk = (chunk + 3) / 4 * 4;
    }
    chunk = std::min<int64_t>(chunk, INT32_MAX / 2);
    // slice boundaries: columns [bound[s], bound[s + 1]) hold about nnz / S
    // ratings each (prefix counts of the column ids)
    const int64_t S = n_slices;
    std::partial_sum(col_count.begin(), col_count.end(), col_count.begin());
    std::vector<int64_t> bound((size_t)S + 1);
    bound[0] = 0;
    bound[(size_t)S] = n_cols;
    for (int64_t s = 1; s < S; ++s) {
        const int64_t target = (nnz * s + S - 1) / S;
        bound[(size_t)s] =
            std::lower_bound(col_count.begin(), col_count.end(), target) - col_count.begin();
        bound[(size_t)s] = std::min(std::max(bound[(size_t)s], bound[(size_t)s - 1]), n_cols);
    }
    // pieces of every row: one per non-empty slice segment, segments longer
    // than `chunk` cut further; a row of more than one piece is a split row
    std::vector<std::vector<int64_t>> by_slice((size_t)S);  // piece ids per slice
    std::vector<int32_t> crow, clen, cslot, srow, sslot0, snslot;
    std::vector<int64_t> cbeg;
    std::vector<int64_t> seg_s, seg_b, seg_e;
    int64_t slots = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t b = ip[(size_t)i], e = ip[(size_t)i + 1];
        seg_s.clear();
        seg_b.clear();
        seg_e.clear();
        int64_t pieces = 0, p0 = b;
        for (int64_t s = 0; s < S && p0 < e; ++s) {
            const int64_t q =
                std::lower_bound(ix.begin() + p0, ix.begin() + e, (int32_t)std::min<int64_t>(bound[(size_t)s + 1], INT32_MAX)) -
                ix.begin();
            if (q > p0) {
                seg_s.push_back(s);
                seg_b.push_back(p0);
                seg_e.push_back(q);
                const int64_t len = q - p0;
                pieces += len <= chunk ? 1 : (len + chunk - 1) / chunk;
            }
            p0 = q;
        }
        if (pieces <= 1) {
            // the whole row in one piece; an empty row (its gradient row is
            // written as zeros) goes to slice i mod S
            by_slice[(size_t)(pieces ? seg_s[0] : i % S)].push_back((int64_t)crow.size());
            crow.push_back((int32_t)i);
            cbeg.push_back(b);
            clen.push_back((int32_t)(e - b));
            cslot.push_back(-1);
            continue;
        }
        const int64_t s0 = slots;
        for (size_t t = 0; t < seg_s.size(); ++t) {
            const int64_t len = seg_e[t] - seg_b[t];
            const int64_t nck = len <= chunk ? 1 : (len + chunk - 1) / chunk;
            const int64_t per = (len + nck - 1) / nck;
            for (int64_t o = 0; o < len; o += per) {
                by_slice[(size_t)seg_s[t]].push_back((int64_t)crow.size());
                crow.push_back((int32_t)i);
                cbeg.push_back(seg_b[t] + o);
                clen.push_back((int32_t)std::min(per, len - o));
                cslot.push_back((int32_t)(slots++));
            }
        }
        srow.push_back((int32_t)i);
        sslot0.push_back((int32_t)s0);
        snslot.push_back((int32_t)(slots - s0));
    }
    if (slots >= INT32_MAX) return ALS_E_INVAL;
    // launch order: slice s on die s mod kXcds, slices s and s + kXcds one
    // after the other (phase s / kXcds); position kXcds k + x of a phase is
    // the k-th longest piece of its slice, or an empty piece that writes
    // zeros to a spare slot when the slice has fewer
    std::vector<int32_t> crow2, clen2, cslot2;
    std::vector<int64_t> cbeg2;
    const int32_t spare = (int32_t)slots;
    bool padded = false;
    for (int64_t ph = 0; ph * kXcds < S; ++ph) {
        size_t K = 0;
        for (int64_t x = 0; x < kXcds && ph * kXcds + x < S; ++x) {
            auto &v = by_slice[(size_t)(ph * kXcds + x)];
            std::stable_sort(v.begin(), v.end(), [&](int64_t a, int64_t c) { return clen[(size_t)a] > clen[(size_t)c]; });
            K = std::max(K, v.size());
        }
        for (size_t k = 0; k < K; ++k)
            for (int64_t x = 0; x < kXcds; ++x) {
                const int64_t s = ph * kXcds + x;
                if (s < S && k < by_slice[(size_t)s].size()) {
                    const size_t c = (size_t)by_slice[(size_t)s][k];
                    crow2.push_back(crow[c]);
                    cbeg2.push_back(cbeg[c]);
                    clen2.push_back(clen[c]);
                    cslot2.push_back(cslot[c]);
                } else {
                    crow2.push_back(0);
                    cbeg2.push_back(0);
                    clen2.push_back(0);
                    cslot2.push_back(spare);
                    padded = true;
                }
            }
    }
    als_plan *p = new (std::nothrow) als_plan();
    if (!p) return ALS_E_NOMEM;
    p->n_rows = n;
    p->nnz = nnz;
    p->n_chunks = (int64_t)crow2.size();
    p->n_split_rows = (int64_t)srow.size();
    p->n_slots = slots + (padded ? 1 : 0);
    p->chunk = chunk;
    p->max_row = max_row;
    p->col_slices = S;
    int rc = upload(&p->chunk_row, crow2);
    if (rc == ALS_OK) rc = upload(&p->chunk_begin, cbeg2);
    if (rc == ALS_OK) rc = upload(&p->chunk_len, clen2);
    if (rc == ALS_OK) rc = upload(&p->chunk_slot, cslot2);
    if (rc == ALS_OK) rc = upload(&p->split_row, srow);
    if (rc == ALS_OK) rc = upload(&p->split_slot0, sslot0);
    if (rc == ALS_OK) rc = upload(&p->split_nslot, snslot);
    if (rc == ALS_OK) {
        std::vector<int32_t> slot_chunk((size_t)p->n_slots, 0);
        for (size_t k = 0; k < cslot2.size(); ++k)
            if (cslot2[k] >= 0) slot_chunk[(size_t)cslot2[k]] = (int32_t)k;
        rc = upload(&p->slot_chunk, slot_chunk);
    }
    if (rc == ALS_OK) {
        p->h_row = crow2;
        p->h_len = clen2;
        p->h_slot = cslot2;
        p->h_beg = cbeg2;
    }
    if (rc != ALS_OK) {
        als_plan_destroy(p);
        return rc;
    }
    *out = p;
    return ALS_OK;
}

int als_sweep(als_ctx *ctx, const als_plan *plan, const als_csr *R, const void *Y, void *X,
              int n_f, int ld, double lambda, als_dtype dt, const void *X_at, void *grad_out,
              int64_t *bad_row, void *stream) {
    if (!ctx || !csr_ok(R) || !plan_matches(plan, R) || !X || ld < n_f || !lambda_ok(lambda) ||
        !dtype_ok(dt, n_f, true))
        return ALS_E_INVAL;
    if (!Y && R->nnz > 0) return ALS_E_INVAL;
    if (Y == X) return ALS_E_INVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return ALS_E_HIP;
    if (grad_out && (grad_out == X || grad_out == X_at || grad_out == Y)) return ALS_E_INVAL;
    return launch_sweep(ctx, plan, R, Y, X, n_f, ld, lambda, dt, X_at, grad_out, bad_row,
                        (hipStream_t)stream);
}

int als_sweep_mixed(als_ctx *ctx, const als_plan *plan, const als_csr *R, const void *Y16,
                    const float *Y32, float *X32, void *X16, int n_f, int ld, double lambda,
                    int refine, int64_t *bad_row, void *stream) {
    if (!ctx || !csr_ok(R) || !plan_matches(plan, R) || !X32 || ld < n_f || n_f < 1 || n_f > 143 ||
        !lambda_ok(lambda))
        return ALS_E_INVAL;
    if (R->nnz > 0 && (!Y16 || (refine && !Y32))) return ALS_E_INVAL;
    if ((const void *)X32 == Y16 || X32 == Y32 ||
        (X16 && (X16 == Y16 || X16 == (const void *)Y32 || X16 == (void *)X32)))
        return ALS_E_INVAL;
    if (plan->n_slots > 0 && !plan->slot_chunk) return ALS_E_INVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return ALS_E_HIP;
    return launch_sweep_mixed(ctx, plan, R, Y16, Y32, X32, X16, n_f, ld, lambda, refine, bad_row,
                              (hipStream_t)stream);
}

int als_to_bf16(als_ctx *ctx, int64_t n, const float *x, void *y, void *stream) {
    if (!ctx || n < 0 || (n > 0 && (!x || !y))) return ALS_E_INVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return ALS_E_HIP;
    return launch_to_bf16(n, x, y, (hipStream_t)stream);
}

int ncg_gradient(als_ctx *ctx, const als_plan *plan_R, const als_csr *R, const als_plan *plan_Rt,
                 const als_csr *Rt, const void *U, const void *M, int n_f, int ld, double lambda,
                 als_dtype dt, void *gU, void *gM, double *out2, void *stream) {
    if (!ctx || !csr_ok(R) || !csr_ok(Rt) || !grad_plan_matches(plan_R, R) ||
        !grad_plan_matches(plan_Rt, Rt) || !U || !M || ld < n_f || !lambda_ok(lambda) ||
        !dtype_ok(dt, n_f, false))
        return ALS_E_INVAL;
    if (R->n_rows != Rt->n_cols || R->n_cols != Rt->n_rows || R->nnz != Rt->nnz) return ALS_E_INVAL;
    if (!gU && !gM && !out2) return ALS_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return ALS_E_HIP;
    return launch_gradient(ctx, plan_R, R, plan_Rt, Rt, U, M, n_f, ld, lambda, dt, gU, gM, out2,
                           (hipStream_t)stream);
}

int linesearch_coeffs(als_ctx *ctx, const als_plan *plan_R, const als_csr *R, const als_csr *Rt,
                      const void *U, const void *M, const void *pU, const void *pM, int n_f,
                      int ld, double lambda, als_dtype dt, double *coeffs, void *stream) {
    if (!ctx || !csr_ok(R) || !Rt || !Rt->indptr || !plan_matches(plan_R, R) || !U || !M ||
        !pU || !pM || !coeffs || ld < n_f || !lambda_ok(lambda) || !dtype_ok(dt, n_f, false))
        return ALS_E_INVAL;
    if (Rt->n_rows != R->n_cols) return ALS_E_INVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return ALS_E_HIP;
    return launch_coeffs(ctx, plan_R, R, Rt, U, M, pU, pM, n_f, ld, lambda, dt, coeffs, nullptr,
                         (hipStream_t)stream);
}

int linesearch_coeffs_noalloc(als_ctx *ctx, const als_plan *plan_R, const als_csr *R,
                              const als_csr *Rt, const void *U, const void *M, const void *pU,
                              const void *pM, int n_f, int ld, double lambda, als_dtype dt,
                              double *coeffs, void *stream) {
    if (!ctx || !csr_ok(R) || !Rt || !Rt->indptr || !plan_matches(plan_R, R) || !U || !M ||
        !pU || !pM || !coeffs || ld < n_f || !lambda_ok(lambda) || !dtype_ok(dt, n_f, false))
        return ALS_E_INVAL;
    if (Rt->n_rows != R->n_cols) return ALS_E_INVAL;
    if (!ctx->scratch) return ALS_E_HIP;
    if (hipSetDevice(ctx->device) != hipSuccess) return ALS_E_HIP;
    return launch_coeffs(ctx, plan_R, R, Rt, U, M, pU, pM, n_f, ld, lambda, dt, coeffs, nullptr,
                         (hipStream_t)stream, ctx->scratch, ctx->scratch_doubles);
}

size_t linesearch_coeffs_noalloc_max_chunks(void) {
    return (alsncg::kScratchDoubles - alsncg::kSumStageDoubles) / 5 - alsncg::kCoeffItemBlocks;
}

int ncg_backtrack(als_ctx *ctx, const double *coeffs, double alpha0, double tau, double c,
                  int max_trials, double *alpha_out, int32_t *trials_out, double *q_out,
                  void *stream) {
    if (!ctx || !coeffs || !alpha_out || !(alpha0 > 0.0) || !(tau > 0.0 && tau < 1.0) ||
        !(c > 0.0 && c < 1.0) || max_trials < 1)
        return ALS_E_INVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return ALS_E_HIP;
    return launch_backtrack(coeffs, alpha0, tau, c, max_trials, alpha_out, trials_out, q_out,
                            (hipStream_t)stream);
}

int ncg_linesearch_exact(als_ctx *ctx, const double *coeffs, double c, double *alpha_out,
                         int32_t *trials_out, double *q_out, void *stream) {
    if (!ctx || !coeffs || !alpha_out || !(c > 0.0 && c < 1.0)) return ALS_E_INVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return ALS_E_HIP;
    return launch_quartic_min(coeffs, c, alpha_out, trials_out, q_out, (hipStream_t)stream);
}

int ncg_axpy(als_ctx *ctx, int64_t n, void *x, const void *p, const double *alpha, als_dtype dt,
             void *stream) {
    if (!ctx || n < 0 || (n > 0 && (!x || !p)) || !alpha) return ALS_E_INVAL;
    if (dt != ALS_F32 && dt != ALS_F64) return ALS_E_INVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return ALS_E_HIP;
    return launch_axpy(n, x, p, alpha, dt, (hipStream_t)stream);
}

int ncg_axpby(als_ctx *ctx, int64_t n, double a, const void *x, double b, void *y,
              als_dtype dt, void *stream) {
    if (!ctx || n < 0 || (n > 0 && (!x || !y)) || !isfinite(a) || !isfinite(b)) return ALS_E_INVAL;
    if (dt != ALS_F32 && dt != ALS_F64) return ALS_E_INVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return ALS_E_HIP;
    return launch_axpby(n, a, x, b, y, dt, (hipStream_t)stream);
}

int ncg_direction(als_ctx *ctx, int64_t n, const void *x, void *xbar, const void *g_new,
                  const void *g_old, void *p, double *scal, int restart, int pr_plus,
                  als_dtype dt, void *stream) {
    if (!ctx || n < 0 || !scal) return ALS_E_INVAL;
    if (n > 0 && (!x || !xbar || !g_new || !p || (!restart && !g_old))) return ALS_E_INVAL;
    if (dt != ALS_F32 && dt != ALS_F64) return ALS_E_INVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return ALS_E_HIP;
    return launch_direction(ctx, n, x, xbar, g_new, g_old, p, scal, restart, nullptr, pr_plus, dt,
                            (hipStream_t)stream);
}

int ncg_direction_dev(als_ctx *ctx, int64_t n, const void *x, void *xbar, const void *g_new,
                      const void *g_old, void *p, double *scal, const double *restart_flag,
                      int pr_plus, als_dtype dt, void *stream) {
    if (!ctx || n < 0 || !scal || !restart_flag) return ALS_E_INVAL;
    if (n > 0 && (!x || !xbar || !g_new || !g_old || !p)) return ALS_E_INVAL;
    if (dt != ALS_F32 && dt != ALS_F64) return ALS_E_INVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return ALS_E_HIP;
    return launch_direction(ctx, n, x, xbar, g_new, g_old, p, scal, 0, restart_flag, pr_plus, dt,
                            (hipStream_t)stream);
}

int ncg_linesearch_step(als_ctx *ctx, const als_plan *plan_R, const als_csr *R, const als_csr *Rt,
                        void *x, void *p, const void *gbar, int n_f, int ld, double lambda,
                        als_dtype dt, int search, double alpha0, double tau, double c,
                        int max_trials, double *state, void *stream) {
    if (search != 0 && search != 1) return ALS_E_INVAL;
    if (!ctx || !csr_ok(R) || !Rt || !Rt->indptr || !plan_matches(plan_R, R) || !x || !p ||
        !gbar || !state || ld < n_f || !lambda_ok(lambda) || !dtype_ok(dt, n_f, false))
        return ALS_E_INVAL;
    if (Rt->n_rows != R->n_cols || !(alpha0 > 0.0) || !(tau > 0.0 && tau < 1.0) ||
        !(c > 0.0 && c < 1.0) || max_trials < 1)
        return ALS_E_INVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return ALS_E_HIP;
    hipStream_t s = (hipStream_t)stream;
    const size_t elt = dt == ALS_F64 ? sizeof(double) : sizeof(float);
    const int64_t n_u = R->n_rows, n = (R->n_rows + R->n_cols) * (int64_t)ld;
    char *xU = (char *)x, *pU = (char *)p;
    char *xM = xU + (size_t)n_u * ld * elt, *pM = pU + (size_t)n_u * ld * elt;
    int rc = launch_coeffs(ctx, plan_R, R, Rt, xU, xM, pU, pM, n_f, ld, lambda, dt, state,
                           nullptr, s);
    if (rc == ALS_OK) rc = launch_ls_first(state, search, alpha0, tau, c, max_trials, s);
    if (rc == ALS_OK) rc = launch_ls_restart_dir(n, p, gbar, state, dt, s);
    if (rc == ALS_OK)
        rc = launch_coeffs(ctx, plan_R, R, Rt, xU, xM, pU, pM, n_f, ld, lambda, dt, state + 8,
                           state + 7, s);
    if (rc == ALS_OK) rc = launch_ls_final(state, search, alpha0, tau, c, max_trials, s);
    if (rc == ALS_OK) rc = launch_axpy(n, x, p, state + 21, dt, s);
    return rc;
}

static bool rank_args_ok(const void *U, const void *M, int64_t n_u, int64_t n_m, int n_f, int ld,
                         als_dtype dt, int t) {
    return U && M && n_u >= 0 && n_u <= INT32_MAX && n_m >= 1 && n_m <= INT32_MAX - 64 && n_f >= 1 &&
           n_f <= 128 && ld >= n_f && (dt == ALS_F32 || dt == ALS_F64) && t >= 1 && t <= 32 &&
           t <= n_m;
}

int rank_top_t(als_ctx *ctx, const void *U, const void *M, int64_t n_u, int64_t n_m, int n_f,
               int ld, als_dtype dt, int t, int32_t *top, void *stream) {
    if (!ctx || !top || !rank_args_ok(U, M, n_u, n_m, n_f, ld, dt, t)) return ALS_E_INVAL;
    return launch_rank_top(U, M, n_u, (int)n_m, n_f, ld, dt, t, top, (hipStream_t)stream);
}

int rank_accuracy(als_ctx *ctx, const void *U, const void *M, int64_t n_u, int64_t n_m, int n_f,
                  int ld, als_dtype dt, int t, const int32_t *top, int64_t *swaps, double *mean_q,
                  void *stream) {
    if (!ctx || !top || !rank_args_ok(U, M, n_u, n_m, n_f, ld, dt, t) || n_u < 1 || n_m < 2)
        return ALS_E_INVAL;
    return launch_rank_accuracy(ctx, U, M, n_u, (int)n_m, n_f, ld, dt, t, top, swaps, mean_q,
                                (hipStream_t)stream);
}

int fold_in(als_ctx *ctx, const void *M, int64_t n_items, int n_f, int ld, double lambda,
            als_dtype dt, int64_t n_req, const int64_t *req_indptr, const int32_t *req_items,
            const float *req_vals, void *U_out, int32_t *req_status, void *stream) {
    if (!ctx || !M || n_items < 0 || ld < n_f || !lambda_ok(lambda) || !dtype_ok(dt, n_f, true) ||
        n_req < 0 || n_req > INT32_MAX)
        return ALS_E_INVAL;
    if (n_req == 0) return ALS_OK;
    if (!req_indptr || !req_items || !req_vals || !U_out) return ALS_E_INVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return ALS_E_HIP;
    return launch_fold_in(ctx, M, n_items, n_f, ld, lambda, dt, n_req, req_indptr, req_items, req_vals,
                          U_out, req_status, (hipStream_t)stream);
}

}  // extern "C"
