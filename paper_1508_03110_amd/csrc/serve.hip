// Fold-in server: continuous batching of new-user solves against fixed item
// factors (the row solve of Eq. (3) applied to rows that are not in R).
//
// Host side only; the device work is the half-sweep kernel of sweep.hip run
// over a per-batch row plan.  Each of `max_inflight` slots owns a stream, a
// pinned staging buffer, a device input buffer, the batch's output and
// status arrays and its split-K workspace, all sized at creation from the
// HBM budget, so no allocation happens while serving.  A batch is formed
// whenever a slot is free: every queued request that fits (FIFO, up to
// max_batch requests and the slot's rating capacity) is packed as one CSR
// plus its plan, copied with one host-to-device transfer, solved, and its
// results copied back on the same stream; an event marks completion.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <new>
#include <numeric>
#include <vector>

#include "internal.h"

namespace alsncg {
namespace {

struct Req {
    int64_t id;
    int64_t n;
    const int32_t *items;  // host (caller memory) when store < 0
    const float *vals;
    int64_t store;         // else byte offset of [items | values] in the server's arena
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    char *h_in = nullptr;   // pinned: packed CSR + plan
    char *d_in = nullptr;
    size_t in_bytes = 0;
    char *h_out = nullptr;  // pinned: U rows (ld wide) then status
    char *d_out = nullptr;
    size_t out_bytes = 0;
    void *d_partial = nullptr;
    std::vector<int64_t> ids;
    int64_t rows = 0;
    bool busy = false;
};

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

}  // namespace
}  // namespace alsncg

using namespace alsncg;

struct als_server {
    Ctx *ctx = nullptr;
    const void *M = nullptr;
    // bits of max |M| (scale of the FP32 Gram), computed once: M does not
    // change while the server lives
    unsigned *ybits = nullptr;
    int64_t n_items = 0;
    int n_f = 0, ld = 0;
    double lambda = 0;
    als_dtype dt = ALS_F32;
    als_server_config cfg{};
    size_t elt = 4, partial_bytes = 0;
    int64_t cap_rows = 0, cap_ratings = 0, cap_chunks = 0, cap_split = 0;
    std::deque<Req> queue;
    std::vector<Slot> slots;
    std::vector<char> arena;  // copies of submitted requests
    int64_t arena_live = 0;
    int64_t inflight = 0;
    // finished but not yet reported (harvested batches)
    std::vector<int64_t> ready_ids;
    std::vector<int32_t> ready_status;
    std::vector<char> ready_U;
    int64_t ready_head = 0;
};

namespace {

// Bytes a slot needs for a batch of `rows` requests and `ratings` ratings
// cut into at most `chunks` chunks of which `split` are split chunks.
size_t in_bytes_for(int64_t rows, int64_t ratings, int64_t chunks, int64_t split) {
    return al((rows + 1) * 8) + al(ratings * 4) + al(ratings * 4) + al(chunks * 4) +
           al(chunks * 8) + al(chunks * 4) + al(chunks * 4) + al(rows * 4) * 3 + al(split * 4);
}

int launch_batch(als_server *S, Slot &sl, std::vector<Req> &batch) {
    const int64_t rows = (int64_t)batch.size();
    for (auto &r : batch)
        if (r.store >= 0) {
            r.items = (const int32_t *)(S->arena.data() + r.store);
            r.vals = (const float *)(S->arena.data() + r.store + r.n * 4);
        }
    int64_t ratings = 0;
    for (auto &r : batch) ratings += r.n;
    // plan: requests longer than `split` are cut into chunks of <= split ratings
    std::vector<int32_t> crow, clen, cslot, srow, sslot0, snslot;
    std::vector<int64_t> cbeg;
    std::vector<int64_t> ip(rows + 1, 0);
    int64_t slots = 0;
    for (int64_t q = 0; q < rows; ++q) {
        ip[q + 1] = ip[q] + batch[q].n;
        const int64_t n = batch[q].n;
        const int64_t sp = S->cfg.split;
        if (sp <= 0 || n <= sp) {
            crow.push_back((int32_t)q);
            cbeg.push_back(ip[q]);
            clen.push_back((int32_t)n);
            cslot.push_back(-1);
            continue;
        }
        const int64_t nck = (n + sp - 1) / sp;
        int64_t per = (n + nck - 1) / nck;
        per = (per + 3) / 4 * 4;
        const int64_t s0 = slots;
        int32_t ns = 0;
        for (int64_t o = 0; o < n; o += per) {
            crow.push_back((int32_t)q);
            cbeg.push_back(ip[q] + o);
            clen.push_back((int32_t)std::min(per, n - o));
            cslot.push_back((int32_t)(slots++));
            ++ns;
        }
        srow.push_back((int32_t)q);
        sslot0.push_back((int32_t)s0);
        snslot.push_back(ns);
    }
    std::vector<int64_t> order(crow.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return clen[a] > clen[b]; });
    const int64_t nch = (int64_t)order.size();
    // pack into pinned staging
    char *h = sl.h_in;
    size_t off = 0;
    auto put = [&](const void *src, size_t bytes) -> size_t {
        const size_t o = off;
        if (bytes) std::memcpy(h + off, src, bytes);
        off += al(bytes);
        return o;
    };
    const size_t o_ip = put(ip.data(), (rows + 1) * 8);
    const size_t o_it = off;
    for (auto &r : batch) {
        std::memcpy(h + off, r.items, r.n * 4);
        off += r.n * 4;
    }
    off = o_it + al(ratings * 4);
    const size_t o_va = off;
    for (auto &r : batch) {
        std::memcpy(h + off, r.vals, r.n * 4);
        off += r.n * 4;
    }
    off = o_va + al(ratings * 4);
    std::vector<int32_t> crow2(nch), clen2(nch), cslot2(nch);
    std::vector<int64_t> cbeg2(nch);
    for (int64_t k = 0; k < nch; ++k) {
        crow2[k] = crow[order[k]];
        cbeg2[k] = cbeg[order[k]];
        clen2[k] = clen[order[k]];
        cslot2[k] = cslot[order[k]];
    }
    const size_t o_cr = put(crow2.data(), nch * 4);
    const size_t o_cb = put(cbeg2.data(), nch * 8);
    const size_t o_cl = put(clen2.data(), nch * 4);
    const size_t o_cs = put(cslot2.data(), nch * 4);
    const size_t o_sr = put(srow.data(), srow.size() * 4);
    const size_t o_s0 = put(sslot0.data(), sslot0.size() * 4);
    const size_t o_sn = put(snslot.data(), snslot.size() * 4);
    if (off > sl.in_bytes) return ALS_E_BUDGET;  // cannot happen: admission checked the caps
    if (hipMemcpyAsync(sl.d_in, sl.h_in, off, hipMemcpyHostToDevice, sl.stream) != hipSuccess)
        return ALS_E_HIP;
    Plan plan;
    plan.n_rows = rows;
    plan.nnz = ratings;
    plan.n_chunks = nch;
    plan.n_split_rows = (int64_t)srow.size();
    plan.n_slots = slots;
    plan.chunk = S->cfg.split;
    plan.chunk_row = (int32_t *)(sl.d_in + o_cr);
    plan.chunk_begin = (int64_t *)(sl.d_in + o_cb);
    plan.chunk_len = (int32_t *)(sl.d_in + o_cl);
    plan.chunk_slot = (int32_t *)(sl.d_in + o_cs);
    plan.split_row = (int32_t *)(sl.d_in + o_sr);
    plan.split_slot0 = (int32_t *)(sl.d_in + o_s0);
    plan.split_nslot = (int32_t *)(sl.d_in + o_sn);
    als_csr R;
    R.n_rows = rows;
    R.n_cols = S->n_items;
    R.nnz = ratings;
    R.indptr = (const int64_t *)(sl.d_in + o_ip);
    R.indices = (const int32_t *)(sl.d_in + o_it);
    R.values = (const float *)(sl.d_in + o_va);
    const size_t u_bytes = al((size_t)rows * S->ld * S->elt);
    int32_t *d_status = (int32_t *)(sl.d_out + u_bytes);
    int rc = launch_sweep_batch(&plan, &R, S->M, S->ybits, sl.d_out, S->n_f, S->ld, S->lambda,
                                S->dt, sl.d_partial, d_status, sl.stream);
    if (rc != ALS_OK) return rc;
    if (hipMemcpyAsync(sl.h_out, sl.d_out, u_bytes + (size_t)rows * 4, hipMemcpyDeviceToHost,
                       sl.stream) != hipSuccess)
        return ALS_E_HIP;
    if (hipEventRecord(sl.done, sl.stream) != hipSuccess) return ALS_E_HIP;
    sl.ids.clear();
    for (auto &r : batch) sl.ids.push_back(r.id);
    sl.rows = rows;
    sl.busy = true;
    S->inflight += rows;
    return ALS_OK;
}

void finish_request(als_server *S, int64_t id, int32_t status, const char *u_row) {
    const size_t rb = (size_t)S->n_f * S->elt;
    S->ready_ids.push_back(id);
    S->ready_status.push_back(status);
    const size_t o = S->ready_U.size();
    S->ready_U.resize(o + rb);
    if (u_row)
        std::memcpy(S->ready_U.data() + o, u_row, rb);
    else
        std::memset(S->ready_U.data() + o, 0, rb);
}

// Harvest finished slots, then fill free slots from the queue.
int progress(als_server *S) {
    for (auto &sl : S->slots) {
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return ALS_E_HIP;
        const size_t u_bytes = al((size_t)sl.rows * S->ld * S->elt);
        const int32_t *st = (const int32_t *)(sl.h_out + u_bytes);
        for (int64_t k = 0; k < sl.rows; ++k)
            finish_request(S, sl.ids[k], st[k], sl.h_out + (size_t)k * S->ld * S->elt);
        S->inflight -= sl.rows;
        sl.busy = false;
    }
    for (auto &sl : S->slots) {
        if (sl.busy || S->queue.empty()) continue;
        std::vector<Req> batch;
        int64_t ratings = 0, chunks = 0, split = 0;
        while (!S->queue.empty() && (int64_t)batch.size() < S->cap_rows) {
            Req &r = S->queue.front();
            if (r.n > S->cap_ratings) {  // can never fit a slot: answer, do not drop
                finish_request(S, r.id, ALS_E_BUDGET, nullptr);
                S->queue.pop_front();
                continue;
            }
            if (r.store >= 0) {
                r.items = (const int32_t *)(S->arena.data() + r.store);
                r.vals = (const float *)(S->arena.data() + r.store + r.n * 4);
            }
            bool ids_ok = true;  // every item id must index a row of M
            for (int64_t k = 0; k < r.n; ++k)
                if ((uint32_t)r.items[k] >= (uint64_t)S->n_items) {
                    ids_ok = false;
                    break;
                }
            if (!ids_ok) {
                finish_request(S, r.id, ALS_E_INVAL, nullptr);
                S->queue.pop_front();
                continue;
            }
            const int64_t sp = S->cfg.split;
            const int64_t nck = (sp > 0 && r.n > sp) ? (r.n + sp - 1) / sp : 1;
            if (ratings + r.n > S->cap_ratings || chunks + nck > S->cap_chunks ||
                split + (nck > 1 ? nck : 0) > S->cap_split)
                break;
            ratings += r.n;
            chunks += nck;
            split += nck > 1 ? nck : 0;
            batch.push_back(r);
            S->queue.pop_front();
        }
        if (batch.empty()) continue;
        const int rc = launch_batch(S, sl, batch);
        if (rc != ALS_OK) return rc;
    }
    return ALS_OK;
}

int64_t drain_ready(als_server *S, int64_t max_done, int64_t *ids, int32_t *status, char *U) {
    const size_t rb = (size_t)S->n_f * S->elt;
    int64_t k = 0;
    while (k < max_done && S->ready_head < (int64_t)S->ready_ids.size()) {
        const int64_t h = S->ready_head++;
        if (ids) ids[k] = S->ready_ids[h];
        if (status) status[k] = S->ready_status[h];
        if (U) std::memcpy(U + k * rb, S->ready_U.data() + h * rb, rb);
        ++k;
    }
    if (S->ready_head == (int64_t)S->ready_ids.size()) {
        S->ready_ids.clear();
        S->ready_status.clear();
        S->ready_U.clear();
        S->ready_head = 0;
    }
    return k;
}

void free_slots(als_server *S) {
    for (auto &sl : S->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.h_in) (void)hipHostFree(sl.h_in);
        if (sl.h_out) (void)hipHostFree(sl.h_out);
        if (sl.d_in) (void)hipFree(sl.d_in);
        if (sl.d_out) (void)hipFree(sl.d_out);
        if (sl.d_partial) (void)hipFree(sl.d_partial);
    }
    S->slots.clear();
    if (S->ybits) (void)hipFree(S->ybits);
    S->ybits = nullptr;
}

}  // namespace

extern "C" {

int als_server_create(als_ctx *ctx, const void *M, int64_t n_items, int n_f, int ld, double lambda,
                      als_dtype dt, const als_server_config *cfg, als_server **out) {
    if (!out) return ALS_E_INVAL;
    *out = nullptr;
    if (!ctx || !M || !cfg || n_items < 1 || n_f < 1 || ld < n_f || !(lambda >= 0.0) ||
        cfg->max_inflight < 1 || cfg->max_batch < 1 || cfg->split < 0 || cfg->hbm_budget_bytes <= 0)
        return ALS_E_INVAL;
    if (!(dt == ALS_F32 && n_f <= 143) && !(dt == ALS_F64 && n_f <= 95)) return ALS_E_INVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return ALS_E_HIP;
    als_server *S = new (std::nothrow) als_server();
    if (!S) return ALS_E_NOMEM;
    S->ctx = ctx;
    S->M = M;
    S->n_items = n_items;
    S->n_f = n_f;
    S->ld = ld;
    S->lambda = lambda;
    S->dt = dt;
    S->cfg = *cfg;
    S->elt = dt == ALS_F64 ? 8 : 4;
    S->partial_bytes = sweep_partial_bytes(n_f, dt);
    // per-slot capacities from the budget: rows first, the rest to ratings
    const size_t per_slot = (size_t)cfg->hbm_budget_bytes / (size_t)cfg->max_inflight;
    S->cap_rows = cfg->max_batch;
    const size_t row_bytes = 8 + (size_t)ld * S->elt + 4 + 4 * 4 + 8 + 4 * 3;
    const size_t fixed = (size_t)S->cap_rows * row_bytes + 32 * 256;
    if (per_slot <= fixed + 4096) {
        delete S;
        return ALS_E_BUDGET;
    }
    const size_t sp = cfg->split;
    // bytes per rating: id + value (+ worst-case split-K share: a chunk slot,
    // its plan entries and its partial Gram per `split` ratings)
    const double per_rating = 8.0 + (sp > 0 ? (S->partial_bytes + 4.0 * 4 + 8.0) / (double)sp : 0.0);
    S->cap_ratings = (int64_t)((double)(per_slot - fixed) / per_rating);
    S->cap_ratings = std::min<int64_t>(S->cap_ratings, INT32_MAX / 2);
    S->cap_split = sp > 0 ? S->cap_ratings / (int64_t)sp + S->cap_rows : 0;
    S->cap_chunks = S->cap_rows + S->cap_split;
    S->slots.resize(cfg->max_inflight);
    int rc = ALS_OK;
    if (dt == ALS_F32) {
        if (hipMalloc((void **)&S->ybits, kAbsMaxWords * sizeof(unsigned)) != hipSuccess) {
            delete S;
            return ALS_E_NOMEM;
        }
        rc = launch_abs_max_bits((const float *)M, n_items, n_f, ld, S->ybits, nullptr);
        if (rc == ALS_OK && hipStreamSynchronize(nullptr) != hipSuccess) rc = ALS_E_HIP;
        if (rc != ALS_OK) {
            (void)hipFree(S->ybits);
            delete S;
            return rc;
        }
    }
    for (auto &sl : S->slots) {
        sl.in_bytes = in_bytes_for(S->cap_rows, S->cap_ratings, S->cap_chunks, S->cap_split);
        sl.out_bytes = al((size_t)S->cap_rows * ld * S->elt) + al((size_t)S->cap_rows * 4);
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
            rc = ALS_E_HIP;
            break;
        }
        if (hipHostMalloc((void **)&sl.h_in, sl.in_bytes, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&sl.h_out, sl.out_bytes, hipHostMallocDefault) != hipSuccess ||
            hipMalloc((void **)&sl.d_in, sl.in_bytes) != hipSuccess ||
            hipMalloc((void **)&sl.d_out, sl.out_bytes) != hipSuccess ||
            hipMalloc(&sl.d_partial, std::max<size_t>(S->cap_split, 1) * S->partial_bytes) != hipSuccess) {
            rc = ALS_E_NOMEM;
            break;
        }
    }
    if (rc != ALS_OK) {
        free_slots(S);
        delete S;
        return rc;
    }
    *out = S;
    return ALS_OK;
}

void als_server_destroy(als_server *S) {
    if (!S) return;
    (void)hipSetDevice(S->ctx->device);
    free_slots(S);
    delete S;
}

int als_server_submit(als_server *S, int64_t n, const int64_t *ids, const int64_t *indptr,
                      const int32_t *items, const float *vals) {
    if (!S || n < 0 || (n > 0 && (!ids || !indptr))) return ALS_E_INVAL;
    if (n == 0) return ALS_OK;
    const int64_t tot = indptr[n] - indptr[0];
    if (tot < 0 || (tot > 0 && (!items || !vals))) return ALS_E_INVAL;
    for (int64_t q = 0; q < n; ++q)
        if (indptr[q + 1] < indptr[q]) return ALS_E_INVAL;
    // copy into the arena as [items | values] per request; launch_batch
    // resolves the offsets, so the arena may grow and move freely.  It is
    // reset whenever nothing queued refers to it (in-flight batches were
    // already copied to their staging buffers).
    if (S->queue.empty()) {
        S->arena.clear();
        S->arena_live = 0;
    }
    for (int64_t q = 0; q < n; ++q) {
        const int64_t len = indptr[q + 1] - indptr[q];
        Req r;
        r.id = ids[q];
        r.n = len;
        r.items = nullptr;
        r.vals = nullptr;
        r.store = (int64_t)S->arena.size();
        S->arena.resize(S->arena.size() + (size_t)len * 8);
        if (len) {
            std::memcpy(S->arena.data() + r.store, items + indptr[q], (size_t)len * 4);
            std::memcpy(S->arena.data() + r.store + len * 4, vals + indptr[q], (size_t)len * 4);
        }
        S->queue.push_back(r);
    }
    S->arena_live += tot;
    return ALS_OK;
}

int als_server_poll(als_server *S, int64_t max_done, int64_t *done_ids, int32_t *done_status,
                    void *done_U, int64_t *n_done) {
    if (!S || max_done < 0 || !n_done) return ALS_E_INVAL;
    if (hipSetDevice(S->ctx->device) != hipSuccess) return ALS_E_HIP;
    const int rc = progress(S);
    *n_done = drain_ready(S, max_done, done_ids, done_status, (char *)done_U);
    return rc;
}

int64_t als_server_pending(const als_server *S) {
    return S ? (int64_t)S->queue.size() + S->inflight : 0;
}

int als_server_replay(als_server *S, int64_t n, const int64_t *arrival_ns, const int32_t *pool_row,
                      int64_t n_pool, const int64_t *pool_indptr, const int32_t *pool_items,
                      const float *pool_vals, int64_t *completion_ns, int32_t *status, void *U_out) {
    if (!S || n < 0 || n_pool < 0 ||
        (n > 0 && (!arrival_ns || !pool_row || !pool_indptr || !completion_ns)))
        return ALS_E_INVAL;
    if (!S->queue.empty() || S->inflight) return ALS_E_INVAL;  // replay needs an idle server
    for (int64_t q = 0; q < n; ++q)
        if (pool_row[q] < 0 || pool_row[q] >= n_pool || (q && arrival_ns[q] < arrival_ns[q - 1]))
            return ALS_E_INVAL;
    if (hipSetDevice(S->ctx->device) != hipSuccess) return ALS_E_HIP;
    const size_t rb = (size_t)S->n_f * S->elt;
    const int64_t t0 = now_ns();
    int64_t next = 0, done = 0;
    while (done < n) {
        const int64_t t = now_ns() - t0;
        while (next < n && arrival_ns[next] <= t) {
            const int64_t pr = pool_row[next];
            Req r;
            r.id = next;
            r.n = pool_indptr[pr + 1] - pool_indptr[pr];
            r.items = pool_items + pool_indptr[pr];
            r.vals = pool_vals + pool_indptr[pr];
            r.store = -1;
            S->queue.push_back(r);
            ++next;
        }
        int rc = progress(S);
        if (rc != ALS_OK) return rc;
        const int64_t tf = now_ns() - t0;
        while (S->ready_head < (int64_t)S->ready_ids.size()) {
            const int64_t h = S->ready_head++;
            const int64_t q = S->ready_ids[h];
            completion_ns[q] = tf;
            if (status) status[q] = S->ready_status[h];
            if (U_out) std::memcpy((char *)U_out + q * rb, S->ready_U.data() + h * rb, rb);
            ++done;
        }
        S->ready_ids.clear();
        S->ready_status.clear();
        S->ready_U.clear();
        S->ready_head = 0;
    }
    return ALS_OK;
}

}  // extern "C"
