// Serving loop with continuous batching (see lt_server_* in lt.h).
//
// Each request becomes ordinary annotated launches on the shared context, so
// admitted requests overlap on the device exactly as independent launches
// do, and every request's result is the one it would get alone.  Admission
// is by device footprint; inputs are cached host-backed arrays whose chunks
// stay in HBM across requests until the memory manager spills them.
#include <algorithm>
#include <chrono>
#include <cstddef>
#include <cstring>
#include <deque>
#include <map>
#include <tuple>

#include "lt_internal.h"

namespace lt {
namespace {

struct SDataset {
    lt_array *a0 = nullptr, *a1 = nullptr;
    int refs = 0;
};

struct SReq {
    uint64_t id = 0;
    lt_request r;
    double t_submit = 0, t_admit = 0;
    Fence computed;          // the output's device copy is final after this
    Fence done;              // ... and back in host memory after this
    bool flushed = false;
    lt_array *out = nullptr;
    int64_t footprint = 0;
    bool hit = false;
    std::vector<lt_array *> owned;
    SDataset *ds = nullptr;
    std::tuple<int, int, int64_t> key;
    int bypassed = 0;        // times a later request was admitted first
};

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int64_t footprint_of(const lt_request &r) {
    const int64_t n = r.size;
    switch (r.kind) {
        case LT_REQ_JACOBI: return n * n * 4 * (r.sweeps >= 3 ? 4 : r.sweeps + 1);
        case LT_REQ_KMEANS: return n * (r.d * 4 + 4) + r.K * r.d * 4;
        case LT_REQ_GEMM: return 3 * n * n * 4;
    }
    return 0;
}

}  // namespace
}  // namespace lt

using namespace lt;

struct lt_server {
    lt_context *ctx = nullptr;
    lt_server_config cfg;
    uint64_t next_id = 1;
    std::deque<SReq *> queue;
    std::vector<SReq *> active;
    std::vector<lt_completion> finished;
    std::map<std::tuple<int, int, int64_t>, SDataset *> cache;
    int64_t admitted = 0;
    lt_kernel *kj = nullptr, *kk = nullptr, *kg = nullptr;
};

namespace {

lt_dist rows_dist(int64_t rows) {
    lt_dist d;
    memset(&d, 0, sizeof d);
    d.kind = LT_DIST_BLOCK;
    d.chunk[0] = rows;
    return d;
}

lt_status make_host(lt_context *ctx, lt_dtype dt, int nd, int64_t r, int64_t c, const lt_dist &d, const void *p,
                    lt_array **out) {
    int64_t shape[2] = {r, c};
    return lt_array_create_host(ctx, dt, nd, shape, &d, const_cast<void *>(p), out);
}

lt_arg iarg(int64_t v) {
    lt_arg a;
    memset(&a, 0, sizeof a);
    a.kind = LT_ARG_INT;
    a.i = v;
    return a;
}

lt_arg aarg(lt_array *x) {
    lt_arg a;
    memset(&a, 0, sizeof a);
    a.kind = LT_ARG_ARRAY;
    a.array = x;
    return a;
}

lt_status admit(lt_server *s, SReq *q) {
    lt_context *ctx = s->ctx;
    const lt_request &r = q->r;
    const int64_t n = r.size;
    const int64_t cr = s->cfg.chunk_rows > 0 ? s->cfg.chunk_rows : (r.kind == LT_REQ_KMEANS ? (1 << 20) : 512);
    const int64_t T = s->cfg.gemm_tile > 0 ? s->cfg.gemm_tile : 4096;
    q->t_admit = now_s();
    q->key = std::make_tuple(r.kind, r.dataset, n);
    SDataset *ds = nullptr;
    auto it = s->cache.find(q->key);
    lt_status st = LT_OK;
    if (s->cfg.keep_resident && it != s->cache.end()) {
        ds = it->second;
        q->hit = true;
    } else {
        ds = new SDataset();
        if (r.kind == LT_REQ_JACOBI) {
            st = make_host(ctx, LT_F32, 2, n, n, rows_dist(cr), r.in0, &ds->a0);
        } else if (r.kind == LT_REQ_KMEANS) {
            st = make_host(ctx, LT_F32, 2, n, r.d, rows_dist(cr), r.in0, &ds->a0);
            if (!st) st = make_host(ctx, LT_F32, 2, r.K, r.d, rows_dist(0), r.in1, &ds->a1);
        } else {
            lt_dist cols;
            memset(&cols, 0, sizeof cols);
            cols.kind = LT_DIST_BLOCK;
            cols.chunk[1] = T;
            st = make_host(ctx, LT_F32, 2, n, n, rows_dist(T), r.in0, &ds->a0);
            if (!st) st = make_host(ctx, LT_F32, 2, n, n, cols, r.in1, &ds->a1);
        }
        if (st) {
            delete ds;
            return st;
        }
        if (s->cfg.keep_resident) s->cache[q->key] = ds;
    }
    ds->refs++;
    q->ds = ds;
    lt_array *out = nullptr;
    if (r.kind == LT_REQ_JACOBI) {
        st = make_host(ctx, LT_F32, 2, n, n, rows_dist(cr), r.out, &out);
        if (st) return st;
        q->owned.push_back(out);
        lt_array *w[2] = {nullptr, nullptr};
        int64_t shape[2] = {n, n};
        lt_dist d = rows_dist(cr);
        for (int i = 0; i < 2 && i < r.sweeps - 1; ++i) {
            st = lt_array_create(ctx, LT_F32, 2, shape, &d, &w[i]);
            if (st) return st;
            q->owned.push_back(w[i]);
        }
        lt_array *src = ds->a0;
        for (int sw = 0; sw < r.sweeps; ++sw) {
            lt_array *dst = (sw == r.sweeps - 1) ? out : w[sw & 1];
            int64_t grid[2] = {n, n}, block[2] = {1, 1}, sb[2] = {cr, 0};
            lt_arg a[4] = {iarg(n), iarg(n), aarg(dst), aarg(src)};
            st = lt_launch(ctx, s->kj, 2, grid, block, sb, nullptr, a, 4, nullptr);
            if (st) return st;
            src = dst;
        }
    } else if (r.kind == LT_REQ_KMEANS) {
        lt_dist d = rows_dist(cr);
        int64_t shape[1] = {n};
        st = lt_array_create_host(ctx, LT_I32, 1, shape, &d, r.out, &out);
        if (st) return st;
        q->owned.push_back(out);
        int64_t grid[1] = {n}, block[1] = {1}, sb[1] = {cr};
        lt_arg a[6] = {iarg(n), iarg(r.d), iarg(r.K), aarg(out), aarg(ds->a0), aarg(ds->a1)};
        st = lt_launch(ctx, s->kk, 1, grid, block, sb, nullptr, a, 6, nullptr);
        if (st) return st;
    } else {
        lt_dist tiles;
        memset(&tiles, 0, sizeof tiles);
        tiles.kind = LT_DIST_BLOCK;
        tiles.chunk[0] = T;
        tiles.chunk[1] = T;
        st = make_host(ctx, LT_F32, 2, n, n, tiles, r.out, &out);
        if (st) return st;
        q->owned.push_back(out);
        int64_t grid[2] = {n, n}, block[2] = {1, 1}, sb[2] = {T, T};
        lt_arg a[6] = {iarg(n), iarg(n), iarg(n), aarg(out), aarg(ds->a0), aarg(ds->a1)};
        st = lt_launch(ctx, s->kg, 2, grid, block, sb, nullptr, a, 6, nullptr);
        if (st) return st;
    }
    // the write-back is issued once the result is computed (progress): the
    // D2H queue then never holds a copy that waits on unfinished work ahead
    // of copies that could run
    q->out = out;
    return array_ready_fence(ctx, out, &q->computed);
}

// Issues the output write-back of requests whose compute has finished.
lt_status flush_ready(lt_server *s) {
    for (SReq *q : s->active) {
        if (q->flushed || !fence_done(s->ctx, q->computed)) continue;
        lt_status st = array_flush_async(s->ctx, q->out, &q->done);
        if (st) return st;
        q->flushed = true;
    }
    return LT_OK;
}

void release(lt_server *s, SReq *q) {
    for (lt_array *a : q->owned) (void)lt_array_destroy(s->ctx, a);
    q->owned.clear();
    if (q->ds) {
        q->ds->refs--;
        if (!s->cfg.keep_resident) {
            if (q->ds->a0) (void)lt_array_destroy(s->ctx, q->ds->a0);
            if (q->ds->a1) (void)lt_array_destroy(s->ctx, q->ds->a1);
            delete q->ds;
        }
        q->ds = nullptr;
    }
}

void finish(lt_server *s, SReq *q, lt_status st) {
    lt_completion c;
    memset(&c, 0, sizeof c);
    c.id = q->id;
    c.status = st;
    c.kind = q->r.kind;
    c.t_submit = q->t_submit;
    c.t_admit = q->t_admit;
    c.t_done = now_s();
    c.footprint = (uint64_t)q->footprint;
    c.cache_hit = q->hit;
    s->finished.push_back(c);
    release(s, q);
    delete q;
}

// Completes finished requests, then admits queued ones in arrival order while
// a slot is free and the footprint fits.
void progress(lt_server *s) {
    lt_status fs = flush_ready(s);
    if (fs != LT_OK && s->ctx->sticky == LT_OK) {
        s->ctx->sticky = fs;
        s->ctx->sticky_msg = s->ctx->err;
    }
    for (size_t i = 0; i < s->active.size();) {
        SReq *q = s->active[i];
        if (q->flushed && fence_done(s->ctx, q->done)) {
            s->admitted -= q->footprint;
            s->active.erase(s->active.begin() + i);
            lt_status st = s->ctx->sticky;
            finish(s, q, st);
        } else {
            ++i;
        }
    }
    const int64_t cap = s->cfg.admit_bytes > 0 ? (int64_t)s->cfg.admit_bytes
                                               : (int64_t)s->ctx->cfg.device_budget_bytes;
    auto fits = [&](const SReq *q) { return s->active.empty() || s->admitted + q->footprint <= cap; };
    const int look = s->cfg.lookahead > 0 ? s->cfg.lookahead : 0;
    const int max_bypass = s->cfg.max_bypass > 0 ? s->cfg.max_bypass : 4 * look;
    while (!s->queue.empty() && (int)s->active.size() < s->cfg.max_active) {
        size_t pick = 0;
        if (look > 0 && s->queue.front()->bypassed < max_bypass) {
            // the oldest queued request on a cached dataset, else the oldest
            // that fits, among the first `look`
            const size_t w = std::min(s->queue.size(), (size_t)look);
            size_t first_fit = w;
            pick = w;
            for (size_t i = 0; i < w; ++i) {
                const SReq *q = s->queue[i];
                if (!fits(q)) continue;
                if (first_fit == w) first_fit = i;
                if (s->cache.count(std::make_tuple(q->r.kind, q->r.dataset, q->r.size))) {
                    pick = i;
                    break;
                }
            }
            if (pick == w) pick = first_fit;
            if (pick == w) break;
        } else if (!fits(s->queue.front())) {
            break;
        }
        SReq *q = s->queue[pick];
        for (size_t i = 0; i < pick; ++i) s->queue[i]->bypassed++;
        s->queue.erase(s->queue.begin() + (std::ptrdiff_t)pick);
        lt_status st = admit(s, q);
        if (st) {
            finish(s, q, st);
            continue;
        }
        s->admitted += q->footprint;
        s->active.push_back(q);
    }
}

int32_t take(lt_server *s, lt_completion *out, int32_t cap) {
    int32_t n = 0;
    while (n < cap && !s->finished.empty()) {
        out[n++] = s->finished.front();
        s->finished.erase(s->finished.begin());
    }
    return n;
}

}  // namespace

extern "C" {

double lt_now(void) { return now_s(); }

lt_status lt_server_create(lt_context *ctx, const lt_server_config *cfg, lt_server **out) {
    if (!ctx || !out) return LT_ERR_INVALID;
    auto *s = new lt_server();
    s->ctx = ctx;
    if (cfg) s->cfg = *cfg;
    else memset(&s->cfg, 0, sizeof s->cfg);
    if (s->cfg.max_active < 1) s->cfg.max_active = 1;
    lt_status st = lt_kernel_get(ctx, "jacobi2d_f32", &s->kj);
    if (!st) st = lt_kernel_get(ctx, "kmeans_assign_f32", &s->kk);
    if (!st) st = lt_kernel_get(ctx, "gemm_f32", &s->kg);
    if (st) {
        delete s;
        return st;
    }
    *out = s;
    return LT_OK;
}

lt_status lt_server_submit(lt_server *s, const lt_request *req, uint64_t *id) {
    if (!s || !req) return LT_ERR_INVALID;
    const lt_request &r = *req;
    if (r.kind < 0 || r.kind > 2 || r.size <= 0 || !r.in0 || !r.out || (r.kind != LT_REQ_JACOBI && !r.in1))
        return set_err(s->ctx, LT_ERR_INVALID, "invalid request");
    if (r.kind == LT_REQ_JACOBI && r.sweeps < 1) return set_err(s->ctx, LT_ERR_INVALID, "sweeps must be >= 1");
    if (r.kind == LT_REQ_KMEANS && (r.d < 1 || r.d > 32 || r.K < 1 || r.K > 256))
        return set_err(s->ctx, LT_ERR_INVALID, "k-means needs 1 <= d <= 32 and 1 <= K <= 256");
    SReq *q = new SReq();
    q->id = s->next_id++;
    q->r = r;
    q->t_submit = now_s();
    q->footprint = footprint_of(r);
    s->queue.push_back(q);
    if (id) *id = q->id;
    progress(s);
    return LT_OK;
}

lt_status lt_server_poll(lt_server *s, lt_completion *out, int32_t cap, int32_t *n) {
    if (!s || !n) return LT_ERR_INVALID;
    progress(s);
    *n = take(s, out, out ? cap : 0);
    return LT_OK;
}

lt_status lt_server_drain(lt_server *s, lt_completion *out, int32_t cap, int32_t *n) {
    if (!s || !n) return LT_ERR_INVALID;
    while (!s->queue.empty() || !s->active.empty()) {
        progress(s);
        if (s->active.empty()) continue;
        // block on the oldest active request: its compute, then its copy
        SReq *q = s->active.front();
        lt_status st = wait_fence(s->ctx, q->flushed ? q->done : q->computed);
        if (st) return st;
    }
    *n = take(s, out, out ? cap : 0);
    return LT_OK;
}

lt_status lt_server_destroy(lt_server *s) {
    if (!s) return LT_ERR_INVALID;
    int32_t n;
    lt_status st = lt_server_drain(s, nullptr, 0, &n);
    for (auto &kv : s->cache) {
        if (kv.second->a0) (void)lt_array_destroy(s->ctx, kv.second->a0);
        if (kv.second->a1) (void)lt_array_destroy(s->ctx, kv.second->a1);
        delete kv.second;
    }
    delete s;
    return st;
}

}  // extern "C"
