// C ABI of the runtime: contexts, arrays, kernels, launch/sync, introspection.
#include <unistd.h>

#include <algorithm>
#include <cstdio>
#include <cstring>

#include "lt_internal.h"

namespace lt {

// ----------------------------------------------------------- built-in table
static const KernelDef kBuiltins[] = {
    {"touch_i32", "global i => readwrite y[i]", 2,
     {{"n", P_INT, LT_I32, 0}, {"y", P_ARRAY, LT_I32, 1}}, 1, launch_touch_i32, KMAXG, DK_TOUCH},
    {"stencil1d_f32", "global i => read x[i-1:i+1], write y[i]", 3,
     {{"n", P_INT, LT_F32, 0}, {"y", P_ARRAY, LT_F32, 1}, {"x", P_ARRAY, LT_F32, 1}}, 1,
     launch_stencil1d_f32, KMAXG, DK_STENCIL1D},
    {"jacobi2d_f32", "global [r, c] => read x[r-1:r+1, c-1:c+1], write y[r, c]", 4,
     {{"n", P_INT, LT_F32, 0}, {"m", P_INT, LT_F32, 0}, {"y", P_ARRAY, LT_F32, 2}, {"x", P_ARRAY, LT_F32, 2}},
     2, launch_jacobi2d_f32, KMAXG, DK_JACOBI2D},
    {"gemm_f32", "global [i, j] => read A[i, :], read B[:, j], write C[i, j]", 6,
     {{"M", P_INT, LT_F32, 0},
      {"N", P_INT, LT_F32, 0},
      {"K", P_INT, LT_F32, 0},
      {"C", P_ARRAY, LT_F32, 2},
      {"A", P_ARRAY, LT_F32, 2},
      {"B", P_ARRAY, LT_F32, 2}},
     2, launch_gemm_f32, 8, -1},
    {"hist256_i32", "global i => read v[i], reduce(+) h[:]", 3,
     {{"n", P_INT, LT_I32, 0}, {"h", P_ARRAY, LT_I32, 1}, {"v", P_ARRAY, LT_I32, 1}}, 1,
     launch_hist256_i32, 1, DK_HIST256, hist_slots, true},
    {"kmeans_assign_f32", "global i => read X[i, :], read Cen[:, :], write lab[i]", 6,
     {{"N", P_INT, LT_F32, 0},
      {"d", P_INT, LT_F32, 0},
      {"K", P_INT, LT_F32, 0},
      {"lab", P_ARRAY, LT_I32, 1},
      {"X", P_ARRAY, LT_F32, 2},
      {"Cen", P_ARRAY, LT_F32, 2}},
     1, launch_kmeans_assign_f32, KMAXG, -1},
    {"rowreduce_f32", "global [i, j] => read A[i, j], reduce(+) out[i]", 4,
     {{"n", P_INT, LT_F32, 0}, {"m", P_INT, LT_F32, 0}, {"out", P_ARRAY, LT_F32, 1}, {"A", P_ARRAY, LT_F32, 2}},
     2, launch_rowreduce_f32, 1, -1},
    {"kmeans_update_f32", "global i => read X[i, :], read lab[i], reduce(+) sums[:, :], reduce(+) counts[:]", 7,
     {{"N", P_INT, LT_F32, 0},
      {"d", P_INT, LT_F32, 0},
      {"K", P_INT, LT_F32, 0},
      {"sums", P_ARRAY, LT_F64, 2},
      {"counts", P_ARRAY, LT_I32, 1},
      {"X", P_ARRAY, LT_F32, 2},
      {"lab", P_ARRAY, LT_I32, 1}},
     1, launch_kmeans_update_f32, 1, -1, kmeans_update_slots, true},
    {"kmeans_centres_f32", "global [k, j] => read sums[k, j], read counts[k], readwrite Cen[k, j]", 5,
     {{"K", P_INT, LT_F32, 0},
      {"d", P_INT, LT_F32, 0},
      {"Cen", P_ARRAY, LT_F32, 2},
      {"sums", P_ARRAY, LT_F64, 2},
      {"counts", P_ARRAY, LT_I32, 1}},
     2, launch_kmeans_centres_f32, KMAXG, -1},
};

const KernelDef *find_builtin(const char *name) {
    if (!name) return nullptr;
    for (const KernelDef &d : kBuiltins)
        if (!strcmp(d.name, name)) return &d;
    return nullptr;
}

static int dtype_size(lt_dtype d) {
    switch (d) {
        case LT_F32:
        case LT_I32: return 4;
        case LT_F64:
        case LT_I64: return 8;
        case LT_U8: return 1;
    }
    return 0;
}

// A handle is live while it belongs to this context and was not destroyed.
// (Handles of destroyed arrays stay valid memory until the next lt_sync.)
static bool live(Ctx *ctx, Array *arr) {
    return arr && arr->magic == LT_ARRAY_MAGIC && arr->owner == ctx && !arr->dead;
}

// ------------------------------------------------------------------- sync
lt_status sync_all(Ctx *ctx) {
    lt_status st = flush_all(ctx);
    // write dirty chunks of host-backed arrays back to their home buffers
    for (Array *arr : ctx->arrays) {
        if (arr->dead || !arr->host_backed) continue;
        for (Chunk *c : arr->chunks) {
            if (st) break;
            if (c->dev_off < 0 || !c->dev_valid || c->host_valid || !c->defined) continue;
            uint64_t p = 0;
            st = write_back(ctx, c, &p);
            if (!st) c->last_access.add(ctx->d2h, p);
        }
    }
    if (!ctx->dry) {
        lt_status ps = prof_close_steps(ctx);
        if (ps && !st) st = ps;
        for (int s = 0; s < ctx->nstreams; ++s) {
            hipError_t r = hipStreamSynchronize(ctx->streams[s].h);
            if (r != hipSuccess && !st) st = hip_fail(ctx, r, "hipStreamSynchronize");
        }
        prof_collect(ctx);
        fold_drain_status(ctx);
        // spill file transfers ran on the streams just drained
        lt_status ds = disk_status(ctx);
        if (ds && !st) st = ds;
        for (int32_t *gs : ctx->graph_status)
            if (*gs && ctx->sticky == LT_OK) {
                ctx->sticky = LT_ERR_TIMEOUT;
                ctx->sticky_msg = "a dependency wait inside a graph's drain exceeded its poll limit";
            }
    }
    for (size_t i = 0; i < ctx->staging_used.size(); ++i) {
        ctx->staging_free.push_back(ctx->staging_used[i]);
        ctx->staging_size_free.push_back(ctx->staging_size_used[i]);
    }
    ctx->staging_used.clear();
    ctx->staging_size_used.clear();
    for (int s = 0; s < ctx->nstreams; ++s) {
        Stream &S = ctx->streams[s];
        S.done = S.seq;
        for (auto &m : S.marks) ctx->event_pool.push_back(m.ev);
        S.marks.clear();
    }
    // every task has completed: forget the DAG
    ctx->tasks.reset(ctx->next_task_id);
    ctx->launches.reset(ctx->next_launch_id);
    ctx->staged.clear();
    ctx->staged_bytes = 0;
    for (Array *arr : ctx->arrays)
        for (Chunk *c : arr->chunks) {
            c->last_writer = 0;
            c->readers.clear();
            c->reducers.clear();
            c->reduce_op = -1;
        }
    // release destroyed arrays
    std::vector<Array *> keep;
    for (Array *arr : ctx->arrays) {
        if (!arr->dead) {
            keep.push_back(arr);
            continue;
        }
        for (Chunk *c : arr->chunks) {
            free_spill(ctx, c);
            delete c;
        }
        arr->magic = 0;
        delete arr;
    }
    ctx->arrays.swap(keep);
    if (st) return st;
    if (ctx->sticky != LT_OK) {
        lt_status s = ctx->sticky;
        ctx->err = ctx->sticky_msg;
        ctx->sticky = LT_OK;
        ctx->sticky_msg.clear();
        return s;
    }
    return LT_OK;
}

// The point after which every chunk of the array holds its final data on
// the device (pending grouped work is issued first).
lt_status array_ready_fence(Ctx *ctx, Array *arr, Fence *out) {
    lt_status st = flush_all(ctx);
    if (st) return st;
    *out = Fence();
    for (Chunk *c : arr->chunks) out->merge(c->data_ready);
    return LT_OK;
}

// Issues the write-back of a host-backed array's dirty chunks to its home
// buffer without waiting; *out = the point after which the home buffer holds
// the array's contents.
lt_status array_flush_async(Ctx *ctx, Array *arr, Fence *out) {
    lt_status st = flush_all(ctx);
    if (st) return st;
    *out = Fence();
    if (!arr->host_backed) return set_err(ctx, LT_ERR_INVALID, "array is not host-backed");
    for (Chunk *c : arr->chunks) {
        if (c->dev_off >= 0 && c->dev_valid && !c->host_valid && c->defined) {
            uint64_t p = 0;
            st = write_back(ctx, c, &p);
            if (st) return st;
            c->last_access.add(ctx->d2h, p);
        }
        out->merge(c->host_ready);
    }
    return LT_OK;
}

void ctx_release_all(Ctx *ctx) {
    for (Array *arr : ctx->arrays) arr->dead = true;
    (void)sync_all(ctx);
    drain_pin_pool(ctx);
    if (!ctx->dry) {
        bounce_release(ctx);
        for (int s = 0; s < ctx->nstreams; ++s)
            if (ctx->streams[s].h) (void)hipStreamDestroy(ctx->streams[s].h);
        for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
        for (hipEvent_t e : ctx->prof_pool) (void)hipEventDestroy(e);
        if (ctx->prof_base) (void)hipEventDestroy(ctx->prof_base);
        if (ctx->arena_owned && ctx->arena_base) (void)hipFree(ctx->arena_base);
        for (void *p : ctx->host_allocs) (void)hipHostFree(p);
        for (void *p : ctx->staging_free) (void)hipHostFree(p);
        if (ctx->status_host) (void)hipHostFree(ctx->status_host);
        if (ctx->spill_fd >= 0) (void)close(ctx->spill_fd);
        ctx->spill_fd = -1;
    } else {
        for (void *p : ctx->staging_free) free(p);
    }
    ctx->staging_free.clear();
    ctx->status_host = nullptr;
    ctx->event_pool.clear();
    ctx->host_allocs.clear();
}

// --------------------------------------------------------------- array I/O
// After a whole-array write or fill every stored copy, halo replicas
// included, holds the new contents.
static void all_copies_current(Array *arr) {
    for (Chunk *c : arr->chunks) {
        c->version++;
        if (c->host_valid) c->host_version = c->version;
    }
    for (Chunk *c : arr->chunks)
        for (HaloSrc &h : c->halo) {
            h.ver = h.k->version;
            h.valid = true;
        }
}

// Writes from `src` (row-major whole array) into every chunk.  Device copies
// are overwritten after all earlier uses; chunks of a host-backed array that
// are not on the device are written in their home buffer.
lt_status array_write(Ctx *ctx, Array *arr, const void *src, bool device_src) {
    lt_status st = flush_all(ctx);
    if (st) return st;
    TaskRec rec;
    rec.id = ctx->next_task_id++;
    rec.kind = LT_TASK_IO;
    rec.stream = ctx->h2d;
    const int nd = arr->ndim;
    bool host_sync = false;
    for (Chunk *c : arr->chunks) {
        int64_t off = 0, ext[MAXD];
        for (int a = 0; a < MAXD; ++a) {
            off += (a < nd ? c->box.lo[a] : 0) * arr->strides[a];
            ext[a] = c->box.hi[a] - c->box.lo[a];
        }
        const char *sp = (const char *)src + off * arr->esz;
        for (uint64_t d : c->readers) rec.deps.push_back(d);
        if (c->last_writer) rec.deps.push_back(c->last_writer);
        if (c->dev_off >= 0 || !arr->host_backed || device_src) {
            Fence mem;
            if (c->dev_off < 0) {
                c->pin++;
                st = alloc_chunk(ctx, c, &mem);
                c->pin--;
                if (st) return st;
                c->last_access.merge(mem);
            }
            st = stream_wait(ctx, ctx->h2d, c->last_access);
            if (st) return st;
            st = copy_box(ctx, ctx->h2d, dev_ptr(ctx, c), c->dev_stride, sp, arr->strides, ext, nd, arr->esz,
                          device_src ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
            if (st) return st;
            uint64_t p = bump(ctx, ctx->h2d);
            trace_op(ctx, device_src ? 3 : 1, ctx->h2d, rec.id, c->id, c->bytes, c->dev_off);
            c->data_ready = Fence();
            c->data_ready.add(ctx->h2d, p);
            c->last_access.add(ctx->h2d, p);
            c->dev_valid = true;
            c->host_valid = false;
            c->defined = true;
        } else {
            // host-backed chunk living only in its home buffer
            if (!host_sync && !ctx->dry) {
                hipError_t r = hipStreamSynchronize(ctx->streams[ctx->d2h].h);
                if (r != hipSuccess) return hip_fail(ctx, r, "hipStreamSynchronize");
                r = hipStreamSynchronize(ctx->streams[ctx->h2d].h);
                if (r != hipSuccess) return hip_fail(ctx, r, "hipStreamSynchronize");
                host_sync = true;
            }
            st = ensure_host_copy(ctx, c);
            if (st) return st;
            // a recycled spill buffer may still be read by a spill file write
            st = wait_fence(ctx, c->host_ready);
            if (st) return st;
            if (c->host_ptr != sp) {
                st = copy_box(ctx, ctx->h2d, c->host_ptr, c->host_stride, sp, arr->strides, ext, nd, arr->esz,
                              hipMemcpyHostToHost);
                if (st) return st;
            }
            c->host_valid = true;
            c->defined = true;
        }
        c->last_writer = rec.id;
        c->readers.clear();
        c->reducers.clear();
        c->reduce_op = -1;
    }
    rec.seq = ctx->streams[ctx->h2d].seq;
    ctx->tasks.at(rec.id) = std::move(rec);
    all_copies_current(arr);
    if (!ctx->dry) {
        hipError_t r = hipStreamSynchronize(ctx->streams[ctx->h2d].h);
        if (r != hipSuccess) return hip_fail(ctx, r, "hipStreamSynchronize");
    }
    return LT_OK;
}

lt_status array_read(Ctx *ctx, Array *arr, void *dst, bool device_dst) {
    if (ctx->dry) return set_err(ctx, LT_ERR_INVALID, "array contents are unavailable in a dry run");
    lt_status st = flush_all(ctx);
    if (st) return st;
    const int nd = arr->ndim;
    bool need_host = false;
    const int64_t zero[MAXD] = {0, 0, 0};
    for (Chunk *c : arr->chunks) {
        // each chunk contributes the elements it owns (its core)
        if (c->dev_off >= 0 && c->dev_valid) {
            st = stream_wait(ctx, ctx->d2h, c->data_ready);
            if (st) return st;
            st = copy_sub(ctx, ctx->d2h, (char *)dst, zero, arr->strides, dev_ptr(ctx, c), c->box.lo, c->dev_stride,
                          c->core, nd, arr->esz, device_dst ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost);
            if (st) return st;
            uint64_t p = bump(ctx, ctx->d2h);
            c->last_access.add(ctx->d2h, p);
        } else if (c->host_valid && (c->host_ptr || c->disk_valid)) {
            need_host = true;
        }
    }
    hipError_t r = hipStreamSynchronize(ctx->streams[ctx->d2h].h);
    if (r != hipSuccess) return hip_fail(ctx, r, "hipStreamSynchronize");
    if (need_host) {
        for (Chunk *c : arr->chunks) {
            if ((c->dev_off >= 0 && c->dev_valid) || !c->host_valid) continue;
            st = host_resident(ctx, c);
            if (st) return st;
            if (!c->host_ptr) continue;
            int64_t off = 0;
            for (int a = 0; a < nd; ++a) off += c->box.lo[a] * arr->strides[a];
            if ((char *)dst + off * arr->esz == c->host_ptr) continue;  // the home buffer itself
            // a read back from the spill file runs on the H2D stream: a
            // device-bound copy waits for it on the stream, a host memcpy here
            st = device_dst ? stream_wait(ctx, ctx->d2h, c->host_ready) : wait_fence(ctx, c->host_ready);
            if (st) return st;
            // host -> host or host -> device through the copy helper on d2h
            st = copy_sub(ctx, ctx->d2h, (char *)dst, zero, arr->strides, c->host_ptr, c->box.lo, c->host_stride,
                          c->core, nd, arr->esz, device_dst ? hipMemcpyHostToDevice : hipMemcpyHostToHost);
            if (st) return st;
        }
        r = hipStreamSynchronize(ctx->streams[ctx->d2h].h);
        if (r != hipSuccess) return hip_fail(ctx, r, "hipStreamSynchronize");
        st = disk_status(ctx);
        if (st) return st;
    }
    if (ctx->sticky != LT_OK) {
        lt_status s = ctx->sticky;
        ctx->err = ctx->sticky_msg;
        ctx->sticky = LT_OK;
        return s;
    }
    return LT_OK;
}

lt_status array_fill(Ctx *ctx, Array *arr, const void *scalar) {
    lt_status st = flush_all(ctx);
    if (st) return st;
    TaskRec rec;
    rec.id = ctx->next_task_id++;
    rec.kind = LT_TASK_IO;
    rec.stream = 0;
    for (Chunk *c : arr->chunks) {
        if (c->dev_off < 0 && arr->host_backed && !ctx->dry) {
            // fill the home buffer on the host after pending copies
            hipError_t r = hipDeviceSynchronize();
            if (r != hipSuccess) return hip_fail(ctx, r, "hipDeviceSynchronize");
            st = ensure_host_copy(ctx, c);
            if (st) return st;
            st = wait_fence(ctx, c->host_ready);
            if (st) return st;
            std::vector<char> tmp((size_t)c->bytes);
            for (int64_t i = 0; i < c->elems; ++i) memcpy(tmp.data() + i * arr->esz, scalar, arr->esz);
            int64_t ext[MAXD], dense[MAXD];
            int64_t s = 1;
            for (int a = MAXD - 1; a >= 0; --a) {
                ext[a] = c->box.hi[a] - c->box.lo[a];
                dense[a] = s;
                s *= ext[a];
            }
            st = copy_box(ctx, ctx->d2h, c->host_ptr, c->host_stride, tmp.data(), dense, ext, arr->ndim, arr->esz,
                          hipMemcpyHostToHost);
            if (st) return st;
            r = hipStreamSynchronize(ctx->streams[ctx->d2h].h);
            if (r != hipSuccess) return hip_fail(ctx, r, "hipStreamSynchronize");
            c->host_valid = true;
            c->defined = true;
        } else {
            Fence mem;
            if (c->dev_off < 0) {
                c->pin++;
                st = alloc_chunk(ctx, c, &mem);
                c->pin--;
                if (st) return st;
                c->last_access.merge(mem);
            }
            st = stream_wait(ctx, 0, c->last_access);
            if (st) return st;
            trace_op(ctx, 4, 0, rec.id, c->id, c->bytes, c->dev_off);
            if (!ctx->dry) {
                hipError_t r = launch_fill(ctx->streams[0].h, dev_ptr(ctx, c), c->elems, arr->esz, scalar);
                if (r != hipSuccess) return hip_fail(ctx, r, "fill");
            }
            uint64_t p = bump(ctx, 0);
            c->data_ready = Fence();
            c->data_ready.add(0, p);
            c->last_access.add(0, p);
            c->dev_valid = true;
            c->host_valid = false;
            c->defined = true;
        }
        for (uint64_t d : c->readers) rec.deps.push_back(d);
        if (c->last_writer) rec.deps.push_back(c->last_writer);
        c->last_writer = rec.id;
        c->readers.clear();
        c->reducers.clear();
    }
    rec.seq = ctx->streams[0].seq;
    ctx->tasks.at(rec.id) = std::move(rec);
    all_copies_current(arr);
    return LT_OK;
}

lt_status array_destroy(Ctx *ctx, Array *arr) {
    // an open batch is issued first (its queued tasks pin their chunks); a
    // graph, or one being recorded, keeps its pins
    lt_status st = flush_all(ctx);
    if (st) return st;
    for (Chunk *c : arr->chunks)
        if (c->pin > 0) return set_err(ctx, LT_ERR_INVALID, "array is in use by a graph");
    arr->dead = true;
    for (Chunk *c : arr->chunks) {
        if (c->dev_off >= 0) {
            Fence f = c->last_access;
            ctx->arena.release(c->dev_off, f);
            trace_op(ctx, 7, -1, ~0ull, c->id, c->bytes, c->dev_off);
            c->dev_off = -1;
            c->dev_valid = false;
        }
    }
    ctx->stats.resident_bytes = (uint64_t)ctx->arena.used;
    return LT_OK;
}

}  // namespace lt

using namespace lt;

// =================================================================== C ABI
extern "C" {

void lt_config_init(lt_config *cfg) {
    memset(cfg, 0, sizeof *cfg);
    cfg->device = 0;
    cfg->n_compute_streams = 1;
    cfg->exec_mode = LT_EXEC_PLAIN;
    cfg->device_budget_bytes = (uint64_t)8 << 30;
    cfg->stage_threshold_bytes = 2000000000ull;
}

static std::string g_create_err;

lt_status lt_context_create(const lt_config *cfg_in, lt_context **out) {
    if (!out) return LT_ERR_INVALID;
    *out = nullptr;
    lt_config cfg;
    if (cfg_in) cfg = *cfg_in;
    else lt_config_init(&cfg);
    if (cfg.n_compute_streams < 1 || cfg.n_compute_streams > MAXSTREAM - 2) {
        g_create_err = "n_compute_streams must be in 1..6";
        return LT_ERR_INVALID;
    }
    if (cfg.device_budget_bytes == 0 && !cfg.device_arena) {
        g_create_err = "device_budget_bytes must be > 0";
        return LT_ERR_INVALID;
    }
    if (cfg.device_arena && cfg.arena_bytes == 0) {
        g_create_err = "arena_bytes must be > 0 with device_arena";
        return LT_ERR_INVALID;
    }
    if (cfg.drain_vectors != 0 && cfg.drain_vectors != 2 && cfg.drain_vectors != 4) {
        g_create_err = "drain_vectors must be 0, 2 or 4";
        return LT_ERR_INVALID;
    }
    if (cfg.drain_tile < 0 || cfg.drain_tile % 4096 != 0) {
        g_create_err = "drain_tile must be 0 or a positive multiple of 4096";
        return LT_ERR_INVALID;
    }
    if (cfg.evict_policy != LT_EVICT_NEXT_USE && cfg.evict_policy != LT_EVICT_LRU) {
        g_create_err = "evict_policy must be LT_EVICT_NEXT_USE or LT_EVICT_LRU";
        return LT_ERR_INVALID;
    }
    if (cfg.sb_order < LT_ORDER_ROWMAJOR || cfg.sb_order > LT_ORDER_BANDS || cfg.sb_band < 0) {
        g_create_err = "sb_order must be LT_ORDER_ROWMAJOR, LT_ORDER_SERPENTINE or LT_ORDER_BANDS, sb_band >= 0";
        return LT_ERR_INVALID;
    }
    Ctx *ctx = new Ctx();
    ctx->cfg = cfg;
    if (cfg.spill_dir) ctx->spill_dir = cfg.spill_dir;
    ctx->cfg.spill_dir = ctx->spill_dir.empty() ? nullptr : ctx->spill_dir.c_str();
    ctx->dry = cfg.dry_run != 0;
    ctx->ncompute = cfg.n_compute_streams;
    ctx->h2d = ctx->ncompute;
    ctx->d2h = ctx->ncompute + 1;
    ctx->nstreams = ctx->ncompute + 2;
    memset(&ctx->stats, 0, sizeof ctx->stats);
    if (!ctx->dry) {
        hipError_t r = hipSetDevice(cfg.device);
        if (r != hipSuccess) {
            g_create_err = std::string("hipSetDevice: ") + hipGetErrorString(r);
            delete ctx;
            return LT_ERR_DEVICE;
        }
        for (int s = 0; s < ctx->nstreams; ++s) {
            r = hipStreamCreateWithFlags(&ctx->streams[s].h, hipStreamNonBlocking);
            if (r != hipSuccess) {
                g_create_err = std::string("hipStreamCreate: ") + hipGetErrorString(r);
                for (int q = 0; q < s; ++q) (void)hipStreamDestroy(ctx->streams[q].h);
                delete ctx;
                return LT_ERR_DEVICE;
            }
        }
        // set-up for lt_batch_end_noalloc: the device scratch's address on
        // this device (a failure only disables that call) and the drain
        // error-flag slots it reuses
        ctx->scratch_err = drain_scratch_address(cfg.device, &ctx->scratch);
        r = hipHostMalloc((void **)&ctx->status_host, 64 * 4, hipHostMallocDefault);
        if (r != hipSuccess) {
            g_create_err = std::string("hipHostMalloc(status slots): ") + hipGetErrorString(r);
            for (int q = 0; q < ctx->nstreams; ++q) (void)hipStreamDestroy(ctx->streams[q].h);
            delete ctx;
            return LT_ERR_DEVICE;
        }
        ctx->status_slots = 64;
    }
    *out = ctx;
    return LT_OK;
}

lt_status lt_context_destroy(lt_context *ctx) {
    if (!ctx) return LT_ERR_INVALID;
    lt_status st = sync_all(ctx);
    ctx_release_all(ctx);
    delete ctx;
    return st;
}

lt_status lt_context_configure(lt_context *ctx, const lt_config *cfg) {
    if (!ctx || !cfg) return LT_ERR_INVALID;
    if (cfg->exec_mode != LT_EXEC_PLAIN && cfg->exec_mode != LT_EXEC_GROUPED)
        return set_err(ctx, LT_ERR_INVALID, "unknown exec_mode %d", cfg->exec_mode);
    if (cfg->drain_vectors != 0 && cfg->drain_vectors != 2 && cfg->drain_vectors != 4)
        return set_err(ctx, LT_ERR_INVALID, "drain_vectors must be 0, 2 or 4");
    if (cfg->drain_tile < 0 || cfg->drain_tile % 4096 != 0)
        return set_err(ctx, LT_ERR_INVALID, "drain_tile must be 0 or a positive multiple of 4096");
    if (cfg->evict_policy != LT_EVICT_NEXT_USE && cfg->evict_policy != LT_EVICT_LRU)
        return set_err(ctx, LT_ERR_INVALID, "evict_policy must be LT_EVICT_NEXT_USE or LT_EVICT_LRU");
    if (cfg->sb_order < LT_ORDER_ROWMAJOR || cfg->sb_order > LT_ORDER_BANDS || cfg->sb_band < 0)
        return set_err(ctx, LT_ERR_INVALID,
                       "sb_order must be LT_ORDER_ROWMAJOR, LT_ORDER_SERPENTINE or LT_ORDER_BANDS, sb_band >= 0");
    lt_status st = flush_all(ctx);
    if (st) return st;
    ctx->cfg.exec_mode = cfg->exec_mode;
    ctx->cfg.stage_threshold_bytes = cfg->stage_threshold_bytes;
    ctx->cfg.sb_order = cfg->sb_order;
    ctx->cfg.sb_band = cfg->sb_band;
    ctx->cfg.drain_workgroups = cfg->drain_workgroups;
    ctx->cfg.batch_flush_tasks = cfg->batch_flush_tasks;
    ctx->cfg.drain_vectors = cfg->drain_vectors;
    ctx->cfg.drain_tile = cfg->drain_tile;
    ctx->cfg.evict_policy = cfg->evict_policy;
    ctx->cfg.trace = cfg->trace;
    return LT_OK;
}

const char *lt_last_error(lt_context *ctx) {
    if (!ctx) return g_create_err.c_str();
    return ctx->err.c_str();
}

static lt_status create_common(lt_context *ctx, lt_dtype dtype, int32_t ndim, const int64_t *shape,
                               const lt_dist *dist, void *host_ptr, lt_array **out) {
    if (!ctx || !out) return LT_ERR_INVALID;
    *out = nullptr;
    int esz = dtype_size(dtype);
    if (!esz) return set_err(ctx, LT_ERR_INVALID, "unknown dtype %d", (int)dtype);
    if (ndim < 1 || ndim > 3 || !shape) return set_err(ctx, LT_ERR_INVALID, "ndim must be 1..3");
    for (int a = 0; a < ndim; ++a)
        if (shape[a] <= 0) return set_err(ctx, LT_ERR_INVALID, "shape[%d] must be > 0", a);
    Array *arr = new Array();
    arr->owner = ctx;
    arr->id = ctx->next_array_id++;
    arr->dtype = dtype;
    arr->esz = esz;
    arr->ndim = ndim;
    for (int a = 0; a < MAXD; ++a) arr->shape[a] = a < ndim ? shape[a] : 1;
    int64_t s = 1;
    for (int a = MAXD - 1; a >= 0; --a) {
        arr->strides[a] = s;
        s *= arr->shape[a];
    }
    arr->host_backed = host_ptr != nullptr;
    arr->host_base = (char *)host_ptr;
    if (host_ptr && !ctx->dry) {
        // pinned memory that kernels reach at the same address (lt_host_alloc,
        // hipHostMalloc) can take copy kernels; pageable memory cannot
        hipPointerAttribute_t at;
        if (hipPointerGetAttributes(&at, host_ptr) == hipSuccess)
            arr->home_pinned = at.type == hipMemoryTypeHost && at.devicePointer == host_ptr;
        else
            (void)hipGetLastError();  // pageable: the query's error is not the caller's
    }
    lt_status st = make_chunks(ctx, arr, dist);
    if (st) {
        for (Chunk *c : arr->chunks) delete c;
        delete arr;
        return st;
    }
    if (arr->host_backed) {
        for (Chunk *c : arr->chunks) {
            ensure_host_copy(ctx, c);
            c->host_valid = true;
            c->defined = true;
        }
    } else {
        // admitted whole when it fits right now: one contiguous placement
        alloc_slab(ctx, arr);
    }
    ctx->arrays.push_back(arr);
    *out = arr;
    return LT_OK;
}

lt_status lt_array_create(lt_context *ctx, lt_dtype dtype, int32_t ndim, const int64_t *shape,
                          const lt_dist *dist, lt_array **out) {
    return create_common(ctx, dtype, ndim, shape, dist, nullptr, out);
}

lt_status lt_array_create_host(lt_context *ctx, lt_dtype dtype, int32_t ndim, const int64_t *shape,
                               const lt_dist *dist, void *host_ptr, lt_array **out) {
    if (!host_ptr) return set_err(ctx, LT_ERR_INVALID, "host_ptr is NULL");
    return create_common(ctx, dtype, ndim, shape, dist, host_ptr, out);
}

lt_status lt_array_destroy(lt_context *ctx, lt_array *arr) {
    if (!ctx || !live(ctx, arr)) return set_err(ctx, LT_ERR_INVALID, "invalid array");
    return array_destroy(ctx, arr);
}

lt_status lt_array_write(lt_context *ctx, lt_array *arr, const void *src) {
    if (!ctx || !live(ctx, arr) || !src) return set_err(ctx, LT_ERR_INVALID, "invalid array or source");
    return array_write(ctx, arr, src, false);
}

lt_status lt_array_read(lt_context *ctx, lt_array *arr, void *dst) {
    if (!ctx || !live(ctx, arr) || !dst) return set_err(ctx, LT_ERR_INVALID, "invalid array or destination");
    return array_read(ctx, arr, dst, false);
}

lt_status lt_array_write_device(lt_context *ctx, lt_array *arr, const void *src) {
    if (!ctx || !live(ctx, arr) || !src) return set_err(ctx, LT_ERR_INVALID, "invalid array or source");
    return array_write(ctx, arr, src, true);
}

lt_status lt_array_read_device(lt_context *ctx, lt_array *arr, void *dst) {
    if (!ctx || !live(ctx, arr) || !dst) return set_err(ctx, LT_ERR_INVALID, "invalid array or destination");
    return array_read(ctx, arr, dst, true);
}

lt_status lt_array_fill(lt_context *ctx, lt_array *arr, const void *scalar) {
    if (!ctx || !live(ctx, arr) || !scalar) return set_err(ctx, LT_ERR_INVALID, "invalid array or value");
    return array_fill(ctx, arr, scalar);
}

uint64_t lt_array_id(lt_array *arr) { return arr ? arr->id : 0; }

lt_status lt_host_alloc(lt_context *ctx, uint64_t bytes, void **out) {
    if (!ctx || !out) return LT_ERR_INVALID;
    void *p = nullptr;
    hipError_t r = hipHostMalloc(&p, (size_t)bytes, hipHostMallocDefault);
    if (r != hipSuccess) return set_err(ctx, LT_ERR_OOM, "hipHostMalloc(%llu): %s", (unsigned long long)bytes,
                                        hipGetErrorString(r));
    ctx->host_allocs.push_back(p);
    *out = p;
    return LT_OK;
}

lt_status lt_host_free(lt_context *ctx, void *ptr) {
    if (!ctx) return LT_ERR_INVALID;
    auto it = std::find(ctx->host_allocs.begin(), ctx->host_allocs.end(), ptr);
    if (it == ctx->host_allocs.end()) return set_err(ctx, LT_ERR_INVALID, "pointer not from lt_host_alloc");
    ctx->host_allocs.erase(it);
    hipError_t r = hipHostFree(ptr);
    if (r != hipSuccess) return hip_fail(ctx, r, "hipHostFree");
    return LT_OK;
}

lt_status lt_kernel_get(lt_context *ctx, const char *name, lt_kernel **out) {
    return lt_kernel_define(ctx, name, nullptr, out);
}

lt_status lt_kernel_define(lt_context *ctx, const char *base, const char *annotation, lt_kernel **out) {
    if (!ctx || !out) return LT_ERR_INVALID;
    const KernelDef *def = find_builtin(base);
    if (!def) return set_err(ctx, LT_ERR_INVALID, "unknown kernel '%s'", base ? base : "(null)");
    auto k = std::make_unique<lt_kernel>();
    k->def = def;
    lt_status st = compile_annotation(ctx, def, annotation ? annotation : def->annotation, &k->annot);
    if (st) return st;
    *out = k.get();
    ctx->kernels.push_back(std::move(k));
    return LT_OK;
}

lt_status lt_kernel_define_source(lt_context *ctx, const char *source, const char *function,
                                  const lt_param *params, int32_t nparams, const char *annotation,
                                  lt_kernel **out) {
    if (!ctx || !out) return LT_ERR_INVALID;
    return rtc_define(ctx, source, function, params, nparams, annotation, out);
}

lt_status lt_rtc_stats_get(lt_rtc_stats *out) {
    if (!out) return LT_ERR_INVALID;
    rtc_counters(&out->compiles, &out->loads, &out->compile_seconds);
    return LT_OK;
}

lt_status lt_kernel_tune(lt_context *ctx, lt_kernel *k, int32_t variant) {
    if (!ctx || !k) return LT_ERR_INVALID;
    k->variant = variant;
    return LT_OK;
}

lt_status lt_launch(lt_context *ctx, lt_kernel *k, int32_t ndim, const int64_t *grid, const int64_t *block,
                    const int64_t *superblock, const char *annotation, const lt_arg *args, int32_t nargs,
                    uint64_t *launch_id) {
    if (!ctx) return LT_ERR_INVALID;
    if (nargs > 0 && !args) return set_err(ctx, LT_ERR_INVALID, "args is NULL");
    for (int i = 0; i < nargs; ++i)
        if (args[i].kind == LT_ARG_ARRAY && !live(ctx, args[i].array))
            return set_err(ctx, LT_ERR_INVALID, "argument %d is not a live array of this context", i);
    return launch(ctx, k, ndim, grid, block, superblock, annotation, args, nargs, launch_id);
}

lt_status lt_launch_many(lt_context *ctx, lt_kernel *const *kernels, int32_t count, int32_t ndim,
                         const int64_t *grids, const int64_t *blocks, const int64_t *superblocks,
                         const char *annotation, const lt_arg *args, int32_t nargs, uint64_t *launch_ids) {
    if (!ctx) return LT_ERR_INVALID;
    if (count < 0 || !kernels || !grids || !blocks || ndim < 1 || ndim > 3 || (nargs > 0 && !args))
        return set_err(ctx, LT_ERR_INVALID, "invalid lt_launch_many arguments");
    for (int32_t i = 0; i < count; ++i) {
        const lt_arg *a = args + (size_t)i * nargs;
        for (int j = 0; j < nargs; ++j)
            if (a[j].kind == LT_ARG_ARRAY && !live(ctx, a[j].array))
                return set_err(ctx, LT_ERR_INVALID, "launch %d argument %d is not a live array", i, j);
        uint64_t id = 0;
        lt_status st = launch(ctx, kernels[i], ndim, grids + (size_t)i * ndim, blocks + (size_t)i * ndim,
                              superblocks ? superblocks + (size_t)i * ndim : nullptr, annotation, a, nargs, &id);
        if (launch_ids) launch_ids[i] = id;
        if (st) return st;
    }
    return LT_OK;
}

lt_status lt_batch_begin(lt_context *ctx) {
    if (!ctx) return LT_ERR_INVALID;
    if (ctx->batch.capture) return set_err(ctx, LT_ERR_INVALID, "a graph is being recorded");
    lt_status st = flush_group(ctx);
    if (st) return st;
    ctx->batch.open = true;
    return LT_OK;
}

lt_status lt_batch_end(lt_context *ctx) {
    if (!ctx) return LT_ERR_INVALID;
    if (ctx->batch.capture) return set_err(ctx, LT_ERR_INVALID, "a graph is being recorded (lt_graph_end)");
    lt_status st = batch_flush(ctx);
    ctx->batch.open = false;
    return st;
}

lt_status lt_batch_end_noalloc(lt_context *ctx) {
    if (!ctx) return LT_ERR_INVALID;
    if (ctx->batch.capture) return set_err(ctx, LT_ERR_INVALID, "a graph is being recorded (lt_graph_end)");
    lt_status st = batch_flush_noalloc(ctx);
    // a batch rejected before its issue (too large for the scratch, no
    // scratch, dry run) stays open and unissued; an issued or dropped one
    // leaves an empty queue
    if (ctx->batch.q.empty()) ctx->batch.open = false;
    return st;
}

lt_status lt_graph_begin(lt_context *ctx) {
    if (!ctx) return LT_ERR_INVALID;
    if (ctx->batch.open) return set_err(ctx, LT_ERR_INVALID, "a batch is already open");
    // the graph's edges are replay-time edges: start from a drained context
    lt_status st = sync_all(ctx);
    if (st) return st;
    ctx->batch.open = true;
    ctx->batch.capture = true;
    return LT_OK;
}

lt_status lt_graph_end(lt_context *ctx, lt_graph **out) {
    if (!ctx || !out) return LT_ERR_INVALID;
    *out = nullptr;
    lt_status st = graph_end(ctx, out);
    if (st) {
        batch_drop(ctx);
        ctx->batch.open = false;
        ctx->batch.capture = false;
    }
    return st;
}

lt_status lt_graph_launch(lt_context *ctx, lt_graph *g) {
    if (!ctx || !g) return LT_ERR_INVALID;
    if (ctx->batch.capture) return set_err(ctx, LT_ERR_INVALID, "cannot replay while recording a graph");
    return graph_launch(ctx, g);
}

lt_status lt_graph_destroy(lt_context *ctx, lt_graph *g) {
    if (!ctx || !g) return LT_ERR_INVALID;
    return graph_destroy(ctx, g);
}

lt_status lt_sync(lt_context *ctx) {
    if (!ctx) return LT_ERR_INVALID;
    return sync_all(ctx);
}

lt_status lt_wait(lt_context *ctx, uint64_t launch_id) {
    if (!ctx) return LT_ERR_INVALID;
    lt_status st = flush_all(ctx);
    if (st) return st;
    if (launch_id == 0 || launch_id >= ctx->next_launch_id)
        return set_err(ctx, LT_ERR_INVALID, "unknown launch id %llu", (unsigned long long)launch_id);
    LaunchRec *lr = ctx->launches.get(launch_id);
    if (!lr) return LT_OK;  // completed before the last lt_sync
    st = wait_fence(ctx, lr->done);
    if (st) return st;
    if (ctx->sticky != LT_OK) {
        lt_status s = ctx->sticky;
        ctx->err = ctx->sticky_msg;
        ctx->sticky = LT_OK;
        return s;
    }
    return LT_OK;
}

lt_status lt_plan_tasks(lt_context *ctx, uint64_t launch_id, lt_task_info *out, int32_t cap, int32_t *n) {
    if (!ctx || !n) return LT_ERR_INVALID;
    flush_all(ctx);
    LaunchRec *lr = ctx->launches.get(launch_id);
    if (!lr) return set_err(ctx, LT_ERR_INVALID, "no task records for launch");
    *n = (int32_t)lr->tasks.size();
    for (int i = 0; i < *n && i < cap; ++i) {
        const TaskRec &r = ctx->tasks.at(lr->tasks[i]);
        lt_task_info &t = out[i];
        memset(&t, 0, sizeof t);
        t.id = r.id;
        t.launch = r.launch;
        t.kind = r.kind;
        t.stream = r.stream;
        t.ndeps = (int32_t)r.deps.size();
        t.nregions = (int32_t)r.regions.size();
        for (int a = 0; a < 3; ++a) {
            t.sb_lo[a] = r.sb.lo[a];
            t.sb_hi[a] = r.sb.hi[a];
        }
    }
    return LT_OK;
}

lt_status lt_plan_regions(lt_context *ctx, uint64_t task_id, lt_region_info *out, int32_t cap, int32_t *n) {
    if (!ctx || !n) return LT_ERR_INVALID;
    flush_group(ctx);
    TaskRec *tr = ctx->tasks.get(task_id);
    if (!tr || !tr->id) return set_err(ctx, LT_ERR_INVALID, "unknown task id");
    *n = (int32_t)tr->regions.size();
    for (int i = 0; i < *n && i < cap; ++i) out[i] = tr->regions[i];
    return LT_OK;
}

lt_status lt_plan_deps(lt_context *ctx, uint64_t task_id, uint64_t *out, int32_t cap, int32_t *n) {
    if (!ctx || !n) return LT_ERR_INVALID;
    flush_group(ctx);
    TaskRec *tr = ctx->tasks.get(task_id);
    if (!tr || !tr->id) return set_err(ctx, LT_ERR_INVALID, "unknown task id");
    *n = (int32_t)tr->deps.size();
    for (int i = 0; i < *n && i < cap; ++i) out[i] = tr->deps[i];
    return LT_OK;
}

lt_status lt_stats_get(lt_context *ctx, lt_stats *out) {
    if (!ctx || !out) return LT_ERR_INVALID;
    ctx->stats.resident_bytes = (uint64_t)ctx->arena.used;
    *out = ctx->stats;
    return LT_OK;
}

lt_status lt_stats_reset(lt_context *ctx) {
    if (!ctx) return LT_ERR_INVALID;
    memset(&ctx->stats, 0, sizeof ctx->stats);
    ctx->stats.resident_bytes = ctx->stats.peak_resident_bytes = (uint64_t)ctx->arena.used;
    return LT_OK;
}

lt_status lt_trace_get(lt_context *ctx, lt_trace_rec *out, uint64_t cap, uint64_t *n) {
    if (!ctx || !n) return LT_ERR_INVALID;
    *n = ctx->trace.size();
    for (uint64_t i = 0; i < *n && i < cap; ++i) out[i] = ctx->trace[i];
    return LT_OK;
}

// The origin of the spans: an event recorded now on compute stream 0.
static lt_status prof_mark_base(Ctx *ctx) {
    ctx->prof_spans.clear();
    if (ctx->dry || !ctx->prof) return LT_OK;
    if (!ctx->prof_base) {
        hipError_t r = hipEventCreate(&ctx->prof_base);
        if (r != hipSuccess) {
            ctx->prof_base = nullptr;
            return hip_fail(ctx, r, "hipEventCreate(profile base)");
        }
    }
    hipError_t r = hipEventRecord(ctx->prof_base, ctx->streams[0].h);
    if (r != hipSuccess) return hip_fail(ctx, r, "hipEventRecord(profile base)");
    return LT_OK;
}

lt_status lt_profile_enable(lt_context *ctx, int32_t on) {
    if (!ctx || on < -1) return LT_ERR_INVALID;
    const bool was = ctx->prof != 0;
    ctx->prof = on;
    ctx->prof_seen.clear();
    if (on && !was) return prof_mark_base(ctx);
    return LT_OK;
}

lt_status lt_profile_spans(lt_context *ctx, lt_span *out, uint64_t cap, uint64_t *n) {
    if (!ctx || !n) return LT_ERR_INVALID;
    *n = ctx->prof_spans.size();
    if (out)
        for (uint64_t i = 0; i < *n && i < cap; ++i) out[i] = ctx->prof_spans[i];
    return LT_OK;
}

lt_status lt_profile_get(lt_context *ctx, lt_kernel_prof *out, int32_t cap, int32_t *n) {
    if (!ctx || !n) return LT_ERR_INVALID;
    *n = (int32_t)ctx->prof_acc.size();
    int i = 0;
    for (auto &kv : ctx->prof_acc) {
        if (i < cap && out) out[i] = kv.second;
        ++i;
    }
    return LT_OK;
}

lt_status lt_profile_reset(lt_context *ctx) {
    if (!ctx) return LT_ERR_INVALID;
    ctx->prof_acc.clear();
    ctx->prof_seen.clear();
    return prof_mark_base(ctx);
}

lt_status lt_trace_clear(lt_context *ctx) {
    if (!ctx) return LT_ERR_INVALID;
    ctx->trace.clear();
    return LT_OK;
}

}  // extern "C"
