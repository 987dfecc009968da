// Launch planning and task issue.
//
// lt_launch (Sec. 2.4 "Execution Planner"): the grid is split into
// superblocks; for each superblock and array argument the annotation gives
// an access region, which is resolved against the array's chunks:
//   - a region inside one chunk, or inside a run of chunks that sit next to
//     each other in device memory with the array's own layout, is handed to
//     the kernel as a direct view (no copy);
//   - otherwise a temporary is assembled from the chunks before the kernel
//     and, for writes, scattered back after it (Sec. 2.4: distributions change
//     performance, never results).  Temporaries are loaded before a write too
//     (write-allocate), so elements of the bounding box that the kernel does
//     not write keep their values;
//   - a reduce(f) argument gets a private partial per superblock, initialised
//     to f's identity; one combine task per launch folds the partials into
//     the target, which is overwritten.
// Conflict analysis: each chunk remembers its last writer and the readers
// and reducers since; a new access adds edges for read-after-write,
// write-after-read/write and reduce/other conflicts (Sec. 2.4), so the
// incremental DAG is sequentially consistent.  Edges become device-side
// event waits; the host never blocks while issuing (Sec. 3.3: scheduling
// overlaps planning; here the GPU's queues run the DAG).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <climits>
#include <cstdio>

#include "lt_internal.h"

namespace lt {

namespace {

struct ArgPlan {
    bool used = false;
    Mode mode = M_READ;
    ROp op = R_ADD;
    Box region;
    std::vector<Chunk *> chunks;
    // a read served by one chunk of a halo array: the other owners of the
    // region's elements (their writes reach the task through halo refreshes)
    std::vector<Chunk *> halo_owners;
};

struct TaskPlan {
    uint64_t id = 0;
    Box sb;
    ArgPlan arg[MAXPARAM];
    int64_t footprint = 0;
    int64_t slots = 1;      // partial slots per reduce parameter
};


struct Partials {       // one reduce argument of one launch
    int param = -1;
    ROp op = R_ADD;
    int64_t off = -1;   // arena offset of the partial block
    int64_t bytes = 0;
    int64_t total_elems = 0;
    Fence ready;        // identity fill done
    int64_t cursor = 0; // next free element of the block
    std::vector<CombinePart> parts;
    std::vector<uint64_t> producers;
    bool batched = false;   // block lives in the batch's partial area
    int64_t rel = 0;        // its byte offset there
    int signal = -1;        // batch signal bumped by each producer
};

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// view of `region` backed by memory with element strides `st` whose element
// `org` sits at byte address `addr`
KView make_view(char *addr, const int64_t *org, const int64_t *st, int nd, int esz) {
    KView v;
    int64_t off = 0;
    for (int a = 0; a < nd; ++a) off += org[a] * st[a];
    v.base = (int64_t)(intptr_t)addr - off * esz;
    for (int a = 0; a < KMAXD; ++a) v.s[a] = a < nd ? st[a] : 0;
    return v;
}

// direct view over the chunks of a region, when possible
bool direct_view(Ctx *ctx, const Array *arr, const std::vector<Chunk *> &ch, KView *v) {
    for (Chunk *c : ch)
        if (c->dev_off < 0 || !c->dev_valid) return false;
    if (ch.size() == 1) {
        *v = make_view(dev_ptr(ctx, ch[0]), ch[0]->box.lo, ch[0]->dev_stride, arr->ndim, arr->esz);
        return true;
    }
    if (!arr->row_slab) return false;
    for (size_t i = 0; i + 1 < ch.size(); ++i)
        if (ch[i + 1]->dev_off != ch[i]->dev_off + ch[i]->bytes || ch[i + 1]->box.lo[0] != ch[i]->box.hi[0])
            return false;
    *v = make_view(dev_ptr(ctx, ch[0]), ch[0]->box.lo, ch[0]->dev_stride, arr->ndim, arr->esz);
    return true;
}

// Grid index of the t-th superblock issued (row-major numbering of `nsb`
// superblocks per axis, last axis fastest), in the context's issue order.
// The orders permute only the last two axes; earlier axes stay outermost.
static void sb_index(int64_t t, int nd, const int64_t *nsb, int order, int band, int64_t *idx) {
    int64_t r = t;
    for (int a = nd - 1; a >= 0; --a) {
        idx[a] = r % nsb[a];
        r /= nsb[a];
    }
    if (nd < 2 || order == LT_ORDER_ROWMAJOR) return;
    const int64_t rows = nsb[nd - 2], cols = nsb[nd - 1];
    if (order == LT_ORDER_SERPENTINE) {
        // reverse the fastest axis on every other row of superblocks
        if ((t / cols) & 1) idx[nd - 1] = cols - 1 - idx[nd - 1];
        return;
    }
    // LT_ORDER_BANDS: bands of h rows; within a band column by column, the
    // rows of a column in turn (reversed on odd columns, so the row a column
    // ends on starts the next); odd bands run right to left
    const int64_t h = band > 0 ? band : 2;
    const int64_t u = t % (rows * cols);
    const int64_t b = u / (h * cols);       // every band before b is full
    const int64_t r0 = b * h;
    const int64_t hb = std::min(h, rows - r0);
    const int64_t v = u - b * h * cols;
    const int64_t ci = v / hb;
    int64_t ri = v % hb;
    if (ci & 1) ri = hb - 1 - ri;
    idx[nd - 2] = r0 + ri;
    idx[nd - 1] = (b & 1) ? cols - 1 - ci : ci;
}

void add_dep(std::vector<uint64_t> *deps, uint64_t id) {
    if (id && std::find(deps->begin(), deps->end(), id) == deps->end()) deps->push_back(id);
}

// dependency edges for one access of `c` (Sec. 2.4 conflicts)
void conflict_edges(const Chunk *c, Mode m, ROp op, std::vector<uint64_t> *deps) {
    add_dep(deps, c->last_writer);
    if (m == M_READ) {
        for (uint64_t r : c->reducers) add_dep(deps, r);
        return;
    }
    if (m == M_REDUCE) {
        for (uint64_t r : c->readers) add_dep(deps, r);
        if (c->reduce_op != (int)op)
            for (uint64_t r : c->reducers) add_dep(deps, r);
        return;
    }
    for (uint64_t r : c->readers) add_dep(deps, r);
    for (uint64_t r : c->reducers) add_dep(deps, r);
}

void record_access(Chunk *c, Mode m, ROp op, uint64_t id) {
    if (m == M_READ) {
        c->readers.push_back(id);
    } else if (m == M_REDUCE) {
        if (c->reduce_op != (int)op) c->reducers.clear();
        c->reduce_op = (int)op;
        c->reducers.push_back(id);
    } else {
        c->last_writer = id;
        c->readers.clear();
        c->reducers.clear();
        c->reduce_op = -1;
    }
}

Fence task_fence(Ctx *ctx, const std::vector<uint64_t> &deps) {
    Fence f;
    for (uint64_t d : deps) {
        TaskRec *r = ctx->tasks.get(d);
        if (r && r->seq) f.add(r->stream, r->seq);
    }
    return f;
}

}  // namespace

static Group &group_of(Ctx *ctx) { return ctx->group; }

static void apply_uses(Ctx *ctx, const std::vector<ChunkUse> &uses, int s, uint64_t p) {
    for (const ChunkUse &u : uses) {
        Chunk *c = u.c;
        c->last_access.add(s, p);
        if (u.write) {
            c->data_ready = Fence();
            c->data_ready.add(s, p);
            c->host_valid = false;
            c->defined = true;
            c->version++;
        }
    }
    (void)ctx;
}

static hipEvent_t prof_event(Ctx *ctx) {
    if (!ctx->prof_pool.empty()) {
        hipEvent_t e = ctx->prof_pool.back();
        ctx->prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

lt_status prof_begin(Ctx *ctx, int s, const char *name, hipEvent_t *a) {
    *a = nullptr;
    if (ctx->prof <= 0 || ctx->dry) return LT_OK;  // off, or whole steps (dispatch)
    if (ctx->prof > 1 && ctx->prof_seen[name]++ % (uint64_t)ctx->prof != 0) return LT_OK;  // sampled
    *a = prof_event(ctx);
    hipError_t r = hipEventRecord(*a, ctx->streams[s].h);
    if (r != hipSuccess) return hip_fail(ctx, r, "hipEventRecord(profile)");
    return LT_OK;
}

lt_status prof_end(Ctx *ctx, int s, const char *name, hipEvent_t a) {
    if (!a) return LT_OK;
    hipEvent_t b = prof_event(ctx);
    hipError_t r = hipEventRecord(b, ctx->streams[s].h);
    if (r != hipSuccess) return hip_fail(ctx, r, "hipEventRecord(profile)");
    ctx->prof_pending.push_back({name, a, b, s, 1});
    return LT_OK;
}

void prof_collect(Ctx *ctx) {
    for (auto &p : ctx->prof_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            lt_kernel_prof &k = ctx->prof_acc[p.name];
            snprintf(k.name, sizeof k.name, "%s", p.name);
            k.dispatches += p.count;
            k.total_ms += ms;
            if (ms > k.max_ms) k.max_ms = ms;
            float t0 = 0.f;
            if (ctx->prof_base && ctx->prof_spans.size() < ((size_t)1 << 22) &&
                hipEventElapsedTime(&t0, ctx->prof_base, p.a) == hipSuccess) {
                lt_span sp;
                memset(&sp, 0, sizeof sp);
                snprintf(sp.name, sizeof sp.name, "%s", p.name);
                sp.stream = p.stream;
                sp.start_ms = t0;
                sp.end_ms = (double)t0 + ms;
                ctx->prof_spans.push_back(sp);
            }
        }
        ctx->prof_pool.push_back(p.a);
        ctx->prof_pool.push_back(p.b);
    }
    ctx->prof_pending.clear();
}

lt_status prof_close_steps(Ctx *ctx) {
    if (ctx->dry) return LT_OK;
    for (int s = 0; s < ctx->nstreams; ++s) {
        Stream &S = ctx->streams[s];
        if (!S.step_a) continue;
        hipEvent_t b = prof_event(ctx);
        hipError_t r = hipEventRecord(b, S.h);
        if (r != hipSuccess) return hip_fail(ctx, r, "hipEventRecord(profile)");
        ctx->prof_pending.push_back({S.step_name, S.step_a, b, s, S.step_count});
        S.step_a = nullptr;
        S.step_count = 0;
    }
    return LT_OK;
}

static lt_status dispatch(Ctx *ctx, const KernelDef *def, KLaunch &kl, int s) {
    ctx->stats.dispatches++;
    trace_op(ctx, 0, s, kl.ntask ? 0 : ~0ull, 0, (uint64_t)kl.ntask, 0);
    if (ctx->dry) return LT_OK;
    kl.stream = ctx->streams[s].h;
    if (ctx->prof < 0) {
        // whole steps: one event before the stream's first dispatch since
        // the last sync, one at the sync
        Stream &S = ctx->streams[s];
        if (!S.step_a) {
            S.step_a = prof_event(ctx);
            hipError_t r = hipEventRecord(S.step_a, S.h);
            if (r != hipSuccess) return hip_fail(ctx, r, "hipEventRecord(profile)");
            S.step_name = def->name;
        }
        S.step_count++;
    }
    hipEvent_t pa;
    lt_status st = prof_begin(ctx, s, def->name, &pa);
    if (st) return st;
    hipError_t r = def->fn(kl);
    if (r != hipSuccess) {
        if (const char *m = rtc_last_error(def)) return set_err(ctx, LT_ERR_DEVICE, "%s", m);
        return hip_fail(ctx, r, def->name);
    }
    return prof_end(ctx, s, def->name, pa);
}

lt_status flush_group(Ctx *ctx) {
    Group &g = group_of(ctx);
    if (!g.open) return LT_OK;
    g.open = false;
    lt_status st = stream_wait(ctx, g.stream, g.wait);
    if (st) return st;
    // tasks beyond the kernel's group size go in further dispatches
    int mg = std::max(1, std::min(g.def->max_group, KMAXG));
    for (size_t i = 0; i < g.tasks.size(); i += mg) {
        KLaunch kl = g.proto;
        kl.ntask = (int)std::min<size_t>(mg, g.tasks.size() - i);
        kl.tasks = g.tasks.data() + i;
        st = dispatch(ctx, g.def, kl, g.stream);
        if (st) return st;
        bump(ctx, g.stream);
    }
    uint64_t p = ctx->streams[g.stream].seq;
    for (uint64_t id : g.ids) {
        TaskRec &r = ctx->tasks.at(id);
        r.stream = g.stream;
        r.seq = p;
    }
    apply_uses(ctx, g.uses, g.stream, p);
    g.tasks.clear();
    g.ids.clear();
    g.uses.clear();
    return LT_OK;
}

static int pick_stream(Ctx *ctx, const Fence &deps) {
    if (ctx->ncompute == 1) return 0;
    int only = -1, cnt = 0;
    for (int s = 0; s < ctx->ncompute; ++s)
        if (deps.s[s] > ctx->streams[s].done) {
            only = s;
            ++cnt;
        }
    if (cnt == 1) return only;
    int s = ctx->rr;
    ctx->rr = (ctx->rr + 1) % ctx->ncompute;
    return s;
}

// Staging throttle (Sec. 3.4): the summed footprint of tasks that have
// loaded data ahead of their execution stays under the threshold; the copy
// stream waits for the oldest staged tasks to finish.  One task is always
// admitted.
static lt_status throttle(Ctx *ctx, int64_t footprint) {
    int64_t thr = (int64_t)ctx->cfg.stage_threshold_bytes;
    while (!ctx->staged.empty() && ctx->staged_bytes + footprint > thr) {
        auto f = ctx->staged.front();
        ctx->staged.pop_front();
        ctx->staged_bytes -= f.second;
        lt_status st = stream_wait(ctx, ctx->h2d, f.first);
        if (st) return st;
        ctx->stats.throttle_waits++;
    }
    return LT_OK;
}

// Makes chunk c resident and valid on the device for an access of mode m
// that covers `region`.  Device-side prerequisites go into *wait.
static lt_status stage_chunk(Ctx *ctx, Chunk *c, Mode m, const Box &region,
                             Fence *wait, bool *staged_copy, int64_t footprint,
                             const Fence &placed) {
    const int nd = c->arr->ndim;
    Fence mem = placed;
    if (c->dev_off < 0) {
        Fence f;
        lt_status st = alloc_chunk(ctx, c, &f);
        if (st) return st;
        mem.merge(f);
        c->dev_valid = false;
    }
    if (!c->dev_valid) {
        lt_status st;
        // a write that covers the whole core need not load the chunk; its
        // halo replicas are then refreshed before they are next read
        bool overwrite = (m == M_WRITE) && region.contains(c->core, nd);
        if (overwrite)
            for (HaloSrc &h : c->halo) h.valid = false;
        if (c->host_valid && c->defined && !overwrite) {
            if (!*staged_copy) {
                st = throttle(ctx, footprint);
                if (st) return st;
                *staged_copy = true;
            }
            Fence f = mem;
            f.merge(c->host_ready);
            if (c->arr->host_backed)
                // the halo comes from the owners' cores in the home buffer
                for (HaloSrc &h : c->halo) {
                    f.merge(h.k->host_ready);
                    h.ver = h.k->host_version;
                    h.valid = true;
                }
            st = host_resident(ctx, c);  // back from the disk tier if it was moved there
            if (st) return st;
            st = stream_wait(ctx, ctx->h2d, f);
            if (st) return st;
            int64_t ext[MAXD];
            for (int a = 0; a < MAXD; ++a) ext[a] = c->box.hi[a] - c->box.lo[a];
            if (c->arr->host_backed && !c->arr->home_pinned && !ctx->dry)
                // a pageable home: packed into pinned bounce buffers first
                st = bounce_h2d(ctx, ctx->h2d, dev_ptr(ctx, c), c->dev_stride, c->host_ptr, c->host_stride, ext,
                                nd, c->arr->esz);
            else
                st = copy_box(ctx, ctx->h2d, dev_ptr(ctx, c), c->dev_stride, c->host_ptr, c->host_stride, ext,
                              nd, c->arr->esz, hipMemcpyHostToDevice);
            if (st) return st;
            uint64_t p = bump(ctx, ctx->h2d);
            trace_op(ctx, 1, ctx->h2d, ~0ull, c->id, c->bytes, c->dev_off);
            c->data_ready = Fence();
            c->data_ready.add(ctx->h2d, p);
            c->last_access = mem;
            c->last_access.add(ctx->h2d, p);
        } else {
            c->data_ready = mem;
            c->last_access = mem;
        }
        c->dev_valid = true;
    }
    if (!c->halo.empty() && m != M_WRITE && m != M_REDUCE) {
        lt_status st = refresh_halo(ctx, c, region);
        if (st) return st;
    }
    wait->merge(c->data_ready);
    // a write must also follow every earlier use of the memory
    if (m != M_READ) wait->merge(c->last_access);
    c->lru = ++ctx->lru_clock;
    return LT_OK;
}

struct Temp {
    int param;
    int64_t off;
    Box region;
    int64_t stride[MAXD];
    std::vector<Chunk *> chunks;
    bool scatter;
};

// Copies between chunk c and a temporary: the part of the region that c
// owns (its core), so halo replicas are never read or written here.
static lt_status copy_region(Ctx *ctx, int s, Chunk *c, const Temp &t, int esz, int nd, bool to_temp) {
    Box o = intersect(c->core, t.region, nd);
    if (o.empty(nd)) return LT_OK;
    int64_t coff = 0, toff = 0, ext[MAXD];
    for (int a = 0; a < MAXD; ++a) {
        int64_t lo = a < nd ? o.lo[a] : 0;
        coff += (lo - (a < nd ? c->box.lo[a] : 0)) * c->dev_stride[a];
        toff += (lo - (a < nd ? t.region.lo[a] : 0)) * t.stride[a];
        ext[a] = a < nd ? o.hi[a] - o.lo[a] : 1;
    }
    char *cp = dev_ptr(ctx, c) + coff * esz;
    char *tp = ctx->arena_base + t.off + toff * esz;
    if (to_temp)
        return copy_box(ctx, s, tp, t.stride, cp, c->dev_stride, ext, nd, esz, hipMemcpyDeviceToDevice);
    return copy_box(ctx, s, cp, c->dev_stride, tp, t.stride, ext, nd, esz, hipMemcpyDeviceToDevice);
}

static void identity_bytes(lt_dtype dt, ROp op, unsigned char *out, int *esz) {
    if (dt == LT_F32) {
        float v = op == R_ADD ? 0.f : op == R_MUL ? 1.f : op == R_MIN ? INFINITY : -INFINITY;
        memcpy(out, &v, 4);
        *esz = 4;
    } else if (dt == LT_I32) {
        int32_t v = op == R_ADD ? 0 : op == R_MUL ? 1 : op == R_MIN ? INT32_MAX : INT32_MIN;
        memcpy(out, &v, 4);
        *esz = 4;
    } else if (dt == LT_F64) {
        double v = op == R_ADD ? 0. : op == R_MUL ? 1. : op == R_MIN ? INFINITY : -INFINITY;
        memcpy(out, &v, 8);
        *esz = 8;
    } else {
        int64_t v = op == R_ADD ? 0 : op == R_MUL ? 1 : op == R_MIN ? INT64_MAX : INT64_MIN;
        memcpy(out, &v, 8);
        *esz = 8;
    }
}

// ------------------------------------------------------------ batched path
// Between lt_batch_begin and lt_batch_end, tasks become entries of a device
// queue drained by one persistent kernel.  Edges to tasks of the same batch
// become counter waits inside the kernel; edges to earlier work become one
// stream wait before the drain.  Every chunk a batched task touches must
// already be resident (no staging inside the drain).

// signal and counter indices are only known at the end: encode them as
// negative markers until then
static int32_t sig_marker(int s) { return -2 - s; }

static lt_status batch_dep(Ctx *ctx, DTask &d, uint64_t dep) {
    Batch &B = ctx->batch;
    int qi = B.find(dep);
    if (qi < 0) {
        TaskRec *tr = ctx->tasks.get(dep);
        if (tr && tr->seq) B.wait.add(tr->stream, tr->seq);
        return LT_OK;
    }
    for (int i = 0; i < d.ndeps; ++i)
        if (d.dep_ctr[i] == qi) return LT_OK;
    if (d.ndeps >= DMAXDEP)
        return set_err(ctx, LT_ERR_UNSUPPORTED, "a batched task has more than %d predecessors in its batch", DMAXDEP);
    d.dep_ctr[d.ndeps] = qi;
    d.dep_val[d.ndeps] = B.q[qi].ntiles;
    d.ndeps++;
    B.q[qi].flags |= DF_RELEASE;  // its stores are read by a later task of the batch
    return LT_OK;
}

static void batch_push(Ctx *ctx, DTask &d, uint64_t id) {
    Batch &B = ctx->batch;
    if (d.ntiles < 1) d.ntiles = 1;  // an empty task still completes (and signals)
    d.tile_begin = B.tiles;
    B.tiles += d.ntiles;
    B.kinds |= 1u << d.kind;
    if (B.index.empty()) B.index_base = id;
    if (id - B.index_base >= B.index.size()) B.index.resize(id - B.index_base + 1, -1);
    B.index[id - B.index_base] = (int)B.q.size();
    B.q.push_back(d);
    B.ids.push_back(id);
}

static lt_status batch_add_exec(Ctx *ctx, const KernelDef *def, TaskPlan &tp, TaskRec &rec, const KLaunch &proto,
                                Array **arrs, std::vector<Partials> &parts) {
    Batch &B = ctx->batch;
    DTask d;
    memset(&d, 0, sizeof d);
    d.signal = -1;
    KTask kt;
    memset(&kt, 0, sizeof kt);
    std::vector<ChunkUse> uses;
    for (int p = 0; p < def->nparam; ++p) {
        ArgPlan &a = tp.arg[p];
        if (!a.used) continue;
        Array *arr = arrs[p];
        if (a.mode == M_REDUCE) {
            Partials *P = nullptr;
            for (auto &x : parts)
                if (x.param == p) P = &x;
            if (tp.slots > 1)
                return set_err(ctx, LT_ERR_UNSUPPORTED, "%s folds floats over several partial slots and cannot "
                               "run inside a batch", def->name);
            CombinePart cp;
            cp.off = P->cursor;
            cp.count = 1;
            P->cursor += a.region.volume(arr->ndim);
            int64_t org = 0, s = 1;
            for (int q = MAXD - 1; q >= 0; --q) {
                org += (q < arr->ndim ? a.region.lo[q] : 0) * s;
                s *= q < arr->ndim ? a.region.hi[q] - a.region.lo[q] : 1;
            }
            for (int q = 0; q < KMAXD; ++q) {
                cp.lo[q] = a.region.lo[q];
                cp.hi[q] = a.region.hi[q];
            }
            P->parts.push_back(cp);
            P->producers.push_back(tp.id);
            // relative byte address of element 0 of the partial's view
            kt.v[p].base = P->rel + (cp.off - org) * arr->esz;
            kt.v[p].s[0] = 1;
            d.signal = sig_marker(P->signal);
            rec.regions.push_back(lt_region_info{p, (int)a.mode, (int)a.op, 2, arr->id,
                                                 {a.region.lo[0], a.region.lo[1], a.region.lo[2]},
                                                 {a.region.hi[0], a.region.hi[1], a.region.hi[2]}});
            continue;
        }
        if (!direct_view(ctx, arr, a.chunks, &kt.v[p]))
            return set_err(ctx, LT_ERR_UNSUPPORTED,
                           "inside a batch every chunk a task touches must be resident and contiguous (%s)",
                           def->params[p].name);
        if (a.mode != M_WRITE)
            for (Chunk *c : a.chunks)
                if (halo_stale(c, a.region))
                    return set_err(ctx, LT_ERR_UNSUPPORTED,
                                   "inside a batch a halo read needs replicas refreshed before the batch (%s)",
                                   def->params[p].name);
        // device work on these chunks outside any task (halo refreshes)
        for (Chunk *c : a.chunks) {
            B.wait.merge(c->data_ready);
            if (a.mode != M_READ) B.wait.merge(c->last_access);
        }
        for (Chunk *c : a.chunks) {
            c->lru = ++ctx->lru_clock;
            uses.push_back({c, a.mode != M_READ});
        }
        rec.regions.push_back(lt_region_info{p, (int)a.mode, (int)a.op, 0, arr->id,
                                             {a.region.lo[0], a.region.lo[1], a.region.lo[2]},
                                             {a.region.hi[0], a.region.hi[1], a.region.hi[2]}});
        ctx->stats.direct_regions++;
    }
    d.lo0 = tp.sb.lo[0];
    d.hi0 = tp.sb.hi[0];
    d.lo1 = tp.sb.lo[1];
    d.hi1 = tp.sb.hi[1];
    bool partial_y = false;
    if (def->dkind == DK_TOUCH) {
        d.kind = DK_TOUCH;
        d.n = proto.iarg[0];
        d.y = kt.v[1].base;
    } else if (def->dkind == DK_STENCIL1D) {
        d.kind = DK_STENCIL1D;
        d.n = proto.iarg[0];
        d.y = kt.v[1].base;
        d.x = kt.v[2].base;
    } else if (def->dkind == DK_HIST256) {
        d.kind = DK_HIST256;
        d.n = proto.iarg[0];
        d.y = kt.v[1].base;
        d.x = kt.v[2].base;
        partial_y = true;
    } else if (def->dkind == DK_JACOBI2D) {
        d.kind = DK_JACOBI2D;
        d.n = proto.iarg[0];
        d.m = proto.iarg[1];
        d.y = kt.v[2].base;
        d.x = kt.v[3].base;
        d.ys = kt.v[2].s[0];
        d.xs = kt.v[3].s[0];
        d.hi0 = std::min(d.hi0, d.n);
        d.hi1 = std::min(d.hi1, d.m);
        d.vec = ((d.x + d.lo1 * 4) & 15) == 0 && ((d.y + d.lo1 * 4) & 15) == 0 && (d.xs & 3) == 0 &&
                (d.ys & 3) == 0 && ((d.hi1 - d.lo1) & 3) == 0;
        int64_t cols = d.hi1 - d.lo1, rows = d.hi0 - d.lo0;
        d.tx = cols > 0 ? (int)((cols + 1023) / 1024) : 1;
        d.ntiles = rows > 0 && cols > 0 ? (int)(((rows + DJROWS - 1) / DJROWS) * d.tx) : 0;
    } else {
        return set_err(ctx, LT_ERR_UNSUPPORTED, "%s cannot run inside a batch", def->name);
    }
    if (d.kind != DK_JACOBI2D) {
        // the touch body walks DSPAN-element tiles; the stencil and
        // histogram bodies take whatever count of interleaved tiles
        // (defaults measured on the 8192-launch mix: stencil tasks stream
        // fastest in tiles of 16 Ki elements, histogram tasks, which flush
        // their sub-histograms once per tile, in tiles of 64 Ki)
        const int64_t span = d.kind == DK_TOUCH              ? DSPAN
                             : ctx->cfg.drain_tile > 0       ? ctx->cfg.drain_tile
                             : d.kind == DK_HIST256          ? DSPAN
                                                             : DTILE;
        int64_t e = std::min(d.hi0, d.n) - d.lo0;
        d.ntiles = e > 0 ? (int)((e + span - 1) / span) : 0;
    }
    for (uint64_t dep : rec.deps) {
        lt_status st = batch_dep(ctx, d, dep);
        if (st) return st;
    }
    for (int p = 0; p < def->nparam; ++p) {
        ArgPlan &a = tp.arg[p];
        if (!a.used || a.mode == M_REDUCE) continue;
        for (Chunk *c : a.chunks) record_access(c, a.mode, a.op, tp.id);
        for (Chunk *k : a.halo_owners) record_access(k, M_READ, a.op, tp.id);
    }
    if (partial_y) {
        B.patch_y.push_back({(int)B.q.size(), 0});
        d.flags |= DF_ATOMIC;  // its partial is built with device-scope atomics
    }
    batch_push(ctx, d, tp.id);
    for (const ChunkUse &u : uses) {
        u.c->pin++;
        B.uses.push_back(u);
        if (u.write) B.written.insert(u.c);
    }
    if (B.launches.empty() || B.launches.back() != rec.launch) B.launches.push_back(rec.launch);
    ctx->tasks.at(tp.id) = std::move(rec);
    return LT_OK;
}

static lt_status batch_add_combine(Ctx *ctx, Partials &P, Array *arr, uint64_t L) {
    Batch &B = ctx->batch;
    const int nd = arr->ndim;
    if (P.parts.empty()) return LT_OK;
    if (nd != 1 || P.op != R_ADD || arr->dtype != LT_I32)
        return set_err(ctx, LT_ERR_UNSUPPORTED, "batched reductions support int32 reduce(+) on 1-D targets");
    for (auto &q : P.parts)
        if (q.lo[0] != P.parts[0].lo[0] || q.hi[0] != P.parts[0].hi[0])
            return set_err(ctx, LT_ERR_UNSUPPORTED, "batched reductions need equal partial boxes");
    Box U;
    U.lo[0] = P.parts[0].lo[0];
    U.hi[0] = P.parts[0].hi[0];
    TaskRec rec;
    rec.id = ctx->next_task_id++;
    rec.launch = L;
    rec.kind = LT_TASK_COMBINE;
    rec.sb = U;
    std::vector<Chunk *> ch;
    chunks_overlapping(arr, U, &ch);
    for (Chunk *c : ch) conflict_edges(c, M_WRITE, R_ADD, &rec.deps);
    DTask d;
    memset(&d, 0, sizeof d);
    d.signal = -1;
    d.kind = DK_SUM_PARTIALS;
    KView tv;
    if (!direct_view(ctx, arr, ch, &tv))
        return set_err(ctx, LT_ERR_UNSUPPORTED, "inside a batch the reduction target must be resident");
    d.y = tv.base;
    d.lo0 = U.lo[0];
    d.hi0 = U.hi[0];
    d.m = U.hi[0] - U.lo[0];
    d.aux = (int64_t)P.parts.size();
    d.x = P.rel;
    d.ndeps = 1;
    d.dep_ctr[0] = sig_marker(P.signal);
    d.dep_val[0] = (int32_t)P.producers.size();
    for (uint64_t dep : rec.deps) {
        lt_status st = batch_dep(ctx, d, dep);
        if (st) return st;
    }
    B.patch_x.push_back({(int)B.q.size(), 0});
    d.ntiles = 1;
    batch_push(ctx, d, rec.id);
    for (Chunk *c : ch) {
        record_access(c, M_WRITE, R_ADD, rec.id);
        c->lru = ++ctx->lru_clock;
        c->pin++;
        B.uses.push_back({c, true});
        B.written.insert(c);
    }
    rec.regions.push_back(lt_region_info{P.param, (int)M_REDUCE, (int)P.op, 0, arr->id,
                                         {U.lo[0], U.lo[1], U.lo[2]}, {U.hi[0], U.hi[1], U.hi[2]}});
    ctx->launches.at(L).tasks.push_back(rec.id);
    if (B.launches.empty() || B.launches.back() != L) B.launches.push_back(L);
    ctx->tasks.at(rec.id) = std::move(rec);
    return LT_OK;
}

static void *staging_get(Ctx *ctx, uint64_t bytes, lt_status *st) {
    for (size_t i = 0; i < ctx->staging_free.size(); ++i)
        if (ctx->staging_size_free[i] >= bytes) {
            void *p = ctx->staging_free[i];
            ctx->staging_used.push_back(p);
            ctx->staging_size_used.push_back(ctx->staging_size_free[i]);
            ctx->staging_free.erase(ctx->staging_free.begin() + i);
            ctx->staging_size_free.erase(ctx->staging_size_free.begin() + i);
            return p;
        }
    uint64_t sz = std::max<uint64_t>(bytes, 1 << 20);
    void *p = nullptr;
    if (ctx->dry) {
        p = malloc(sz);
    } else {
        hipError_t r = hipHostMalloc(&p, sz, hipHostMallocDefault);
        if (r != hipSuccess) {
            *st = set_err(ctx, LT_ERR_OOM, "pinned staging buffer: %s", hipGetErrorString(r));
            return nullptr;
        }
    }
    ctx->staging_used.push_back(p);
    ctx->staging_size_used.push_back(sz);
    return p;
}

// Reads of halo replicas while a batch is open.  Versions move only when a
// batch is issued, so a replica whose owner a queued task writes still looks
// current: it can be refreshed only after the batch has run, so the batch is
// issued first (*flush).  A graph cannot refresh replicas between or inside
// its replays, so a graph that reads replicas is refused.
static lt_status batch_halo_reads(Ctx *ctx, std::vector<TaskPlan> &plans, Array **arrs, int nparam,
                                  bool *flush) {
    Batch &B = ctx->batch;
    *flush = false;
    for (auto &tp : plans)
        for (int p = 0; p < nparam; ++p) {
            ArgPlan &a = tp.arg[p];
            if (!a.used || a.mode == M_WRITE || a.mode == M_REDUCE || !arrs[p]->has_halo) continue;
            const int nd = arrs[p]->ndim;
            for (Chunk *c : a.chunks)
                for (const HaloSrc &h : c->halo) {
                    if (intersect(h.box, a.region, nd).empty(nd)) continue;
                    if (B.capture)
                        return set_err(ctx, LT_ERR_UNSUPPORTED,
                                       "a graph cannot read halo replicas: a replay could not refresh them");
                    if (B.written.count(h.k)) *flush = true;
                }
        }
    return LT_OK;
}

// Halo replicas that the reads of a launch will use, refreshed up front from
// owners on the device with one copy dispatch (per element size), so the
// launch's tasks find their halos current and keep their direct views and
// grouped dispatch.  Pieces whose owner is not on the device are left to the
// per-task staging (refresh_halo).
static lt_status refresh_launch_halos(Ctx *ctx, std::vector<TaskPlan> &plans, Array **arrs, int nparam) {
    std::vector<std::pair<Chunk *, HaloSrc *>> pieces;
    std::vector<HaloSrc *> seen;
    for (auto &tp : plans)
        for (int p = 0; p < nparam; ++p) {
            ArgPlan &a = tp.arg[p];
            if (!a.used || a.mode == M_WRITE || a.mode == M_REDUCE || a.chunks.size() != 1) continue;
            Array *arr = arrs[p];
            if (!arr->has_halo) continue;
            Chunk *c = a.chunks[0];
            if (c->dev_off < 0 || !c->dev_valid) continue;
            const int nd = arr->ndim;
            for (HaloSrc &h : c->halo) {
                Chunk *k = h.k;
                if ((h.valid && h.ver >= k->version) || intersect(h.box, a.region, nd).empty(nd)) continue;
                if (!k->defined) {
                    h.ver = k->version;
                    h.valid = true;
                    continue;
                }
                if (k->dev_off < 0 || !k->dev_valid) continue;
                if (std::find(seen.begin(), seen.end(), &h) != seen.end()) continue;
                seen.push_back(&h);
                pieces.push_back({c, &h});
            }
        }
    if (pieces.empty()) return LT_OK;
    lt_status st = flush_group(ctx);
    if (st) return st;
    for (int esz : {1, 4, 8}) {
        std::vector<CopyBoxEntry> table;
        std::vector<std::pair<Chunk *, HaloSrc *>> mine;
        Fence wait;
        int64_t max_elems = 0;
        for (auto &pc : pieces) {
            Chunk *c = pc.first;
            HaloSrc &h = *pc.second;
            Chunk *k = h.k;
            const Array *arr = c->arr;
            if (arr->esz != esz) continue;
            const int nd = arr->ndim;
            CopyBoxEntry e;
            int64_t so = 0, dof = 0, vol = 1;
            for (int a = 0; a < 3; ++a) {
                const bool in = a < nd;
                so += in ? (h.box.lo[a] - k->box.lo[a]) * k->dev_stride[a] : 0;
                dof += in ? (h.box.lo[a] - c->box.lo[a]) * c->dev_stride[a] : 0;
                e.ext[a] = in ? h.box.hi[a] - h.box.lo[a] : 1;
                e.ss[a] = k->dev_stride[a];
                e.ds[a] = c->dev_stride[a];
                vol *= e.ext[a];
            }
            e.src = (int64_t)(intptr_t)(dev_ptr(ctx, k) + so * esz);
            e.dst = (int64_t)(intptr_t)(dev_ptr(ctx, c) + dof * esz);
            max_elems = std::max(max_elems, vol);
            table.push_back(e);
            mine.push_back(pc);
            wait.merge(k->data_ready);
            wait.merge(c->data_ready);
            wait.merge(c->last_access);
        }
        for (size_t b = 0; b < table.size(); b += 65535) {
            const int n = (int)std::min<size_t>(65535, table.size() - b);
            const int64_t bytes = (int64_t)n * (int64_t)sizeof(CopyBoxEntry);
            // the table's arena range must not evict the chunks being copied
            for (size_t i = b; i < b + n; ++i) {
                mine[i].first->pin++;
                mine[i].second->k->pin++;
            }
            int64_t off;
            Fence mem;
            st = alloc_range(ctx, (bytes + 255) / 256 * 256, 2, nullptr, &off, &mem);
            for (size_t i = b; i < b + n; ++i) {
                mine[i].first->pin--;
                mine[i].second->k->pin--;
            }
            if (st) return st;
            void *stage = staging_get(ctx, (uint64_t)bytes, &st);
            if (!stage) return st;
            memcpy(stage, table.data() + b, (size_t)bytes);
            Fence f = wait;
            f.merge(mem);
            const int s = pick_stream(ctx, f);
            st = stream_wait(ctx, s, f);
            if (st) return st;
            if (!ctx->dry) {
                hipStream_t hs = ctx->streams[s].h;
                hipError_t r = hipMemcpyAsync(ctx->arena_base + off, stage, (size_t)bytes, hipMemcpyHostToDevice, hs);
                if (r != hipSuccess) return hip_fail(ctx, r, "halo table upload");
                r = launch_copy_boxes(hs, reinterpret_cast<const CopyBoxEntry *>(ctx->arena_base + off), n, esz,
                                      max_elems);
                if (r != hipSuccess) return hip_fail(ctx, r, "halo refresh");
            }
            const uint64_t p = bump(ctx, s);
            ctx->stats.dispatches++;
            trace_op(ctx, 0, s, ~0ull, 0, (uint64_t)n, 2);
            Fence done;
            done.add(s, p);
            ctx->arena.release(off, done);
            for (size_t i = b; i < b + n; ++i) {
                Chunk *c = mine[i].first;
                HaloSrc &h = *mine[i].second;
                c->data_ready.add(s, p);
                c->last_access.add(s, p);
                h.k->last_access.add(s, p);
                if (!c->arr->host_backed) c->host_valid = false;
                h.ver = h.k->version;
                h.valid = true;
                ctx->stats.halo_copies++;
            }
        }
    }
    return LT_OK;
}

void batch_drop(Ctx *ctx) {
    Batch &B = ctx->batch;
    for (const ChunkUse &u : B.uses) u.c->pin--;
    const bool open = B.open;
    B = Batch();
    B.open = open;
}

static lt_status batch_issue(Ctx *ctx, bool noalloc = false);

// Bytes of device memory the open batch needs at issue: queue, counters
// (one per task and signal, the ticket and the error flag), partials.
static void batch_layout(const Batch &B, int64_t *qbytes, int64_t *qalloc, int64_t *calloc_, int64_t *total) {
    const int ntasks = (int)B.q.size();
    const int nctr = ntasks + B.nsignals + 2;
    *qbytes = (int64_t)ntasks * (int64_t)sizeof(DTask);
    *qalloc = (*qbytes + 255) / 256 * 256;
    *calloc_ = ((int64_t)nctr * 4 + 255) / 256 * 256;
    *total = *qalloc + *calloc_ + B.part_bytes;
}

lt_status batch_flush(Ctx *ctx) {
    Batch &B = ctx->batch;
    if (B.q.empty() || B.capture) return LT_OK;
    lt_status st = flush_group(ctx);
    if (st) return st;
    st = batch_issue(ctx);
    if (st) {
        // the queued tasks are in the DAG but will never run: every later
        // result could be wrong, so the failure is sticky until lt_sync
        if (ctx->sticky == LT_OK) {
            ctx->sticky = st;
            ctx->sticky_msg = "a batch could not be issued: " + ctx->err;
        }
        batch_drop(ctx);
    }
    return st;
}

// Issues the open batch from the fixed device scratch instead of an arena
// range, with no allocation: no arena range (so no eviction), no pinned
// staging buffer (the queue is uploaded from the planner's own host copy)
// and no new status slot (when the preallocated slots are used up, the drain
// stream is synchronized and their flags folded first).  A batch too large
// for the scratch is left open and unissued (LT_ERR_BUDGET).
lt_status batch_flush_noalloc(Ctx *ctx) {
    Batch &B = ctx->batch;
    if (B.capture) return set_err(ctx, LT_ERR_INVALID, "a graph is being recorded");
    if (B.q.empty()) return LT_OK;
    int64_t qbytes, qalloc, calloc_, total;
    batch_layout(B, &qbytes, &qalloc, &calloc_, &total);
    if (total > NOALLOC_SCRATCH_BYTES)
        return set_err(ctx, LT_ERR_BUDGET,
                       "the batch needs %lld bytes of device scratch (%d tasks, %lld bytes of partials); "
                       "the no-allocation issue holds at most %lld: issue it with lt_batch_end",
                       (long long)total, (int)B.q.size(), (long long)B.part_bytes,
                       (long long)NOALLOC_SCRATCH_BYTES);
    if (ctx->dry) return set_err(ctx, LT_ERR_UNSUPPORTED, "the no-allocation batch issue needs a device");
    if (!ctx->scratch)
        return set_err(ctx, LT_ERR_DEVICE, "device scratch lookup failed at context creation: %s",
                       hipGetErrorString(ctx->scratch_err));
    lt_status st = flush_group(ctx);
    if (st) return st;
    st = batch_issue(ctx, true);
    if (st) {
        if (ctx->sticky == LT_OK) {
            ctx->sticky = st;
            ctx->sticky_msg = "a batch could not be issued: " + ctx->err;
        }
        batch_drop(ctx);
    }
    return st;
}

// Folds the drain error flags copied back so far into the sticky error
// (every status copy is on compute stream 0, which must have completed).
void fold_drain_status(Ctx *ctx) {
    for (int i = 0; i < ctx->status_next; ++i)
        if (ctx->status_host[i] && ctx->sticky == LT_OK) {
            ctx->sticky = LT_ERR_TIMEOUT;
            ctx->sticky_msg = "a dependency wait inside the batch drain exceeded its poll limit";
        }
    ctx->status_next = 0;
}

// Uploads the queue of the open batch and issues its drain.  The queue,
// counters and partials take one arena range; the batch's chunks are pinned,
// so making room for it never evicts them (LT_ERR_BUDGET when it cannot fit).
// With `noalloc` they take the fixed device scratch instead.
static lt_status batch_issue(Ctx *ctx, bool noalloc) {
    Batch &B = ctx->batch;
    lt_status st;
    const int ntasks = (int)B.q.size();
    int64_t qbytes, qalloc, calloc_, total;
    batch_layout(B, &qbytes, &qalloc, &calloc_, &total);
    int64_t off = -1;
    Fence mem;
    char *base;
    if (noalloc) {
        base = static_cast<char *>(ctx->scratch);
        // the previous user of the scratch on this context is a drain on
        // compute stream 0, where this batch is issued too
    } else {
        st = alloc_range(ctx, total, 2, nullptr, &off, &mem);
        if (st) return st;
        base = ctx->arena_base + off;
    }
    int64_t part_base = (int64_t)(intptr_t)(base + qalloc + calloc_);
    for (auto &pr : B.patch_y) B.q[pr.first].y += part_base;
    for (auto &pr : B.patch_x) B.q[pr.first].x += part_base;
    for (DTask &d : B.q) {
        if (d.signal <= -2) d.signal = ntasks + (-2 - d.signal);
        for (int i = 0; i < d.ndeps; ++i)
            if (d.dep_ctr[i] <= -2) d.dep_ctr[i] = ntasks + (-2 - d.dep_ctr[i]);
    }
    const void *stage = B.q.data();
    if (!noalloc) {
        void *p = staging_get(ctx, (uint64_t)qbytes, &st);
        if (!p) {
            ctx->arena.release(off, mem);
            return st;
        }
        memcpy(p, B.q.data(), (size_t)qbytes);
        stage = p;
    }
    const int s = 0;
    B.wait.merge(mem);
    st = stream_wait(ctx, s, B.wait);
    if (st) return st;
    int nwg = ctx->cfg.drain_workgroups > 0 ? ctx->cfg.drain_workgroups : 1024;
    if (!ctx->dry) {
        hipStream_t h = ctx->streams[s].h;
        // from pageable memory (no-allocation issue) the copy has read its
        // source when the call returns, so the queue can be dropped below
        hipError_t r = hipMemcpyAsync(base, stage, (size_t)qbytes, hipMemcpyHostToDevice, h);
        if (r != hipSuccess) return hip_fail(ctx, r, "batch queue upload");
        uint32_t zero = 0;
        r = launch_fill(h, base + qalloc, (calloc_ + B.part_bytes) / 4, 4, &zero);
        if (r != hipSuccess) return hip_fail(ctx, r, "batch clear");
        hipEvent_t pa;
        st = prof_begin(ctx, s, "drain", &pa);
        if (st) return st;
        r = launch_drain(h, reinterpret_cast<const DTask *>(base), ntasks,
                         reinterpret_cast<int32_t *>(base + qalloc), ntasks + B.nsignals, B.tiles, nwg,
                         (int64_t)1 << 26, B.kinds, ctx->cfg.drain_vectors);
        if (r != hipSuccess) return hip_fail(ctx, r, "drain");
        st = prof_end(ctx, s, "drain", pa);
        if (st) return st;
        // error flag back to pinned host memory, checked at lt_sync
        if (noalloc && ctx->status_next >= ctx->status_slots) {
            // every slot's copy is on this stream: wait for them and reuse
            r = hipStreamSynchronize(h);
            if (r != hipSuccess) return hip_fail(ctx, r, "hipStreamSynchronize");
            fold_drain_status(ctx);
        }
        if (ctx->status_next >= ctx->status_slots) {
            int ns = std::max(64, ctx->status_slots * 2);
            int32_t *p = nullptr;
            r = hipHostMalloc((void **)&p, (size_t)ns * 4, hipHostMallocDefault);
            if (r != hipSuccess) return hip_fail(ctx, r, "status buffer");
            if (ctx->status_host) {
                // earlier slots are still pending; keep the old buffer alive
                r = hipStreamSynchronize(h);
                if (r != hipSuccess) return hip_fail(ctx, r, "hipStreamSynchronize");
                memcpy(p, ctx->status_host, (size_t)ctx->status_slots * 4);
                (void)hipHostFree(ctx->status_host);
            }
            ctx->status_host = p;
            ctx->status_slots = ns;
        }
        int slot = ctx->status_next++;
        r = hipMemcpyAsync(ctx->status_host + slot, base + qalloc + (int64_t)(ntasks + B.nsignals + 1) * 4, 4,
                           hipMemcpyDeviceToHost, h);
        if (r != hipSuccess) return hip_fail(ctx, r, "drain status copy");
    }
    ctx->stats.dispatches += 2;
    trace_op(ctx, 0, s, ~0ull, 0, (uint64_t)ntasks, 0);
    uint64_t p = bump(ctx, s);
    for (uint64_t id : B.ids) {
        TaskRec &r = ctx->tasks.at(id);
        r.stream = s;
        r.seq = p;
    }
    apply_uses(ctx, B.uses, s, p);
    Fence done;
    done.add(s, p);
    if (off >= 0) ctx->arena.release(off, done);
    for (uint64_t L : B.launches) ctx->launches.at(L).done.add(s, p);  // they complete with the drain
    batch_drop(ctx);
    return LT_OK;
}

// Builds a HIP graph from the captured batch: queue upload, counter clear,
// drain and error-flag copy, recorded on compute stream 0.
lt_status graph_end(Ctx *ctx, lt_graph **out) {
    Batch &B = ctx->batch;
    if (!B.capture) return set_err(ctx, LT_ERR_INVALID, "no graph is being recorded");
    if (B.q.empty()) return set_err(ctx, LT_ERR_INVALID, "the graph has no tasks");
    if (ctx->dry) return set_err(ctx, LT_ERR_UNSUPPORTED, "graphs need a device");
    const int ntasks = (int)B.q.size();
    const int nctr = ntasks + B.nsignals + 2;
    const int64_t qbytes = (int64_t)ntasks * (int64_t)sizeof(DTask);
    const int64_t qalloc = (qbytes + 255) / 256 * 256;
    const int64_t calloc_ = ((int64_t)nctr * 4 + 255) / 256 * 256;
    const int64_t total = qalloc + calloc_ + B.part_bytes;
    auto g = std::make_unique<lt_graph>();
    Fence mem;
    lt_status st = alloc_range(ctx, total, 2, nullptr, &g->off, &mem);
    if (st) return st;
    char *base = ctx->arena_base + g->off;
    int64_t part_base = (int64_t)(intptr_t)(base + qalloc + calloc_);
    for (auto &pr : B.patch_y) B.q[pr.first].y += part_base;
    for (auto &pr : B.patch_x) B.q[pr.first].x += part_base;
    for (DTask &d : B.q) {
        if (d.signal <= -2) d.signal = ntasks + (-2 - d.signal);
        for (int i = 0; i < d.ndeps; ++i)
            if (d.dep_ctr[i] <= -2) d.dep_ctr[i] = ntasks + (-2 - d.dep_ctr[i]);
    }
    // on failure below, the arena range and host buffers go back
    auto undo = [&]() {
        ctx->arena.release(g->off, mem);
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        if (g->staging) (void)hipHostFree(g->staging);
        if (g->status) (void)hipHostFree(g->status);
    };
    hipError_t r = hipHostMalloc(&g->staging, (size_t)qbytes, hipHostMallocDefault);
    if (r != hipSuccess) {
        g->staging = nullptr;
        undo();
        return hip_fail(ctx, r, "graph staging");
    }
    r = hipHostMalloc((void **)&g->status, 4, hipHostMallocDefault);
    if (r != hipSuccess) {
        g->status = nullptr;
        undo();
        return hip_fail(ctx, r, "graph status");
    }
    *g->status = 0;
    memcpy(g->staging, B.q.data(), (size_t)qbytes);
    const int s = 0;
    g->stream = s;
    st = stream_wait(ctx, s, mem);
    if (st) {
        undo();
        return st;
    }
    hipStream_t h = ctx->streams[s].h;
    int nwg = ctx->cfg.drain_workgroups > 0 ? ctx->cfg.drain_workgroups : 1024;
    r = hipStreamBeginCapture(h, hipStreamCaptureModeThreadLocal);
    if (r != hipSuccess) {
        undo();
        return hip_fail(ctx, r, "hipStreamBeginCapture");
    }
    hipError_t r1 = hipMemcpyAsync(base, g->staging, (size_t)qbytes, hipMemcpyHostToDevice, h);
    uint32_t zero = 0;
    hipError_t r2 = launch_fill(h, base + qalloc, (calloc_ + B.part_bytes) / 4, 4, &zero);
    hipError_t r3 = launch_drain(h, reinterpret_cast<const DTask *>(base), ntasks,
                                 reinterpret_cast<int32_t *>(base + qalloc), ntasks + B.nsignals, B.tiles, nwg,
                                 (int64_t)1 << 26, B.kinds, ctx->cfg.drain_vectors);
    hipError_t r4 = hipMemcpyAsync(g->status, base + qalloc + (int64_t)(ntasks + B.nsignals + 1) * 4, 4,
                                   hipMemcpyDeviceToHost, h);
    r = hipStreamEndCapture(h, &g->graph);
    if (r1 != hipSuccess || r2 != hipSuccess || r3 != hipSuccess || r4 != hipSuccess || r != hipSuccess) {
        undo();
        return hip_fail(ctx, r != hipSuccess ? r : (r1 != hipSuccess ? r1 : (r2 != hipSuccess ? r2 : (r3 != hipSuccess ? r3 : r4))),
                        "graph capture");
    }
    r = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (r != hipSuccess) {
        g->exec = nullptr;
        undo();
        return hip_fail(ctx, r, "hipGraphInstantiate");
    }
    // chunks the graph touches stay where they are while it lives; the
    // capture recorded no work, so their histories go back to empty
    for (const ChunkUse &u : B.uses) {
        auto it = std::find(g->chunks.begin(), g->chunks.end(), u.c);
        if (it == g->chunks.end()) {
            g->chunks.push_back(u.c);
            g->writes.push_back(u.write);
            u.c->pin++;
        } else if (u.write) {
            g->writes[it - g->chunks.begin()] = 1;
        }
    }
    for (Chunk *c : g->chunks) {
        c->last_writer = 0;
        c->readers.clear();
        c->reducers.clear();
        c->reduce_op = -1;
    }
    g->ntasks = ntasks;
    ctx->graph_status.push_back(g->status);
    batch_drop(ctx);  // the graph holds its own pins
    ctx->batch.open = false;
    *out = g.release();
    return LT_OK;
}

lt_status graph_launch(Ctx *ctx, lt_graph *g) {
    lt_status st = flush_all(ctx);
    if (st) return st;
    TaskRec rec;
    rec.id = ctx->next_task_id++;
    rec.kind = LT_TASK_EXEC;
    Fence wait;
    for (size_t i = 0; i < g->chunks.size(); ++i) {
        Chunk *c = g->chunks[i];
        conflict_edges(c, g->writes[i] ? M_WRITE : M_READ, R_ADD, &rec.deps);
        wait.merge(c->data_ready);
        if (g->writes[i]) wait.merge(c->last_access);
    }
    wait.merge(task_fence(ctx, rec.deps));
    st = stream_wait(ctx, g->stream, wait);
    if (st) return st;
    hipEvent_t pa;
    st = prof_begin(ctx, g->stream, "graph", &pa);
    if (st) return st;
    hipError_t r = hipGraphLaunch(g->exec, ctx->streams[g->stream].h);
    if (r != hipSuccess) return hip_fail(ctx, r, "hipGraphLaunch");
    st = prof_end(ctx, g->stream, "graph", pa);
    if (st) return st;
    ctx->stats.dispatches++;
    uint64_t p = bump(ctx, g->stream);
    g->last = p;
    std::vector<ChunkUse> uses;
    for (size_t i = 0; i < g->chunks.size(); ++i) {
        record_access(g->chunks[i], g->writes[i] ? M_WRITE : M_READ, R_ADD, rec.id);
        uses.push_back({g->chunks[i], g->writes[i] != 0});
    }
    apply_uses(ctx, uses, g->stream, p);
    rec.stream = g->stream;
    rec.seq = p;
    ctx->tasks.at(rec.id) = std::move(rec);
    return LT_OK;
}

lt_status graph_destroy(Ctx *ctx, lt_graph *g) {
    lt_status st = flush_all(ctx);
    if (st) return st;
    if (!ctx->dry) {
        hipError_t r = hipStreamSynchronize(ctx->streams[g->stream].h);
        if (r != hipSuccess) st = hip_fail(ctx, r, "hipStreamSynchronize");
        if (*g->status && ctx->sticky == LT_OK) {
            ctx->sticky = LT_ERR_TIMEOUT;
            ctx->sticky_msg = "a dependency wait inside a graph's drain exceeded its poll limit";
        }
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        if (g->staging) (void)hipHostFree(g->staging);
    }
    for (Chunk *c : g->chunks) c->pin--;
    Fence done;
    done.add(g->stream, g->last);
    ctx->arena.release(g->off, done);
    auto it = std::find(ctx->graph_status.begin(), ctx->graph_status.end(), g->status);
    if (it != ctx->graph_status.end()) ctx->graph_status.erase(it);
    if (!ctx->dry && g->status) (void)hipHostFree(g->status);
    delete g;
    return st;
}

lt_status flush_all(Ctx *ctx) {
    lt_status st = flush_group(ctx);
    if (st) return st;
    return batch_flush(ctx);
}

static lt_status issue_exec(Ctx *ctx, lt_kernel *k, TaskPlan &tp, uint64_t L,
                            const KLaunch &proto, Array **arrs, std::vector<Partials> &parts,
                            int nd) {
    const KernelDef *def = k->def;
    Group &g = group_of(ctx);
    TaskRec rec;
    rec.id = tp.id;
    rec.launch = L;
    rec.kind = LT_TASK_EXEC;
    rec.sb = tp.sb;

    // conflict analysis
    bool has_reduce = false;
    for (int p = 0; p < def->nparam; ++p) {
        ArgPlan &a = tp.arg[p];
        if (!a.used) continue;
        if (a.mode == M_REDUCE) {
            has_reduce = true;
            continue;  // the combine task accesses the target
        }
        for (Chunk *c : a.chunks) conflict_edges(c, a.mode, a.op, &rec.deps);
        for (Chunk *k : a.halo_owners) conflict_edges(k, M_READ, a.op, &rec.deps);
    }

    if (ctx->batch.open) return batch_add_exec(ctx, def, tp, rec, proto, arrs, parts);

    // can this task join the open group without staging or copies?
    bool simple = !has_reduce;
    KTask kt;
    memset(&kt, 0, sizeof kt);
    for (int a = 0; a < MAXD; ++a) {
        kt.lo[a] = tp.sb.lo[a];
        kt.hi[a] = tp.sb.hi[a];
    }
    if (simple)
        for (int p = 0; p < def->nparam && simple; ++p) {
            ArgPlan &a = tp.arg[p];
            if (!a.used) continue;
            if (!direct_view(ctx, arrs[p], a.chunks, &kt.v[p])) simple = false;
            // halo replicas to refresh first: take the staging path
            if (a.mode != M_WRITE)
                for (Chunk *c : a.chunks)
                    if (halo_stale(c, a.region)) simple = false;
        }
    bool in_group = false;
    if (simple && ctx->cfg.exec_mode == LT_EXEC_GROUPED && g.open && g.launch == L && g.def == def) {
        in_group = true;
        for (uint64_t d : rec.deps)
            if (std::find(g.ids.begin(), g.ids.end(), d) != g.ids.end()) in_group = false;
    }
    lt_status st;
    if (!in_group) {
        st = flush_group(ctx);
        if (st) return st;
    }

    if (simple) {
        Fence wait = task_fence(ctx, rec.deps);
        std::vector<ChunkUse> uses;
        for (int p = 0; p < def->nparam; ++p) {
            ArgPlan &a = tp.arg[p];
            if (!a.used) continue;
            for (Chunk *c : a.chunks) {
                wait.merge(c->data_ready);
                if (a.mode != M_READ) wait.merge(c->last_access);
                c->lru = ++ctx->lru_clock;
                uses.push_back({c, a.mode != M_READ});
            }
            rec.regions.push_back(lt_region_info{p, (int)a.mode, (int)a.op, 0, arrs[p]->id,
                                                 {a.region.lo[0], a.region.lo[1], a.region.lo[2]},
                                                 {a.region.hi[0], a.region.hi[1], a.region.hi[2]}});
            ctx->stats.direct_regions++;
            for (Chunk *c : a.chunks) record_access(c, a.mode, a.op, tp.id);
        for (Chunk *k : a.halo_owners) record_access(k, M_READ, a.op, tp.id);
        }
        if (!g.open) {
            g.open = true;
            g.launch = L;
            g.def = def;
            g.stream = pick_stream(ctx, wait);
            g.proto = proto;
            g.wait = Fence();
        }
        g.wait.merge(wait);
        g.tasks.push_back(kt);
        g.ids.push_back(tp.id);
        g.uses.insert(g.uses.end(), uses.begin(), uses.end());
        ctx->tasks.at(tp.id) = std::move(rec);
        if (ctx->cfg.exec_mode != LT_EXEC_GROUPED || (int)g.tasks.size() >= std::min(def->max_group, KMAXG))
            return flush_group(ctx);
        return LT_OK;
    }

    // ---- general path: staging, temporaries, partials
    Fence wait = task_fence(ctx, rec.deps);
    std::vector<Chunk *> pinned;
    for (int p = 0; p < def->nparam; ++p)
        for (Chunk *c : tp.arg[p].chunks) {
            c->pin++;
            pinned.push_back(c);
        }
    auto unpin = [&]() {
        for (Chunk *c : pinned) c->pin--;
    };
    bool staged_copy = false;
    std::vector<ChunkUse> uses;
    // runs of neighbouring chunks that must sit contiguously go first, while
    // the arena has the most room for them; single chunks fit any gap
    for (int pass = 0; pass < 2; ++pass)
        for (int p = 0; p < def->nparam; ++p) {
            ArgPlan &a = tp.arg[p];
            if (!a.used || a.mode == M_REDUCE) continue;
            const bool run = a.chunks.size() > 1 && arrs[p]->row_slab;
            if (run != (pass == 0)) continue;
            Fence placed;
            if (run) {
                st = place_run(ctx, a.chunks, &placed);
                if (st) {
                    unpin();
                    return st;
                }
            }
            for (Chunk *c : a.chunks) {
                st = stage_chunk(ctx, c, a.mode, a.region, &wait, &staged_copy, tp.footprint, placed);
                if (st) {
                    unpin();
                    return st;
                }
                uses.push_back({c, a.mode != M_READ});
            }
        }
    // views: direct, assembled temporaries, partials
    std::vector<Temp> temps;
    for (int p = 0; p < def->nparam; ++p) {
        ArgPlan &a = tp.arg[p];
        if (!a.used) continue;
        Array *arr = arrs[p];
        int resolved = 0;
        if (a.mode == M_REDUCE) {
            Partials *P = nullptr;
            for (auto &x : parts)
                if (x.param == p) P = &x;
            // this superblock's partial
            CombinePart cp;
            cp.off = P->cursor;
            cp.count = tp.slots;
            P->cursor += a.region.volume(arr->ndim) * tp.slots;
            kt.slot[p] = tp.slots > 1 ? a.region.volume(arr->ndim) : 0;
            for (int d = 0; d < KMAXD; ++d) {
                cp.lo[d] = a.region.lo[d];
                cp.hi[d] = a.region.hi[d];
            }
            int64_t st_[MAXD];
            int64_t s = 1;
            for (int d = MAXD - 1; d >= 0; --d) {
                st_[d] = s;
                s *= d < arr->ndim ? a.region.hi[d] - a.region.lo[d] : 1;
            }
            kt.v[p] = make_view(ctx->arena_base + P->off + cp.off * arr->esz, a.region.lo, st_, arr->ndim, arr->esz);
            P->parts.push_back(cp);
            P->producers.push_back(tp.id);
            wait.merge(P->ready);
            resolved = 2;
        } else if (direct_view(ctx, arr, a.chunks, &kt.v[p])) {
            resolved = 0;
            ctx->stats.direct_regions++;
        } else {
            Temp t;
            t.param = p;
            t.region = a.region;
            t.chunks = a.chunks;
            t.scatter = a.mode != M_READ;
            int64_t s = 1;
            for (int d = MAXD - 1; d >= 0; --d) {
                t.stride[d] = s;
                s *= d < arr->ndim ? a.region.hi[d] - a.region.lo[d] : 1;
            }
            Fence mem;
            st = alloc_range(ctx, (a.region.volume(arr->ndim) * arr->esz + 255) / 256 * 256, 2, nullptr,
                             &t.off, &mem);
            if (st) {
                unpin();
                return st;
            }
            wait.merge(mem);
            kt.v[p] = make_view(ctx->arena_base + t.off, a.region.lo, t.stride, arr->ndim, arr->esz);
            temps.push_back(t);
            resolved = 1;
            ctx->stats.assembled_regions++;
        }
        rec.regions.push_back(lt_region_info{p, (int)a.mode, (int)a.op, resolved, arr->id,
                                             {a.region.lo[0], a.region.lo[1], a.region.lo[2]},
                                             {a.region.hi[0], a.region.hi[1], a.region.hi[2]}});
    }
    int s = pick_stream(ctx, wait);
    st = stream_wait(ctx, s, wait);
    if (st) {
        unpin();
        return st;
    }
    // assemble (also for writes: write-allocate)
    for (Temp &t : temps) {
        Array *arr = arrs[t.param];
        for (Chunk *c : t.chunks) {
            st = copy_region(ctx, s, c, t, arr->esz, arr->ndim, true);
            if (st) {
                unpin();
                return st;
            }
        }
        if (!t.chunks.empty()) bump(ctx, s);
    }
    KLaunch kl = proto;
    kl.ntask = 1;
    kl.tasks = &kt;
    st = dispatch(ctx, def, kl, s);
    if (st) {
        unpin();
        return st;
    }
    bump(ctx, s);
    for (Temp &t : temps) {
        if (!t.scatter) continue;
        Array *arr = arrs[t.param];
        for (Chunk *c : t.chunks) {
            st = copy_region(ctx, s, c, t, arr->esz, arr->ndim, false);
            if (st) {
                unpin();
                return st;
            }
        }
        bump(ctx, s);
    }
    uint64_t pt = ctx->streams[s].seq;
    rec.stream = s;
    rec.seq = pt;
    for (int p = 0; p < def->nparam; ++p) {
        ArgPlan &a = tp.arg[p];
        if (!a.used || a.mode == M_REDUCE) continue;
        for (Chunk *c : a.chunks) record_access(c, a.mode, a.op, tp.id);
        for (Chunk *k : a.halo_owners) record_access(k, M_READ, a.op, tp.id);
    }
    apply_uses(ctx, uses, s, pt);
    Fence done;
    done.add(s, pt);
    for (Temp &t : temps) ctx->arena.release(t.off, done);
    // Mark this task's end now, while it is the stream's last operation, when
    // the copy streams will wait for it: the throttle waits for staged tasks,
    // and once the budget binds, write-backs and reloads wait for the last
    // users of the chunks they evict.  A mark taken later would also cover
    // every task issued since (the host runs ahead of the device).
    if (staged_copy || ctx->budget_binds) {
        st = mark_tail(ctx, s);
        if (st) {
            unpin();
            return st;
        }
    }
    if (staged_copy) {
        ctx->staged.push_back({done, tp.footprint});
        ctx->staged_bytes += tp.footprint;
        ctx->stats.staged_peak_bytes = std::max<uint64_t>(ctx->stats.staged_peak_bytes, ctx->staged_bytes);
    }
    unpin();
    ctx->tasks.at(tp.id) = std::move(rec);
    return LT_OK;
}

// One combine task per reduce argument of a launch: the target region (the
// union of the partial boxes) is overwritten by the fold of the partials.
static lt_status issue_combine(Ctx *ctx, Partials &P, Array *arr, uint64_t L) {
    const int nd = arr->ndim;
    if (P.parts.empty()) return LT_OK;
    if (P.batched) return batch_add_combine(ctx, P, arr, L);
    Box U;
    for (int a = 0; a < MAXD; ++a) {
        U.lo[a] = P.parts[0].lo[a];
        U.hi[a] = P.parts[0].hi[a];
    }
    for (auto &q : P.parts) {
        Box b;
        for (int a = 0; a < MAXD; ++a) {
            b.lo[a] = q.lo[a];
            b.hi[a] = q.hi[a];
        }
        U = bbox_union(U, b, nd);
    }
    TaskRec rec;
    rec.id = ctx->next_task_id++;
    rec.launch = L;
    rec.kind = LT_TASK_COMBINE;
    rec.sb = U;
    std::vector<Chunk *> ch;
    chunks_overlapping(arr, U, &ch);
    for (uint64_t pid : P.producers) add_dep(&rec.deps, pid);
    for (Chunk *c : ch) conflict_edges(c, M_WRITE, R_ADD, &rec.deps);
    lt_status st = flush_group(ctx);
    if (st) return st;
    Fence wait = task_fence(ctx, rec.deps);
    for (Chunk *c : ch) c->pin++;
    bool staged_copy = false;
    std::vector<ChunkUse> uses;
    Fence placed;
    if (ch.size() > 1 && arr->row_slab) {
        st = place_run(ctx, ch, &placed);
        if (st) {
            for (Chunk *x : ch) x->pin--;
            return st;
        }
    }
    for (Chunk *c : ch) {
        st = stage_chunk(ctx, c, M_WRITE, U, &wait, &staged_copy, 0, placed);
        if (st) {
            for (Chunk *x : ch) x->pin--;
            return st;
        }
        uses.push_back({c, true});
    }
    KView tv;
    Temp t;
    bool tmp = false;
    if (!direct_view(ctx, arr, ch, &tv)) {
        tmp = true;
        t.param = 0;
        t.region = U;
        t.chunks = ch;
        t.scatter = true;
        int64_t s = 1;
        for (int d = MAXD - 1; d >= 0; --d) {
            t.stride[d] = s;
            s *= d < nd ? U.hi[d] - U.lo[d] : 1;
        }
        Fence mem;
        st = alloc_range(ctx, (U.volume(nd) * arr->esz + 255) / 256 * 256, 2, nullptr, &t.off, &mem);
        if (st) {
            for (Chunk *x : ch) x->pin--;
            return st;
        }
        wait.merge(mem);
        tv = make_view(ctx->arena_base + t.off, U.lo, t.stride, nd, arr->esz);
        ctx->stats.assembled_regions++;
    }
    int s = pick_stream(ctx, wait);
    st = stream_wait(ctx, s, wait);
    if (!st && tmp) {
        for (Chunk *c : ch)
            if (!st) st = copy_region(ctx, s, c, t, arr->esz, nd, true);
        bump(ctx, s);
    }
    bool slotted = false;
    for (auto &q : P.parts) slotted |= q.count > 1;
    for (size_t i = 0; slotted && i < P.parts.size() && !st; i += KMAXPART) {
        // first level: the slots of each superblock's partial, in slot order
        CombineArgs ca;
        memset(&ca, 0, sizeof ca);
        ca.ndim = nd;
        ca.dtype = arr->dtype;
        ca.op = P.op;
        ca.part_base = (int64_t)(intptr_t)(ctx->arena_base + P.off);
        ca.nparts = (int)std::min<size_t>(KMAXPART, P.parts.size() - i);
        for (int j = 0; j < ca.nparts; ++j) ca.parts[j] = P.parts[i + j];
        ctx->stats.dispatches++;
        trace_op(ctx, 0, s, rec.id, 0, ca.nparts, 1);
        if (!ctx->dry) {
            hipError_t r = launch_fold_slots(ctx->streams[s].h, ca);
            if (r != hipSuccess) st = hip_fail(ctx, r, "fold slots");
        }
        bump(ctx, s);
    }
    for (size_t i = 0; i < P.parts.size() && !st; i += KMAXPART) {
        CombineArgs ca;
        memset(&ca, 0, sizeof ca);
        ca.ndim = nd;
        ca.dtype = arr->dtype;
        ca.op = P.op;
        ca.accumulate = i > 0;
        for (int a = 0; a < KMAXD; ++a) {
            ca.lo[a] = a < nd ? U.lo[a] : 0;
            ca.hi[a] = a < nd ? U.hi[a] : 1;
        }
        ca.target = tv;
        ca.part_base = (int64_t)(intptr_t)(ctx->arena_base + P.off);
        ca.nparts = (int)std::min<size_t>(KMAXPART, P.parts.size() - i);
        for (int j = 0; j < ca.nparts; ++j) ca.parts[j] = P.parts[i + j];
        ctx->stats.dispatches++;
        trace_op(ctx, 0, s, rec.id, 0, ca.nparts, 0);
        if (!ctx->dry) {
            hipError_t r = launch_combine(ctx->streams[s].h, ca);
            if (r != hipSuccess) st = hip_fail(ctx, r, "combine");
        }
        bump(ctx, s);
    }
    if (!st && tmp) {
        for (Chunk *c : ch)
            if (!st) st = copy_region(ctx, s, c, t, arr->esz, nd, false);
        bump(ctx, s);
    }
    for (Chunk *x : ch) x->pin--;
    if (st) return st;
    uint64_t pt = ctx->streams[s].seq;
    rec.stream = s;
    rec.seq = pt;
    for (Chunk *c : ch) record_access(c, M_WRITE, R_ADD, rec.id);
    apply_uses(ctx, uses, s, pt);
    Fence done;
    done.add(s, pt);
    if (tmp) ctx->arena.release(t.off, done);
    ctx->arena.release(P.off, done);
    rec.regions.push_back(lt_region_info{P.param, (int)M_REDUCE, (int)P.op, tmp ? 1 : 0, arr->id,
                                         {U.lo[0], U.lo[1], U.lo[2]}, {U.hi[0], U.hi[1], U.hi[2]}});
    ctx->launches.at(L).tasks.push_back(rec.id);
    ctx->tasks.at(rec.id) = std::move(rec);
    return LT_OK;
}

lt_status launch(Ctx *ctx, lt_kernel *k, int nd, const int64_t *grid,
                 const int64_t *block, const int64_t *sb, const char *annotation,
                 const lt_arg *args, int nargs, uint64_t *launch_id) {
    double t0 = now_s();
    if (!k || !k->def) return set_err(ctx, LT_ERR_INVALID, "NULL kernel");
    const KernelDef *def = k->def;
    if (ctx->sticky != LT_OK)
        return set_err(ctx, ctx->sticky, "earlier asynchronous error: %s", ctx->sticky_msg.c_str());
    std::shared_ptr<Annotation> an = k->annot;
    if (annotation) {
        lt_status st = compile_annotation(ctx, def, annotation, &an);
        if (st) return st;
    }
    // bind arguments
    if (nargs != def->nparam)
        return set_err(ctx, LT_ERR_INVALID, "%s takes %d arguments, got %d", def->name, def->nparam, nargs);
    Array *arrs[MAXPARAM] = {nullptr};
    int64_t iparams[MAXPARAM] = {0};
    double fparams[MAXPARAM] = {0};
    bool bound[MAXPARAM] = {false};
    for (int i = 0; i < nargs; ++i) {
        int p = i;
        if (args[i].name) {
            p = -1;
            for (int q = 0; q < def->nparam; ++q)
                if (!strcmp(args[i].name, def->params[q].name)) p = q;
            if (p < 0) return set_err(ctx, LT_ERR_INVALID, "%s has no parameter '%s'", def->name, args[i].name);
        }
        if (bound[p]) return set_err(ctx, LT_ERR_INVALID, "parameter '%s' given twice", def->params[p].name);
        bound[p] = true;
        const ParamDef &pd = def->params[p];
        if (pd.kind == P_ARRAY) {
            if (args[i].kind != LT_ARG_ARRAY || !args[i].array)
                return set_err(ctx, LT_ERR_INVALID, "parameter '%s' must be an array", pd.name);
            Array *a = args[i].array;
            if (a->dead) return set_err(ctx, LT_ERR_INVALID, "array for '%s' was destroyed", pd.name);
            if (a->dtype != pd.dtype || a->ndim != pd.ndim)
                return set_err(ctx, LT_ERR_INVALID, "array for '%s' has the wrong dtype or rank", pd.name);
            arrs[p] = a;
        } else if (pd.kind == P_INT) {
            if (args[i].kind != LT_ARG_INT)
                return set_err(ctx, LT_ERR_INVALID, "parameter '%s' must be an integer", pd.name);
            iparams[p] = args[i].i;
        } else {
            if (args[i].kind == LT_ARG_FLOAT) fparams[p] = args[i].f;
            else if (args[i].kind == LT_ARG_INT) fparams[p] = (double)args[i].i;
            else return set_err(ctx, LT_ERR_INVALID, "parameter '%s' must be a number", pd.name);
        }
    }
    if (nd != def->grid_ndim)
        return set_err(ctx, LT_ERR_INVALID, "%s needs a %d-D grid, got %d-D", def->name, def->grid_ndim, nd);
    for (int kd = 0; kd < 3; ++kd)
        if (an->nbound[kd] >= 0 && an->nbound[kd] != nd)
            return set_err(ctx, LT_ERR_PARSE, "annotation binds %d axes but the grid has %d", an->nbound[kd], nd);
    int64_t G[MAXD] = {1, 1, 1}, S[MAXD] = {1, 1, 1}, B[MAXD] = {1, 1, 1}, nsb[MAXD] = {1, 1, 1};
    int64_t total = 1;
    for (int a = 0; a < nd; ++a) {
        if (!grid || !block) return set_err(ctx, LT_ERR_INVALID, "grid and block are required");
        if (grid[a] < 0 || block[a] < 1)
            return set_err(ctx, LT_ERR_INVALID, "axis %d: grid must be >= 0 and block >= 1", a);
        B[a] = block[a];
        G[a] = (grid[a] + B[a] - 1) / B[a] * B[a];
        int64_t s = sb ? sb[a] : 0;
        if (s < 0 || (s > 0 && s % B[a] != 0))
            return set_err(ctx, LT_ERR_INVALID, "axis %d: superblock %lld is not a multiple of block %lld", a,
                           (long long)s, (long long)B[a]);
        S[a] = (s == 0 || s > G[a]) ? G[a] : s;
        nsb[a] = S[a] > 0 ? (G[a] + S[a] - 1) / S[a] : 0;
        total *= nsb[a];
    }
    if (total > ((int64_t)1 << 22)) return set_err(ctx, LT_ERR_INVALID, "too many superblocks (%lld)", (long long)total);
    if (def->user && B[0] * B[1] * B[2] > 1024)
        return set_err(ctx, LT_ERR_INVALID, "%s: a block of %lld threads is more than 1024", def->name,
                       (long long)(B[0] * B[1] * B[2]));
    // combined access per array parameter
    Mode pmode[MAXPARAM];
    ROp pop[MAXPARAM];
    bool pany[MAXPARAM] = {false};
    for (auto &ac : an->acc) {
        int p = ac.param;
        if (!pany[p]) {
            pmode[p] = ac.mode;
            pop[p] = ac.op;
            pany[p] = true;
        } else if (pmode[p] == M_REDUCE || ac.mode == M_REDUCE) {
            if (pmode[p] != ac.mode || pop[p] != ac.op)
                return set_err(ctx, LT_ERR_PARSE, "array '%s' mixes reductions", def->params[p].name);
        } else if (pmode[p] != ac.mode) {
            pmode[p] = M_RW;
        }
    }
    // plan every superblock
    std::vector<TaskPlan> plans;
    plans.reserve((size_t)total);
    int64_t idx[MAXD] = {0, 0, 0};
    std::vector<Chunk *> seen;
    for (int64_t t = 0; t < total; ++t) {
        sb_index(t, nd, nsb, ctx->cfg.sb_order, ctx->cfg.sb_band, idx);
        TaskPlan tp;
        int64_t blo[MAXD], bhi[MAXD];
        for (int a = 0; a < nd; ++a) {
            tp.sb.lo[a] = idx[a] * S[a];
            tp.sb.hi[a] = std::min(G[a], tp.sb.lo[a] + S[a]);
            blo[a] = tp.sb.lo[a] / B[a];
            bhi[a] = tp.sb.hi[a] / B[a];
        }
        VarRange vr;
        var_ranges(nd, blo, bhi, B, &vr);
        for (auto &ac : an->acc) {
            int p = ac.param;
            Box rg;
            if (!access_region(ac, nd, B, vr, iparams, arrs[p], &rg)) continue;
            ArgPlan &a = tp.arg[p];
            a.region = a.used ? bbox_union(a.region, rg, arrs[p]->ndim) : rg;
            a.used = true;
            a.mode = pmode[p];
            a.op = pop[p];
        }
        seen.clear();
        // batched bodies fold into one partial per task
        if (def->slots && !(ctx->batch.open && def->dkind >= 0))
            tp.slots = std::max<int64_t>(1, def->slots(tp.sb.lo, tp.sb.hi, iparams));
        for (int p = 0; p < def->nparam; ++p) {
            ArgPlan &a = tp.arg[p];
            if (!a.used) continue;
            Array *arr = arrs[p];
            if (a.mode == M_REDUCE) {
                tp.footprint += a.region.volume(arr->ndim) * arr->esz * tp.slots;
                continue;
            }
            chunks_overlapping(arr, a.region, &a.chunks);
            if (arr->has_halo && a.mode == M_READ && a.chunks.size() > 1) {
                // a read inside one chunk's stored box is served by that chunk
                if (Chunk *e = enclosing_chunk(arr, a.region)) {
                    for (Chunk *k : a.chunks)
                        if (k != e) a.halo_owners.push_back(k);
                    a.chunks.assign(1, e);
                }
            }
            bool multi = a.chunks.size() > 1;
            for (Chunk *c : a.chunks)
                if (std::find(seen.begin(), seen.end(), c) == seen.end()) {
                    seen.push_back(c);
                    tp.footprint += (c->bytes + 255) / 256 * 256;
                }
            if (multi && !arr->row_slab) tp.footprint += a.region.volume(arr->ndim) * arr->esz + 256;
        }
        plans.push_back(std::move(tp));
    }
    lt_status st;
    if (ctx->batch.open) {
        bool flush = false;
        st = batch_halo_reads(ctx, plans, arrs, def->nparam, &flush);
        if (st) return st;
        if (flush) {
            st = batch_flush(ctx);
            if (st) return st;
        }
    }
    st = ensure_arena(ctx);
    if (st) return st;
    // partial blocks for reduce arguments
    std::vector<Partials> parts;
    int64_t part_bytes = 0;
    for (int p = 0; p < def->nparam; ++p) {
        if (def->params[p].kind != P_ARRAY || !pany[p] || pmode[p] != M_REDUCE) continue;
        Partials P;
        P.param = p;
        P.op = pop[p];
        for (auto &tp : plans)
            if (tp.arg[p].used) P.total_elems += tp.arg[p].region.volume(arrs[p]->ndim) * tp.slots;
        P.bytes = (P.total_elems * arrs[p]->esz + 255) / 256 * 256;
        part_bytes += P.bytes;
        parts.push_back(P);
    }
    for (auto &tp : plans)
        if (tp.footprint + part_bytes > ctx->arena.capacity)
            return set_err(ctx, LT_ERR_BUDGET,
                           "a task of %s needs %lld device bytes; the budget is %lld", def->name,
                           (long long)(tp.footprint + part_bytes), (long long)ctx->arena.capacity);
    uint64_t L = ctx->next_launch_id++;
    if (launch_id) *launch_id = L;
    ctx->stats.launches++;
    KLaunch proto;
    memset(&proto, 0, sizeof proto);
    proto.ndim = nd;
    for (int p = 0; p < MAXPARAM && p < KMAXP; ++p) {
        proto.iarg[p] = iparams[p];
        proto.farg[p] = fparams[p];
    }
    for (int a = 0; a < MAXD; ++a) proto.block[a] = B[a];
    proto.variant = k->variant;
    proto.user = def->user;
    for (int p = 0; p < def->nparam && p < KMAXP; ++p)
        if (pany[p] && pmode[p] == M_REDUCE) proto.rop[p] = (int32_t)pop[p];
    for (auto &P : parts) {
        if (P.total_elems == 0) continue;
        if (ctx->batch.open) {
            // partials live in the batch's area, cleared once before the drain
            if (P.op != R_ADD)
                return set_err(ctx, LT_ERR_UNSUPPORTED, "batched reductions support reduce(+) only");
            P.batched = true;
            P.rel = ctx->batch.part_bytes;
            ctx->batch.part_bytes += P.bytes;
            P.signal = ctx->batch.nsignals++;
            continue;
        }
        st = flush_group(ctx);
        if (st) return st;
        Fence mem;
        st = alloc_range(ctx, P.bytes, 2, nullptr, &P.off, &mem);
        if (st) return st;
        int s = 0;
        st = stream_wait(ctx, s, mem);
        if (st) return st;
        if (def->slots_written) {
            // the body stores every element of its slots: no identity fill,
            // only the memory's earlier users to wait for
            P.ready.merge(mem);
            continue;
        }
        unsigned char idv[8];
        int esz;
        identity_bytes(arrs[P.param]->dtype, P.op, idv, &esz);
        trace_op(ctx, 4, s, ~0ull, 0, (uint64_t)P.bytes, (uint64_t)P.off);
        if (!ctx->dry) {
            hipError_t r = launch_fill(ctx->streams[s].h, ctx->arena_base + P.off, P.total_elems, esz, idv);
            if (r != hipSuccess) return hip_fail(ctx, r, "fill");
        }
        P.ready.add(s, bump(ctx, s));
    }
    st = refresh_launch_halos(ctx, plans, arrs, def->nparam);
    if (st) return st;
    // which of this launch's tasks use each chunk, for eviction by next use
    for (size_t i = 0; i < plans.size(); ++i) {
        auto note = [&](Chunk *c) {
            if (c->fut_launch != L) {
                c->fut.clear();
                c->fut_pos = 0;
                c->fut_launch = L;
            }
            if (c->fut.empty() || c->fut.back() != (int32_t)i) c->fut.push_back((int32_t)i);
        };
        for (int p = 0; p < def->nparam; ++p) {
            const ArgPlan &a = plans[i].arg[p];
            if (!a.used) continue;
            for (Chunk *c : a.chunks) note(c);
            for (Chunk *c : a.halo_owners) note(c);
        }
    }
    ctx->cur_launch = L;
    for (size_t i = 0; i < plans.size(); ++i) {
        TaskPlan &tp = plans[i];
        ctx->cur_task = (int32_t)i;
        tp.id = ctx->next_task_id++;
        ctx->launches.at(L).tasks.push_back(tp.id);
        st = issue_exec(ctx, k, tp, L, proto, arrs, parts, nd);
        if (st) {
            ctx->cur_launch = ~0ull;
            return st;
        }
        ctx->stats.tasks++;
    }
    ctx->cur_launch = ~0ull;
    st = flush_group(ctx);
    if (st) return st;
    for (auto &P : parts) {
        st = issue_combine(ctx, P, arrs[P.param], L);
        if (st) return st;
    }
    LaunchRec &lr = ctx->launches.at(L);
    for (uint64_t id : lr.tasks) {
        TaskRec *r = ctx->tasks.get(id);
        if (r && r->seq) lr.done.add(r->stream, r->seq);
    }
    if (ctx->batch.open && !ctx->batch.capture && ctx->cfg.batch_flush_tasks > 0 &&
        (int64_t)ctx->batch.q.size() >= ctx->cfg.batch_flush_tasks) {
        st = batch_flush(ctx);
        if (st) return st;
    }
    ctx->stats.plan_seconds += now_s() - t0;
    return LT_OK;
}

}  // namespace lt
