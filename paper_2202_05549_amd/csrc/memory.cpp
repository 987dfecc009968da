// Device arena, streams/fences and the memory manager.
//
// Memory manager (Sec. 3.4 "Memory Management"): chunks live in one
// pre-allocated device arena whose size is the device budget (the paper uses
// pre-allocated pools because device and page-locked allocations are slow).
// When a task's chunks do not fit, least-recently-used chunks that the task
// does not need are evicted: a chunk whose device copy is newer than its
// host copy is first copied back (device -> pinned host), a clean one is
// dropped.  Evicted data is reloaded asynchronously when a later task needs
// it.  All copies are asynchronous on dedicated copy streams.
//
// Ordering without host blocking: every stream operation gets a sequence
// number; a Fence is a vector clock over streams.  Freed memory carries the
// fence of its last users, and whoever reuses it first waits for that fence
// on the device (an event wait), so the host issues the whole schedule ahead
// and never waits for the GPU except in lt_sync / lt_wait / lt_array_read.
#include <fcntl.h>
#include <unistd.h>

#include <algorithm>
#include <climits>
#include <cerrno>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "kernels.h"
#include "lt_internal.h"

namespace lt {

static int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

lt_status set_err(Ctx *ctx, lt_status st, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return st;
}

lt_status hip_fail(Ctx *ctx, hipError_t e, const char *what) {
    char buf[512];
    snprintf(buf, sizeof buf, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
    if (ctx) {
        ctx->err = buf;
        if (ctx->sticky == LT_OK) {
            ctx->sticky = LT_ERR_DEVICE;
            ctx->sticky_msg = buf;
        }
    }
    return LT_ERR_DEVICE;
}

// ------------------------------------------------------------------ arena
void Arena::init(int64_t cap) {
    capacity = cap;
    segs.clear();
    free_by_size.clear();
    Seg s;
    s.off = 0;
    s.size = cap;
    segs[0] = s;
    index_add(s);
    used = peak = 0;
}

Seg *Arena::find(int64_t off) {
    auto it = segs.find(off);
    return it == segs.end() ? nullptr : &it->second;
}

int64_t Arena::largest_free() const {
    return free_by_size.empty() ? 0 : free_by_size.rbegin()->first;
}

int64_t Arena::take_free(int64_t size, Fence *fence_out, int kind, Chunk *owner) {
    auto it = free_by_size.lower_bound(size);  // best fit
    if (it == free_by_size.end()) return -1;
    return take_at(it->second, size, fence_out, kind, owner);
}

int64_t Arena::take_at(int64_t off, int64_t size, Fence *fence_out, int kind, Chunk *owner) {
    // the free segment containing `off`
    auto it = segs.upper_bound(off);
    if (it == segs.begin()) return -1;
    --it;
    Seg s = it->second;
    if (s.kind != 0 || off + size > s.off + s.size) return -1;
    index_del(s);
    segs.erase(it);
    if (off > s.off) {
        Seg head = s;
        head.size = off - s.off;
        segs[head.off] = head;
        index_add(head);
    }
    Seg mid = s;
    mid.off = off;
    mid.size = size;
    mid.kind = kind;
    mid.chunk = owner;
    segs[off] = mid;
    if (off + size < s.off + s.size) {
        Seg tail = s;
        tail.off = off + size;
        tail.size = s.off + s.size - tail.off;
        segs[tail.off] = tail;
        index_add(tail);
    }
    if (fence_out) *fence_out = s.fence;
    used += size;
    peak = std::max(peak, used);
    return off;
}

void Arena::release(int64_t off, const Fence &fence) {
    auto it = segs.find(off);
    if (it == segs.end() || it->second.kind == 0) return;
    used -= it->second.size;
    it->second.kind = 0;
    it->second.chunk = nullptr;
    it->second.fence.merge(fence);
    // coalesce with the next and previous free segments
    auto nx = std::next(it);
    if (nx != segs.end() && nx->second.kind == 0) {
        index_del(nx->second);
        it->second.size += nx->second.size;
        it->second.fence.merge(nx->second.fence);
        segs.erase(nx);
    }
    if (it != segs.begin()) {
        auto pv = std::prev(it);
        if (pv->second.kind == 0) {
            index_del(pv->second);
            pv->second.size += it->second.size;
            pv->second.fence.merge(it->second.fence);
            segs.erase(it);
            it = pv;
        }
    }
    index_add(it->second);
}

// ---------------------------------------------------------------- tracing
void trace_op(Ctx *ctx, int kind, int stream, uint64_t task, uint64_t chunk,
              uint64_t bytes, uint64_t offset) {
    if (!ctx->cfg.trace) return;
    lt_trace_rec r;
    r.kind = kind;
    r.stream = stream;
    r.task = task;
    r.chunk = chunk;
    r.bytes = bytes;
    r.offset = offset;
    r.resident = (uint64_t)ctx->arena.used;
    ctx->trace.push_back(r);
}

// ---------------------------------------------------------------- streams
static hipEvent_t get_event(Ctx *ctx) {
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

uint64_t bump(Ctx *ctx, int s) { return ++ctx->streams[s].seq; }

// Event whose completion implies stream t has executed through `seq`: the
// first mark at or after seq, else a new mark at the stream's current end
// (which also covers everything issued after seq, so a wait on it may be
// longer than needed; mark_tail avoids that for fences known to be waited on).
static lt_status mark_at(Ctx *ctx, int t, uint64_t seq, hipEvent_t *ev, uint64_t *mseq) {
    Stream &S = ctx->streams[t];
    // marks are recorded in increasing seq order
    auto it = std::lower_bound(S.marks.begin(), S.marks.end(), seq,
                               [](const Mark &m, uint64_t v) { return m.seq < v; });
    if (it != S.marks.end()) {
        *ev = it->ev;
        *mseq = it->seq;
        return LT_OK;
    }
    hipEvent_t e = get_event(ctx);
    if (!e) return set_err(ctx, LT_ERR_DEVICE, "hipEventCreate failed");
    hipError_t r = hipEventRecord(e, S.h);
    if (r != hipSuccess) return hip_fail(ctx, r, "hipEventRecord");
    S.marks.push_back({S.seq, e});
    *ev = e;
    *mseq = S.seq;
    return LT_OK;
}

lt_status mark_tail(Ctx *ctx, int s) {
    if (ctx->dry) return LT_OK;
    Stream &S = ctx->streams[s];
    // marks at or before what is known to have completed are never needed
    // again (waits already enqueued on them keep their own snapshot)
    while (!S.marks.empty() && S.marks.front().seq <= S.done) {
        ctx->event_pool.push_back(S.marks.front().ev);
        S.marks.pop_front();
    }
    if (!S.marks.empty() && S.marks.back().seq == S.seq) return LT_OK;
    hipEvent_t ev;
    uint64_t mseq;
    return mark_at(ctx, s, S.seq, &ev, &mseq);
}

lt_status stream_wait(Ctx *ctx, int s, const Fence &f) {
    Stream &S = ctx->streams[s];
    for (int t = 0; t < ctx->nstreams; ++t) {
        if (t == s) continue;
        uint64_t need = f.s[t];
        if (need <= ctx->streams[t].done || need <= S.waited[t]) continue;
        if (ctx->dry) {
            S.waited[t] = need;
            continue;
        }
        hipEvent_t ev;
        uint64_t mseq;
        lt_status st = mark_at(ctx, t, need, &ev, &mseq);
        if (st) return st;
        hipError_t r = hipStreamWaitEvent(S.h, ev, 0);
        if (r != hipSuccess) return hip_fail(ctx, r, "hipStreamWaitEvent");
        S.waited[t] = mseq;
    }
    return LT_OK;
}

// Non-blocking: has every stream reached its entry of f?  Learns completed
// sequence numbers along the way.
bool fence_done(Ctx *ctx, const Fence &f) {
    if (ctx->dry) return true;
    for (int t = 0; t < ctx->nstreams; ++t) {
        if (f.s[t] <= ctx->streams[t].done) continue;
        hipEvent_t ev;
        uint64_t mseq;
        if (mark_at(ctx, t, f.s[t], &ev, &mseq)) return false;
        hipError_t r = hipEventQuery(ev);
        if (r == hipErrorNotReady) return false;
        if (r != hipSuccess) {
            hip_fail(ctx, r, "hipEventQuery");
            return true;
        }
        if (mseq > ctx->streams[t].done) ctx->streams[t].done = mseq;
    }
    return true;
}

lt_status wait_fence(Ctx *ctx, const Fence &f) {
    if (ctx->dry) return LT_OK;
    for (int t = 0; t < ctx->nstreams; ++t) {
        if (f.s[t] <= ctx->streams[t].done) continue;
        hipEvent_t ev;
        uint64_t mseq;
        lt_status st = mark_at(ctx, t, f.s[t], &ev, &mseq);
        if (st) return st;
        hipError_t r = hipEventSynchronize(ev);
        if (r != hipSuccess) return hip_fail(ctx, r, "hipEventSynchronize");
    }
    return LT_OK;
}

// ------------------------------------------------------------------ copies
// Copies a box of `ext` elements between two strided layouts (element
// strides; the last axis is contiguous on both sides).  Axes that are
// contiguous on both sides are merged first.
lt_status copy_box(Ctx *ctx, int stream, char *dst, const int64_t *ds,
                   const char *src, const int64_t *ss, const int64_t *ext,
                   int nd, int esz, hipMemcpyKind kind, bool by_kernel) {
    // axes from the innermost outwards; an outer axis is merged into the
    // current innermost group when both layouts are contiguous across them
    int64_t e[MAXD], d[MAXD], s[MAXD];
    int n = 0;
    for (int a = nd - 1; a >= 0; --a) {
        if (ext[a] <= 0) return LT_OK;
        if (n > 0 && ds[a] == e[n - 1] * d[n - 1] && ss[a] == e[n - 1] * s[n - 1]) {
            e[n - 1] *= ext[a];
            continue;
        }
        e[n] = ext[a];
        d[n] = ds[a];
        s[n] = ss[a];
        ++n;
    }
    // reorder outermost first
    for (int i = 0; i < n / 2; ++i) {
        std::swap(e[i], e[n - 1 - i]);
        std::swap(d[i], d[n - 1 - i]);
        std::swap(s[i], s[n - 1 - i]);
    }
    int64_t bytes = esz;
    for (int a = 0; a < n; ++a) bytes *= e[a];
    int tk = kind == hipMemcpyHostToDevice ? 1 : kind == hipMemcpyDeviceToHost ? 2 : 3;
    if (tk == 1) {
        ctx->stats.bytes_h2d += bytes;
        ctx->stats.copies_h2d++;
    } else if (tk == 2) {
        ctx->stats.bytes_d2h += bytes;
        ctx->stats.copies_d2h++;
    } else {
        ctx->stats.bytes_d2d += bytes;
        ctx->stats.copies_d2d++;
    }
    if (ctx->dry) return LT_OK;
    if (kind == hipMemcpyHostToHost) {
        // plain CPU copy; the caller has synchronized pending device copies
        for (int64_t i = 0; i < (n == 3 ? e[0] : 1); ++i) {
            int64_t rows = n >= 2 ? e[n - 2] : 1;
            for (int64_t r = 0; r < rows; ++r) {
                int64_t doff = (n == 3 ? i * d[0] : 0) + (n >= 2 ? r * d[n - 2] : 0);
                int64_t soff = (n == 3 ? i * s[0] : 0) + (n >= 2 ? r * s[n - 2] : 0);
                memcpy(dst + doff * esz, src + soff * esz, (size_t)(e[n - 1] * esz));
            }
        }
        return LT_OK;
    }
    hipStream_t h = ctx->streams[stream].h;
    hipError_t r = hipSuccess;
    // with profiling on, copies over the host link are timed like kernels
    const char *pname = tk == 1 ? "copy_h2d" : tk == 2 ? "copy_d2h" : nullptr;
    hipEvent_t pa = nullptr;
    if (pname) {
        lt_status st = prof_begin(ctx, stream, pname, &pa);
        if (st) return st;
    }
    if (by_kernel) {
        // rows of the innermost axis; a third axis loops over planes
        const int64_t planes = n == 3 ? e[0] : 1;
        for (int64_t i = 0; i < planes && r == hipSuccess; ++i) {
            char *dp = dst + (n == 3 ? i * d[0] * esz : 0);
            const char *sp = src + (n == 3 ? i * s[0] * esz : 0);
            r = n == 1 ? launch_copy_rows(h, dp, 0, sp, 0, e[0] * esz, 1)
                       : launch_copy_rows(h, dp, d[n - 2] * esz, sp, s[n - 2] * esz, e[n - 1] * esz, e[n - 2]);
        }
    } else if (n == 1) {
        r = hipMemcpyAsync(dst, src, e[0] * esz, kind, h);
    } else if (n == 2) {
        r = hipMemcpy2DAsync(dst, d[0] * esz, src, s[0] * esz, e[1] * esz, e[0], kind, h);
    } else {
        for (int64_t i = 0; i < e[0] && r == hipSuccess; ++i)
            r = hipMemcpy2DAsync(dst + i * d[0] * esz, d[1] * esz, src + i * s[0] * esz,
                                 s[1] * esz, e[2] * esz, e[1], kind, h);
    }
    if (r != hipSuccess) return hip_fail(ctx, r, "hipMemcpyAsync");
    return pname ? prof_end(ctx, stream, pname, pa) : LT_OK;
}

// ------------------------------------------------------------------- arena
lt_status ensure_arena(Ctx *ctx) {
    if (ctx->arena.capacity > 0) return LT_OK;
    int64_t cap = (int64_t)ctx->cfg.device_budget_bytes;
    if (ctx->cfg.device_arena) {
        if (cap <= 0 || cap > (int64_t)ctx->cfg.arena_bytes) cap = (int64_t)ctx->cfg.arena_bytes;
        ctx->arena_base = (char *)ctx->cfg.device_arena;
        ctx->arena_owned = false;
    } else if (!ctx->dry) {
        void *p = nullptr;
        hipError_t r = hipMalloc(&p, (size_t)cap);
        if (r != hipSuccess) return hip_fail(ctx, r, "hipMalloc(device arena)");
        ctx->arena_base = (char *)p;
        ctx->arena_owned = true;
    }
    ctx->arena.init(cap);
    return LT_OK;
}

static void note_resident(Ctx *ctx) {
    ctx->stats.resident_bytes = (uint64_t)ctx->arena.used;
    if (ctx->stats.resident_bytes > ctx->stats.peak_resident_bytes)
        ctx->stats.peak_resident_bytes = ctx->stats.resident_bytes;
}

// ------------------------------------------------------------ disk tier
// Spill buffers of device-home arrays live in pinned host memory up to
// cfg.host_budget_bytes; beyond it the least recently used ones move to a
// spill file (one slot per chunk) and come back on demand (Sec. 3.4: the
// memory hierarchy continues below host memory).  The file reads and writes
// run as host functions on the copy streams (hipLaunchHostFunc), ordered
// with the copies by the streams themselves: a write follows the copies
// into or out of its buffer on the D2H stream, and a read precedes the H2D
// copy of its chunk on the H2D stream.  The issuing thread never waits for
// the disk.

static lt_status open_spill_file(Ctx *ctx) {
    if (ctx->spill_fd >= 0 || ctx->dry) return LT_OK;
    const char *env = getenv("TMPDIR");
    std::string dir = ctx->cfg.spill_dir ? ctx->cfg.spill_dir : (env && *env ? env : "/tmp");
    std::string path = dir + "/lt_spill_XXXXXX";
    std::vector<char> name(path.begin(), path.end());
    name.push_back('\0');
    int fd = mkstemp(name.data());
    if (fd < 0) return set_err(ctx, LT_ERR_OOM, "cannot create a spill file in %s: %s", dir.c_str(), strerror(errno));
    unlink(name.data());  // the file lives as long as the descriptor
    ctx->spill_fd = fd;
    return LT_OK;
}

// One spill file transfer, run by the HIP runtime's host-function thread.
struct DiskJob {
    Ctx *ctx;
    int fd;
    char *p;
    int64_t bytes, off;
    bool write;
};

static void disk_io(void *arg) {
    DiskJob *j = static_cast<DiskJob *>(arg);
    int64_t done = 0;
    while (done < j->bytes) {
        const ssize_t r = j->write ? pwrite(j->fd, j->p + done, (size_t)(j->bytes - done), j->off + done)
                                   : pread(j->fd, j->p + done, (size_t)(j->bytes - done), j->off + done);
        if (r <= 0) {
            int expected = 0;
            // the first error wins; its operation is published after it
            if (j->ctx->disk_errno.compare_exchange_strong(expected, r < 0 ? errno : EIO))
                j->ctx->disk_errop.store(j->write ? 2 : 1);
            break;
        }
        done += r;
    }
    delete j;
}

// Enqueues a transfer of `bytes` between p and the spill file at `off` on
// stream s; *seq is the stream position after it.
static lt_status enqueue_disk(Ctx *ctx, int s, char *p, int64_t bytes, int64_t off, bool write, uint64_t *seq) {
    DiskJob *j = new DiskJob{ctx, ctx->spill_fd, p, bytes, off, write};
    const hipError_t r = hipLaunchHostFunc(ctx->streams[s].h, disk_io, j);
    if (r != hipSuccess) {
        delete j;
        return hip_fail(ctx, r, write ? "hipLaunchHostFunc(spill file write)" : "hipLaunchHostFunc(spill file read)");
    }
    *seq = bump(ctx, s);
    return LT_OK;
}

lt_status disk_status(Ctx *ctx) {
    const int e = ctx->disk_errno.load();
    if (!e) return LT_OK;
    int op = 0;
    while (!(op = ctx->disk_errop.load())) {
    }
    ctx->disk_errop.store(0);
    ctx->disk_errno.store(0);
    return set_err(ctx, LT_ERR_OOM, "spill file %s: %s", op == 2 ? "write" : "read", strerror(e));
}

// Pinned spill buffers are recycled through a pool keyed by size: pinning
// and unpinning host memory costs milliseconds per buffer (hipHostFree may
// also wait for the device), while chunks of one array all have one size.
// Pooled buffers count against the host budget; without a budget the pool
// keeps at most PIN_POOL_CAP bytes.
constexpr int64_t PIN_POOL_CAP = (int64_t)2 << 30;

static void pin_release(Ctx *ctx, char *p) {
    if (ctx->dry) free(p);
    else (void)hipHostFree(p);
}

static char *pool_take(Ctx *ctx, int64_t bytes, Fence *ready) {
    auto it = ctx->pin_pool.find(bytes);
    if (it == ctx->pin_pool.end()) return nullptr;
    char *p = it->second.p;
    *ready = it->second.ready;
    ctx->pin_pool.erase(it);
    ctx->pin_pooled -= bytes;
    return p;
}

// Frees one pooled buffer (the largest), after the transfers still using
// it; false when the pool is empty.
static bool pool_shrink(Ctx *ctx) {
    if (ctx->pin_pool.empty()) return false;
    auto it = std::prev(ctx->pin_pool.end());
    (void)wait_fence(ctx, it->second.ready);
    ctx->pin_pooled -= it->first;
    pin_release(ctx, it->second.p);
    ctx->pin_pool.erase(it);
    return true;
}

void drain_pin_pool(Ctx *ctx) {
    while (pool_shrink(ctx)) {
    }
}

// Returns c's spill buffer to the pool (or frees it), free for a new owner
// after `release`.
static void release_spill(Ctx *ctx, Chunk *c, const Fence &release) {
    if (!c->host_owned || !c->host_ptr) return;
    const int64_t cap = (int64_t)ctx->cfg.host_budget_bytes;
    if (cap > 0 || ctx->pin_pooled + c->bytes <= PIN_POOL_CAP) {
        ctx->pin_pool.emplace(c->bytes, Ctx::PooledPin{c->host_ptr, release});
        ctx->pin_pooled += c->bytes;
    } else {
        (void)wait_fence(ctx, release);
        pin_release(ctx, c->host_ptr);
    }
    c->host_ptr = nullptr;
    ctx->host_spill_bytes -= c->bytes;
    ctx->stats.host_spill_bytes = (uint64_t)ctx->host_spill_bytes;
}

void free_spill(Ctx *ctx, Chunk *c) {
    // any copy into or out of the buffer, and a pending spill file write
    Fence f = c->host_ready;
    f.merge(c->last_access);
    f.merge(c->disk_ready);
    release_spill(ctx, c, f);
}

// Moves one spill buffer to the spill file (if it holds data the file does
// not have yet) and releases it.
static lt_status demote(Ctx *ctx, Chunk *c) {
    Fence f = c->host_ready;
    f.merge(c->last_access);
    Fence release = f;
    if (c->host_valid && c->defined && !c->disk_valid) {
        lt_status st = open_spill_file(ctx);
        if (st) return st;
        if (c->disk_off < 0) {
            c->disk_off = ctx->disk_next;
            ctx->disk_next += round_up(c->bytes, 4096);
        }
        if (!ctx->dry) {
            // after the copies into and out of the buffer
            st = stream_wait(ctx, ctx->d2h, f);
            if (st) return st;
            uint64_t seq;
            st = enqueue_disk(ctx, ctx->d2h, c->host_ptr, c->bytes, c->disk_off, true, &seq);
            if (st) return st;
            c->disk_ready = Fence();
            c->disk_ready.add(ctx->d2h, seq);
            release = c->disk_ready;
        }
        c->disk_valid = true;
        ctx->stats.bytes_disk_write += (uint64_t)c->bytes;
        trace_op(ctx, 8, -1, ~0ull, c->id, (uint64_t)c->bytes, (uint64_t)c->disk_off);
    }
    release_spill(ctx, c, release);
    return LT_OK;
}

// A pinned buffer of `need` bytes for chunk `keep`: from the pool when one of
// that size is there (free after *ready), else newly pinned once the held
// and pooled buffers leave room under the host budget.  Room is made by
// freeing pooled buffers, then by moving the least recently used spill
// buffer to the disk tier (its buffer returns to the pool and is taken here
// when it fits).
static lt_status pinned_for(Ctx *ctx, int64_t need, const Chunk *keep, char **out, Fence *ready) {
    const int64_t cap = (int64_t)ctx->cfg.host_budget_bytes;
    if (cap > 0 && need > cap)
        return set_err(ctx, LT_ERR_BUDGET, "a %lld-byte spill buffer exceeds the host budget of %lld bytes",
                       (long long)need, (long long)cap);
    *ready = Fence();
    for (;;) {
        if (char *p = pool_take(ctx, need, ready)) {
            *out = p;
            return LT_OK;
        }
        if (cap <= 0 || ctx->host_spill_bytes + ctx->pin_pooled + need <= cap) break;
        if (pool_shrink(ctx)) continue;
        // any other buffer may go: its new owner's transfers wait for the
        // copies and the spill file write using it
        Chunk *victim = nullptr;
        for (Array *arr : ctx->arrays)
            for (Chunk *c : arr->chunks)
                if (c != keep && c->host_owned && c->host_ptr && (!victim || c->lru < victim->lru)) victim = c;
        if (!victim)
            return set_err(ctx, LT_ERR_BUDGET, "the host budget of %lld bytes is held by spill buffers in use",
                           (long long)cap);
        lt_status st = demote(ctx, victim);
        if (st) return st;
    }
    void *p = nullptr;
    if (ctx->dry) {
        p = malloc(1);
    } else {
        hipError_t r = hipHostMalloc(&p, (size_t)need, hipHostMallocDefault);
        if (r != hipSuccess) return set_err(ctx, LT_ERR_OOM, "pinned spill buffer of %lld bytes: %s",
                                            (long long)need, hipGetErrorString(r));
    }
    *out = (char *)p;
    return LT_OK;
}

lt_status host_resident(Ctx *ctx, Chunk *c) {
    if (c->host_ptr || !c->host_owned || !c->disk_valid) return LT_OK;
    lt_status st = ensure_host_copy(ctx, c);
    if (st) return st;
    if (!ctx->dry) {
        // after the buffer's previous users and the slot's write; the H2D
        // copy of the chunk follows on the same stream
        Fence f = c->host_ready;
        f.merge(c->disk_ready);
        st = stream_wait(ctx, ctx->h2d, f);
        if (st) return st;
        uint64_t seq;
        st = enqueue_disk(ctx, ctx->h2d, c->host_ptr, c->bytes, c->disk_off, false, &seq);
        if (st) return st;
        c->host_ready = Fence();
        c->host_ready.add(ctx->h2d, seq);
    }
    ctx->stats.bytes_disk_read += (uint64_t)c->bytes;
    trace_op(ctx, 9, -1, ~0ull, c->id, (uint64_t)c->bytes, (uint64_t)c->disk_off);
    return LT_OK;
}

lt_status ensure_host_copy(Ctx *ctx, Chunk *c) {
    if (c->host_ptr) return LT_OK;
    Array *arr = c->arr;
    if (arr->host_backed) {
        int64_t off = 0;
        for (int a = 0; a < arr->ndim; ++a) off += c->box.lo[a] * arr->strides[a];
        c->host_ptr = arr->host_base + off * arr->esz;
        for (int a = 0; a < MAXD; ++a) c->host_stride[a] = arr->strides[a];
        return LT_OK;
    }
    char *p = nullptr;
    Fence ready;
    lt_status st = pinned_for(ctx, c->bytes, c, &p, &ready);
    if (st) return st;
    c->host_ptr = p;
    c->host_owned = true;
    // writers into the buffer wait for its previous owner's transfers
    c->host_ready = ready;
    ctx->host_spill_bytes += c->bytes;
    ctx->stats.host_spill_bytes = (uint64_t)ctx->host_spill_bytes;
    for (int a = 0; a < MAXD; ++a) c->host_stride[a] = c->dev_stride[a];
    return LT_OK;
}

static void chunk_ext(const Chunk *c, int64_t *ext) {
    for (int a = 0; a < MAXD; ++a) ext[a] = c->box.hi[a] - c->box.lo[a];
}

char *dev_ptr(Ctx *ctx, const Chunk *c) { return ctx->arena_base + c->dev_off; }

lt_status copy_sub(Ctx *ctx, int stream, char *dst, const int64_t *dlo, const int64_t *ds, const char *src,
                   const int64_t *slo, const int64_t *ss, const Box &sub, int nd, int esz, hipMemcpyKind kind,
                   bool by_kernel) {
    int64_t doff = 0, soff = 0, ext[MAXD];
    for (int a = 0; a < MAXD; ++a) {
        const int64_t lo = a < nd ? sub.lo[a] : 0;
        doff += (lo - (a < nd ? dlo[a] : 0)) * ds[a];
        soff += (lo - (a < nd ? slo[a] : 0)) * ss[a];
        ext[a] = a < nd ? sub.hi[a] - sub.lo[a] : 1;
    }
    return copy_box(ctx, stream, dst + doff * esz, ds, src + soff * esz, ss, ext, nd, esz, kind, by_kernel);
}

lt_status write_back(Ctx *ctx, Chunk *c, uint64_t *seq) {
    lt_status st = ensure_host_copy(ctx, c);
    if (st) return st;
    // after the device copy is written, and after earlier transfers of the
    // host buffer (a pooled buffer's previous owner included)
    Fence f = c->data_ready;
    f.merge(c->host_ready);
    st = stream_wait(ctx, ctx->d2h, f);
    if (st) return st;
    const Array *arr = c->arr;
    const Box &part = arr->host_backed ? c->core : c->box;
    hipEvent_t pa = nullptr;
    const bool by_kernel = c->host_owned && !ctx->dry && c->bytes >= ((int64_t)1 << 20);
    if (by_kernel) {
        st = prof_begin(ctx, ctx->d2h, "copy_d2h", &pa);
        if (st) return st;
    }
    if (by_kernel &&
        launch_copy_linear(ctx->streams[ctx->d2h].h, c->host_ptr, dev_ptr(ctx, c), c->bytes) == hipSuccess) {
        // a spill buffer (pinned by the runtime, so kernels can write it)
        // holds the whole box with the device layout: one linear copy, done
        // by a copy kernel
        ctx->stats.bytes_d2h += (uint64_t)c->bytes;
        ctx->stats.copies_d2h++;
        st = prof_end(ctx, ctx->d2h, "copy_d2h", pa);
        if (st) return st;
    } else {
        if (pa) {
            // the copy kernel could not take it: the timing goes to copy_box
            ctx->prof_pool.push_back(pa);
        }
        // a pinned home buffer can take a copy kernel too (d2h_kernel = 1)
        const bool k = arr->host_backed && arr->home_pinned && ctx->cfg.d2h_kernel && !ctx->dry;
        st = copy_sub(ctx, ctx->d2h, c->host_ptr, c->box.lo, c->host_stride, dev_ptr(ctx, c), c->box.lo,
                      c->dev_stride, part, arr->ndim, arr->esz, hipMemcpyDeviceToHost, k);
        if (st) return st;
    }
    *seq = bump(ctx, ctx->d2h);
    c->host_ready = Fence();
    c->host_ready.add(ctx->d2h, *seq);
    c->host_valid = true;
    c->disk_valid = false;
    c->host_version = c->version;
    trace_op(ctx, 2, ctx->d2h, ~0ull, c->id, c->bytes, c->dev_off);
    return LT_OK;
}

lt_status refresh_halo(Ctx *ctx, Chunk *c, const Box &region) {
    const Array *arr = c->arr;
    const int nd = arr->ndim;
    for (HaloSrc &h : c->halo) {
        Chunk *k = h.k;
        if ((h.valid && h.ver >= k->version) || intersect(h.box, region, nd).empty(nd)) continue;
        if (!k->defined) {
            h.ver = k->version;
            h.valid = true;
            continue;
        }
        // the copy overwrites part of c: after every earlier use of c; it
        // reads k: after k's last write (or load)
        Fence f = c->last_access;
        f.merge(c->data_ready);
        lt_status st;
        if (k->dev_off >= 0 && k->dev_valid) {
            f.merge(k->data_ready);
            st = stream_wait(ctx, ctx->h2d, f);
            if (st) return st;
            st = copy_sub(ctx, ctx->h2d, dev_ptr(ctx, c), c->box.lo, c->dev_stride, dev_ptr(ctx, k), k->box.lo,
                          k->dev_stride, h.box, nd, arr->esz, hipMemcpyDeviceToDevice);
            if (st) return st;
            ctx->stats.halo_copies++;
            trace_op(ctx, 3, ctx->h2d, ~0ull, c->id, (uint64_t)(h.box.volume(nd) * arr->esz), c->dev_off);
        } else {
            // the owner is not on the device: its newest copy is the host one
            st = host_resident(ctx, k);
            if (st) return st;
            if (!k->host_valid || !k->host_ptr)
                return set_err(ctx, LT_ERR_INVALID, "internal: halo owner chunk %llu has no valid copy",
                               (unsigned long long)k->id);
            f.merge(k->host_ready);
            st = stream_wait(ctx, ctx->h2d, f);
            if (st) return st;
            st = copy_sub(ctx, ctx->h2d, dev_ptr(ctx, c), c->box.lo, c->dev_stride, k->host_ptr, k->box.lo,
                          k->host_stride, h.box, nd, arr->esz, hipMemcpyHostToDevice);
            if (st) return st;
            ctx->stats.halo_copies++;
            trace_op(ctx, 1, ctx->h2d, ~0ull, c->id, (uint64_t)(h.box.volume(nd) * arr->esz), c->dev_off);
        }
        const uint64_t p = bump(ctx, ctx->h2d);
        c->data_ready.add(ctx->h2d, p);
        c->last_access.add(ctx->h2d, p);
        k->last_access.add(ctx->h2d, p);  // the copy reads k's device or host copy
        // a spill buffer holds the whole stored box, so it no longer matches;
        // a host-backed home buffer only ever receives c's core
        if (!arr->host_backed) c->host_valid = false;
        h.ver = k->version;
        h.valid = true;
    }
    return LT_OK;
}

// Evicts one unpinned chunk: write back if its device copy is newer.
lt_status evict_chunk(Ctx *ctx, Chunk *c) {
    ctx->budget_binds = true;
    Fence f = c->last_access;
    if (c->dev_valid && !c->host_valid && c->defined) {
        uint64_t p = 0;
        lt_status st = write_back(ctx, c, &p);
        if (st) return st;
        f.add(ctx->d2h, p);
        ctx->stats.evictions_dirty++;
    } else {
        ctx->stats.evictions_clean++;
    }
    ctx->arena.release(c->dev_off, f);
    trace_op(ctx, 5, -1, ~0ull, c->id, c->bytes, c->dev_off);
    c->dev_off = -1;
    c->dev_valid = false;
    note_resident(ctx);
    return LT_OK;
}

// Eviction rank of chunk c under the next-use policy (higher = evict
// first): the index of the next task of the launch being issued that uses c,
// INT32_MAX when none does.  A chunk used by one of the last EVICT_RECENT
// tasks ranks -1 whatever its next use: those tasks have most likely not run
// yet (the host issues ahead of the device), so reusing the chunk's memory
// would make the current task wait for them and for the chunk's write-back.
constexpr int32_t EVICT_RECENT = 2;
static int32_t evict_rank(Ctx *ctx, Chunk *c) {
    if (ctx->cur_launch == ~0ull || c->fut_launch != ctx->cur_launch) return INT32_MAX;
    while (c->fut_pos < c->fut.size() && c->fut[c->fut_pos] <= ctx->cur_task) ++c->fut_pos;
    if (c->fut_pos > 0 && ctx->cur_task - c->fut[c->fut_pos - 1] <= EVICT_RECENT) return -1;
    return c->fut_pos < c->fut.size() ? c->fut[c->fut_pos] : INT32_MAX;
}

// Allocates `size` bytes of the arena, evicting unpinned chunks when no free
// range is large enough.  `fence` receives the point after which the memory
// may be overwritten.
lt_status alloc_range(Ctx *ctx, int64_t size, int kind, Chunk *owner,
                      int64_t *off, Fence *fence) {
    lt_status st = ensure_arena(ctx);
    if (st) return st;
    Arena &A = ctx->arena;
    int64_t o = A.take_free(size, fence, kind, owner);
    if (o < 0) {
        // choose a contiguous window of free or evictable segments; pinned
        // chunks and temporaries block a window.  LRU: the window whose most
        // recently used chunk is the oldest (exact LRU when chunks have equal
        // sizes).  Next use: first the window whose lowest-ranked chunk
        // (evict_rank) ranks highest, then LRU among equals.
        const bool by_use = ctx->cfg.evict_policy == LT_EVICT_NEXT_USE;
        std::vector<Seg *> order;
        order.reserve(A.segs.size());
        for (auto &kv : A.segs) order.push_back(&kv.second);
        int64_t best_start = -1;
        uint64_t best_cost = ~0ull;
        int32_t best_use = INT32_MIN;
        size_t n = order.size();
        for (size_t i = 0; i < n; ++i) {
            int64_t sum = 0;
            uint64_t cost = 0;
            int32_t use = INT32_MAX;
            size_t j = i;
            bool ok = false;
            for (; j < n; ++j) {
                Seg *s = order[j];
                if (s->kind == 2 || (s->kind == 1 && s->chunk->pin > 0)) break;
                if (s->kind == 1) {
                    cost = std::max<uint64_t>(cost, s->chunk->lru + 1);
                    if (by_use) use = std::min(use, evict_rank(ctx, s->chunk));
                }
                sum += s->size;
                if (sum >= size) {
                    ok = true;
                    break;
                }
            }
            if (!ok) continue;
            if (use > best_use || (use == best_use && cost < best_cost)) {
                best_use = use;
                best_cost = cost;
                best_start = order[i]->off;
            }
        }
        if (best_start < 0)
            return set_err(ctx, LT_ERR_BUDGET,
                           "cannot place %lld bytes in the device budget of %lld bytes "
                           "(%lld in use, largest free range %lld)",
                           (long long)size, (long long)A.capacity, (long long)A.used,
                           (long long)A.largest_free());
        // evict every chunk in the window
        std::vector<Chunk *> victims;
        int64_t sum = 0;
        for (auto it = A.segs.find(best_start); it != A.segs.end() && sum < size; ++it) {
            if (it->second.kind == 1) victims.push_back(it->second.chunk);
            sum += it->second.size;
        }
        for (Chunk *v : victims) {
            st = evict_chunk(ctx, v);
            if (st) return st;
        }
        o = A.take_at(best_start, size, fence, kind, owner);
        if (o < 0) return set_err(ctx, LT_ERR_BUDGET, "internal: eviction window did not free %lld bytes",
                                  (long long)size);
    }
    *off = o;
    trace_op(ctx, 6, -1, ~0ull, owner ? owner->id : 0, size, o);
    note_resident(ctx);
    return LT_OK;
}

// Places a chunk in the arena.  A chunk of a row-slab array goes right after
// its resident predecessor when that space is free, so runs of neighbouring
// chunks stay contiguous and regions spanning them resolve to direct views.
lt_status alloc_chunk(Ctx *ctx, Chunk *c, Fence *fence) {
    lt_status st = ensure_arena(ctx);
    if (st) return st;
    Array *arr = c->arr;
    if (arr->row_slab && c->index > 0) {
        Chunk *p = arr->chunks[c->index - 1];
        if (p->dev_off >= 0) {
            int64_t o = ctx->arena.take_at(p->dev_off + p->bytes, c->bytes, fence, 1, c);
            if (o >= 0) {
                c->dev_off = o;
                trace_op(ctx, 6, -1, ~0ull, c->id, c->bytes, o);
                note_resident(ctx);
                return LT_OK;
            }
        }
    }
    int64_t off;
    st = alloc_range(ctx, round_up(c->bytes, 256), 1, c, &off, fence);
    if (st) return st;
    c->dev_off = off;
    return LT_OK;
}

// Splits the arena range [off, off + total) into one segment per chunk, in
// order, each chunk directly after the previous one.
static void carve(Ctx *ctx, int64_t off, int64_t total, const std::vector<Chunk *> &run, const Fence &f) {
    Arena &A = ctx->arena;
    Seg whole = A.segs[off];
    A.segs.erase(off);
    int64_t cur = off;
    for (size_t i = 0; i < run.size(); ++i) {
        Chunk *c = run[i];
        Seg s;
        s.off = cur;
        s.size = (i + 1 == run.size()) ? (off + total - cur) : c->bytes;
        s.kind = 1;
        s.chunk = c;
        s.fence = f;
        A.segs[cur] = s;
        c->dev_off = cur;
        cur += c->bytes;
    }
    (void)whole;
}

// Makes a run of neighbouring chunks of a row-slab array resident in one
// contiguous range, in order, so that a region spanning them is a direct
// view.  Scattered members are moved into a new window with device-to-device
// copies (dirty ones stay dirty: nothing goes through the host); members not
// resident are loaded afterwards by stage_chunk.  Only when the window does
// not fit beside the old copies are the resident members evicted (their data
// goes back to the host copy) and everything reloaded into the window.
// Returns the fence after which the window's memory may be written.
lt_status place_run(Ctx *ctx, const std::vector<Chunk *> &run, Fence *mem) {
    bool contiguous = true;
    for (size_t i = 0; i < run.size(); ++i) {
        if (run[i]->dev_off < 0) contiguous = false;
        else if (i > 0 && run[i - 1]->dev_off >= 0 && run[i]->dev_off != run[i - 1]->dev_off + run[i - 1]->bytes)
            contiguous = false;
    }
    if (contiguous) return LT_OK;
    // try to extend in place: every missing member right after its predecessor
    bool ok = true;
    for (size_t i = 1; i < run.size() && ok; ++i) {
        if (run[i]->dev_off >= 0) continue;
        if (run[i - 1]->dev_off < 0) {
            ok = false;
            break;
        }
        Fence f;
        int64_t o = ctx->arena.take_at(run[i - 1]->dev_off + run[i - 1]->bytes, run[i]->bytes, &f, 1, run[i]);
        if (o < 0) {
            ok = false;
            break;
        }
        run[i]->dev_off = o;
        run[i]->dev_valid = false;
        mem->merge(f);
    }
    if (ok) {
        bool cont = true;
        for (size_t i = 1; i < run.size(); ++i)
            if (run[i]->dev_off != run[i - 1]->dev_off + run[i - 1]->bytes) cont = false;
        if (cont) return LT_OK;
    }
    // move: the resident members keep their pins, so the window cannot
    // take their old ranges, which are released once the copies are issued
    for (Chunk *c : run)
        if (c->dev_off >= 0 && !c->dev_valid) {  // placed above but not loaded yet
            ctx->arena.release(c->dev_off, Fence());
            c->dev_off = -1;
        }
    {
        int64_t total = 0;
        for (Chunk *c : run) total += c->bytes;
        const int64_t rounded = round_up(total, 256);
        int64_t off;
        Fence f;
        if (alloc_range(ctx, rounded, 1, nullptr, &off, &f) == LT_OK) {
            std::vector<std::pair<Chunk *, int64_t>> moved;
            for (Chunk *c : run)
                if (c->dev_off >= 0) moved.push_back({c, c->dev_off});
            carve(ctx, off, rounded, run, f);
            for (auto &mv : moved) {
                Chunk *c = mv.first;
                Fence w = f;
                w.merge(c->data_ready);
                lt_status st = stream_wait(ctx, ctx->h2d, w);
                if (st) return st;
                const int64_t one = 1, ext = c->bytes;
                st = copy_box(ctx, ctx->h2d, ctx->arena_base + c->dev_off, &one, ctx->arena_base + mv.second, &one,
                              &ext, 1, 1, hipMemcpyDeviceToDevice);
                if (st) return st;
                const uint64_t p = bump(ctx, ctx->h2d);
                trace_op(ctx, 3, ctx->h2d, ~0ull, c->id, (uint64_t)c->bytes, (uint64_t)c->dev_off);
                Fence rel = c->last_access;
                rel.add(ctx->h2d, p);
                ctx->arena.release(mv.second, rel);
                c->data_ready = Fence();
                c->data_ready.add(ctx->h2d, p);
                c->last_access = c->data_ready;
            }
            for (Chunk *c : run) {
                bool was = false;
                for (auto &mv : moved) was = was || mv.first == c;
                if (!was) c->dev_valid = false;
            }
            mem->merge(f);
            note_resident(ctx);
            return LT_OK;
        }
    }
    // evict every resident member and reload the run into one window
    for (Chunk *c : run)
        if (c->dev_off >= 0) {
            if (!c->dev_valid) {  // placed above but not loaded yet
                ctx->arena.release(c->dev_off, Fence());
                c->dev_off = -1;
                continue;
            }
            lt_status st = evict_chunk(ctx, c);
            if (st) return st;
        }
    int64_t total = 0;
    for (Chunk *c : run) total += c->bytes;
    int64_t rounded = round_up(total, 256);
    for (Chunk *c : run) c->pin--;
    int64_t off;
    Fence f;
    lt_status st = alloc_range(ctx, rounded, 1, nullptr, &off, &f);
    for (Chunk *c : run) c->pin++;
    if (st) return st;
    carve(ctx, off, rounded, run, f);
    for (Chunk *c : run) c->dev_valid = false;
    mem->merge(f);
    return LT_OK;
}

// Allocates every chunk of a device-home array as one contiguous range if it
// fits in free memory right now (no eviction).  Returns true on success.
bool alloc_slab(Ctx *ctx, Array *arr) {
    if (ensure_arena(ctx)) return false;
    int64_t total = 0;
    for (Chunk *c : arr->chunks) total += c->bytes;
    int64_t rounded = round_up(total, 256);
    Fence f;
    int64_t o = ctx->arena.take_free(rounded, &f, 1, nullptr);
    if (o < 0) return false;
    carve(ctx, o, rounded, arr->chunks, f);
    for (Chunk *c : arr->chunks) {
        c->dev_valid = true;
        c->data_ready = f;
        c->last_access = f;
    }
    note_resident(ctx);
    return true;
}

}  // namespace lt
