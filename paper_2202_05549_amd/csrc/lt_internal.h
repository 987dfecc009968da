// Internal data structures of the annotated-launch runtime.
//
// Planner side (no HIP dependency): boxes, affine index forms, compiled
// annotations, distributions and chunks, task records with their dependency
// edges.  Executor side: streams with sequence numbers, vector-clock fences,
// the device arena and the memory manager.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "lt.h"
#include "kernels.h"

namespace lt {

constexpr int MAXD = 3;
constexpr int MAXPARAM = 8;
constexpr int MAXSTREAM = 8;

// ------------------------------------------------------------------- boxes
// Half-open [lo, hi) per axis; unused axes are [0, 1).
struct Box {
    int64_t lo[MAXD] = {0, 0, 0};
    int64_t hi[MAXD] = {1, 1, 1};
    bool empty(int nd) const {
        for (int a = 0; a < nd; ++a)
            if (hi[a] <= lo[a]) return true;
        return false;
    }
    int64_t volume(int nd) const {
        int64_t v = 1;
        for (int a = 0; a < nd; ++a) v *= (hi[a] > lo[a] ? hi[a] - lo[a] : 0);
        return v;
    }
    bool contains(const Box &o, int nd) const {
        for (int a = 0; a < nd; ++a)
            if (o.lo[a] < lo[a] || o.hi[a] > hi[a]) return false;
        return true;
    }
    bool contains_point(const int64_t *p, int nd) const {
        for (int a = 0; a < nd; ++a)
            if (p[a] < lo[a] || p[a] >= hi[a]) return false;
        return true;
    }
    bool equals(const Box &o, int nd) const {
        for (int a = 0; a < nd; ++a)
            if (o.lo[a] != lo[a] || o.hi[a] != hi[a]) return false;
        return true;
    }
};

inline Box intersect(const Box &a, const Box &b, int nd) {
    Box r;
    for (int x = 0; x < nd; ++x) {
        r.lo[x] = a.lo[x] > b.lo[x] ? a.lo[x] : b.lo[x];
        r.hi[x] = a.hi[x] < b.hi[x] ? a.hi[x] : b.hi[x];
    }
    return r;
}

inline Box bbox_union(const Box &a, const Box &b, int nd) {
    Box r;
    for (int x = 0; x < nd; ++x) {
        r.lo[x] = a.lo[x] < b.lo[x] ? a.lo[x] : b.lo[x];
        r.hi[x] = a.hi[x] > b.hi[x] ? a.hi[x] : b.hi[x];
    }
    return r;
}

// ------------------------------------------------------------- annotations
enum Mode { M_READ = 0, M_WRITE = 1, M_RW = 2, M_REDUCE = 3 };
enum ROp { R_ADD = 0, R_MUL = 1, R_MIN = 2, R_MAX = 3 };

// Variable slots: kind * 3 + position, kind 0 = global, 1 = block, 2 = local.
constexpr int NVAR = 9;

// c0 + sum v[k] * var_k + sum p[q] * scalar_param_q
struct Affine {
    int64_t c0 = 0;
    int64_t v[NVAR] = {0};
    int64_t p[MAXPARAM] = {0};
    bool is_const() const {
        for (int k = 0; k < NVAR; ++k)
            if (v[k]) return false;
        for (int k = 0; k < MAXPARAM; ++k)
            if (p[k]) return false;
        return true;
    }
};

struct IndexSpec {
    bool has_lo = true, has_hi = true;  // slice bounds present (point: both)
    Affine lo, hi;                      // point: lo == hi
};

struct Access {
    Mode mode = M_READ;
    ROp op = R_ADD;
    int param = -1;                     // kernel parameter index (an array)
    std::vector<IndexSpec> idx;
};

struct Annotation {
    std::string text;
    int nbound[3] = {-1, -1, -1};       // names bound per kind (-1 = unbound)
    std::vector<Access> acc;
};

// ------------------------------------------------------------- kernel defs
enum ParamKind { P_ARRAY = 0, P_INT = 1, P_FLOAT = 2 };

struct ParamDef {
    const char *name;
    ParamKind kind;
    lt_dtype dtype;  // arrays
    int ndim;        // arrays: required rank
};

struct KernelDef {
    const char *name;
    const char *annotation;
    int nparam;
    ParamDef params[MAXPARAM];
    int grid_ndim;          // rank of the launch grid the body expects
    KernelFn fn;            // host launcher
    int max_group;          // tasks per grouped dispatch
    int dkind;              // body id in the batch drain (DK_*), -1 = not batchable
    // partial slots per task of a reduce parameter (nullptr = 1): a body that
    // folds floats over several workgroups writes one partial per workgroup
    int64_t (*slots)(const int64_t *lo, const int64_t *hi, const int64_t *iarg);
    // the body writes every element of every partial slot it is given
    // (empty tasks included), so partials need no identity fill
    bool slots_written = false;
    void *user = nullptr;   // the RtcKernel of a runtime-compiled user kernel
};

// H2D out of pageable home buffers (csrc/bounce.cpp): pinned bounce
// buffers of BOUNCE_BYTES in a ring of BOUNCE_BUFS, packed by BOUNCE_THREADS
// host threads (the caller included).
constexpr int64_t BOUNCE_BYTES = (int64_t)64 << 20;
constexpr int BOUNCE_BUFS = 4;
constexpr int BOUNCE_THREADS = 8;
struct BounceRing;

// A user kernel compiled at run time (csrc/rtc.cpp): its definition, the
// owned strings the definition points to, and its source.
struct RtcKernel {
    KernelDef def{};
    std::vector<std::string> names;
    std::string source, function;
    std::string source_key;           // source hash, function, parameter signature
    bool is_const[MAXPARAM] = {false};
    std::string last_error;           // compile/load/launch failure of the last dispatch
};

const KernelDef *find_builtin(const char *name);

}  // namespace lt

struct lt_kernel {
    const lt::KernelDef *def;
    std::shared_ptr<lt::Annotation> annot;
    int variant = 0;
};

namespace lt {

// ------------------------------------------------------------ fences/points
// A fence is a vector clock: for each stream the sequence number of the
// last operation that must have completed.
struct Fence {
    uint64_t s[MAXSTREAM] = {0};
    void merge(const Fence &o) {
        for (int i = 0; i < MAXSTREAM; ++i)
            if (o.s[i] > s[i]) s[i] = o.s[i];
    }
    void add(int stream, uint64_t seq) {
        if (seq > s[stream]) s[stream] = seq;
    }
};

using Array = ::lt_array;  // declared in lt.h, defined below

// ------------------------------------------------------------------ chunks
struct Chunk;

// One piece of a chunk's halo: the elements `box` (inside the chunk's stored
// box) are owned by chunk k; `ver` is the version of k they hold.
struct HaloSrc {
    Chunk *k = nullptr;
    Box box;
    uint64_t ver = 0;
    bool valid = true;   // false: the piece holds no copy at all (never loaded)
};

struct Chunk {
    uint64_t id = 0;
    Array *arr = nullptr;
    int index = 0;
    Box box;                   // stored elements (the core plus any halo)
    Box core;                  // owned elements; the cores of an array's chunks partition it
    int64_t elems = 0, bytes = 0;
    // halo coherence (Sec. 2.2 overlapping distributions): version counts the
    // writes of the core; host_version is the version in the host copy's core
    uint64_t version = 0, host_version = 0;
    std::vector<HaloSrc> halo;

    // device copy
    int64_t dev_off = -1;      // arena offset; -1 = not allocated
    int64_t dev_stride[MAXD];  // element strides of the device copy
    bool dev_valid = false;
    // host copy (home for host-backed arrays; spill copy otherwise)
    char *host_ptr = nullptr;  // address of element box.lo
    int64_t host_stride[MAXD] = {0, 0, 0};
    bool host_owned = false;   // runtime-allocated pinned spill buffer
    int64_t disk_off = -1;     // offset of the chunk's slot in the spill file (-1 = none)
    bool disk_valid = false;   // the spill file slot holds the current host copy
    bool host_valid = false;
    bool defined = false;      // holds data written by someone (else undefined)

    // access history for conflict analysis (task ids; program order)
    uint64_t last_writer = 0;  // 0 = none
    std::vector<uint64_t> readers;
    std::vector<uint64_t> reducers;
    int reduce_op = -1;

    Fence data_ready;   // the device copy holds valid data after this
    Fence last_access;  // every device-side use so far
    Fence host_ready;   // host copy complete (after a write-back or a read from the spill file)
    Fence disk_ready;   // the spill file slot is written (the write is a host function on the D2H stream)
    uint64_t lru = 0;
    int pin = 0;

    // the tasks (indices within the launch being issued) that will use this
    // chunk, in order; valid while fut_launch is that launch
    std::vector<int32_t> fut;
    size_t fut_pos = 0;
    uint64_t fut_launch = ~0ull;
};

// ------------------------------------------------------------------ arrays
}  // namespace lt

constexpr uint32_t LT_ARRAY_MAGIC = 0x4c544152u;

struct lt_array {
    uint32_t magic = LT_ARRAY_MAGIC;
    void *owner = nullptr;   // the context
    uint64_t id = 0;
    lt_dtype dtype = LT_F32;
    int esz = 4;
    int ndim = 1;
    int64_t shape[lt::MAXD] = {1, 1, 1};
    int64_t strides[lt::MAXD] = {1, 1, 1};
    bool host_backed = false;
    char *host_base = nullptr;
    bool home_pinned = false;  // host_base is pinned memory kernels can address directly
    bool row_slab = false;   // every chunk spans full trailing axes
    bool has_halo = false;   // chunks store a halo around their core (LT_DIST_STENCIL)
    int64_t halo[lt::MAXD] = {0, 0, 0};
    int dist_kind = LT_DIST_BLOCK;
    int64_t dist_chunk[lt::MAXD] = {0, 0, 0};  // BLOCK
    int64_t nch[lt::MAXD] = {1, 1, 1};         // BLOCK: chunks per axis
    std::vector<lt::Chunk *> chunks;
    bool dead = false;
};

struct lt_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t off = -1;                  // arena range holding queue, counters, partials
    void *staging = nullptr;           // pinned copy of the queue
    int32_t *status = nullptr;         // pinned error flag
    std::vector<lt::Chunk *> chunks;   // chunks it touches (pinned while it lives)
    std::vector<char> writes;
    int stream = 0;
    uint64_t last = 0;                 // seq of its last replay on `stream`
    int ntasks = 0;
};

namespace lt {

// ------------------------------------------------------------------- tasks
struct RegionRec {
    lt_region_info info;
};

struct TaskRec {
    uint64_t id = 0, launch = 0;
    int kind = LT_TASK_EXEC;
    int stream = 0;
    uint64_t seq = 0;                  // completion point on `stream`
    Box sb;
    std::vector<uint64_t> deps;
    std::vector<lt_region_info> regions;
};

// Records keyed by sequential ids (tasks, launches), dropped at lt_sync.
template <class T>
struct IdTable {
    uint64_t base = 1;
    std::deque<T> v;
    T *get(uint64_t id) { return (id >= base && id < base + v.size()) ? &v[id - base] : nullptr; }
    T &at(uint64_t id) {
        while (base + v.size() <= id) v.emplace_back();
        return v[id - base];
    }
    void reset(uint64_t next) {
        v.clear();
        base = next;
    }
};

struct LaunchRec {
    std::vector<uint64_t> tasks;
    Fence done;
};

// --------------------------------------------------------------- streams
struct Mark {
    uint64_t seq;
    hipEvent_t ev;
};

struct Stream {
    hipStream_t h = nullptr;
    uint64_t seq = 0;                  // operations issued
    uint64_t done = 0;                 // operations known to have completed
    std::deque<Mark> marks;            // events recorded at given seqs
    uint64_t waited[MAXSTREAM] = {0};  // highest seq of other streams waited on
    // step profiling (lt_profile_enable(ctx, -1)): the event before the
    // stream's first dispatch since the last sync, its body and the count
    hipEvent_t step_a = nullptr;
    const char *step_name = nullptr;
    uint64_t step_count = 0;
};

// ------------------------------------------------------------- the arena
struct Seg {
    int64_t off = 0, size = 0;
    int kind = 0;                      // 0 free, 1 chunk, 2 temporary
    Chunk *chunk = nullptr;
    Fence fence;                       // free: memory reusable after this
};

struct TraceSink;

struct Arena {
    int64_t capacity = 0;
    std::map<int64_t, Seg> segs;       // covers [0, capacity)
    std::multimap<int64_t, int64_t> free_by_size;  // free segments: size -> offset
    int64_t used = 0, peak = 0;
    void index_add(const Seg &s) { free_by_size.insert({s.size, s.off}); }
    void index_del(const Seg &s) {
        auto r = free_by_size.equal_range(s.size);
        for (auto it = r.first; it != r.second; ++it)
            if (it->second == s.off) {
                free_by_size.erase(it);
                return;
            }
    }
    void init(int64_t cap);
    // best fit among free segments; returns offset or -1
    int64_t take_free(int64_t size, Fence *fence_out, int kind, Chunk *owner);
    // takes [off, off+size) if a free segment covers it; returns off or -1
    int64_t take_at(int64_t off, int64_t size, Fence *fence_out, int kind, Chunk *owner);
    void release(int64_t off, const Fence &fence);
    Seg *find(int64_t off);
    int64_t largest_free() const;
};

// ------------------------------------------------------------ open group
// Tasks of one launch collected for a single grouped dispatch.
struct ChunkUse {
    Chunk *c;
    bool write;
};

struct Batch {
    bool open = false;                 // between lt_batch_begin and lt_batch_end
    bool capture = false;              // building a graph: never issued directly
    std::vector<DTask> q;
    std::vector<uint64_t> ids;         // task id of each queue entry
    uint64_t index_base = 0;           // queue index of task id: index[id - index_base]
    std::vector<int> index;
    std::vector<uint64_t> launches;    // launches with tasks in this batch
    int find(uint64_t id) const {
        if (index.empty() || id < index_base || id - index_base >= index.size()) return -1;
        return index[id - index_base];
    }
    std::vector<std::pair<int, int64_t>> patch_y, patch_x;  // partial-relative views
    int64_t part_bytes = 0;
    int nsignals = 0;
    int64_t tiles = 0;
    uint32_t kinds = 0;                // bit k set: a task of body DK k is queued
    // every chunk a queued task touches, one entry per use; each entry holds
    // a pin on its chunk until the batch is issued or dropped, so that no
    // allocation made meanwhile (the batch's own queue area, halo tables)
    // evicts memory that a queued task addresses directly
    std::vector<ChunkUse> uses;
    std::unordered_set<Chunk *> written;  // chunks a queued task writes
    Fence wait;                        // dependencies issued before the batch
};

struct Group {
    bool open = false;
    uint64_t launch = 0;
    const KernelDef *def = nullptr;
    int stream = 0;
    KLaunch proto;
    std::vector<KTask> tasks;
    std::vector<uint64_t> ids;
    std::vector<ChunkUse> uses;
    Fence wait;
};

}  // namespace lt

struct lt_context {
    lt_config cfg;
    std::string err;
    int ncompute = 1;
    int h2d = 1, d2h = 2;              // stream indices
    int nstreams = 3;
    lt::Stream streams[lt::MAXSTREAM];
    std::vector<hipEvent_t> event_pool;
    bool dry = false;

    // memory
    lt::Arena arena;
    char *arena_base = nullptr;
    bool arena_owned = false;
    uint64_t lru_clock = 0;
    bool budget_binds = false;    // a chunk has been evicted (sticky)
    uint64_t cur_launch = ~0ull;  // launch whose tasks are being issued
    int32_t cur_task = 0;         // index of the task being issued in it
    // disk tier: pinned spill memory in use, the spill file and its next free slot
    int64_t host_spill_bytes = 0;
    // recycled pinned spill buffers by size, each free for a new owner once
    // its fence has passed (a pending spill file write may still read it)
    struct PooledPin {
        char *p;
        lt::Fence ready;
    };
    std::multimap<int64_t, PooledPin> pin_pool;
    int64_t pin_pooled = 0;
    int spill_fd = -1;
    // first error of a spill file read or write, set by the host functions
    // that run them: errno, and 1 for a read or 2 for a write
    std::atomic<int> disk_errno{0};
    std::atomic<int> disk_errop{0};
    int64_t disk_next = 0;
    std::string spill_dir;             // copy of cfg.spill_dir

    // objects
    uint64_t next_array_id = 1, next_chunk_id = 1, next_task_id = 1;
    uint64_t next_launch_id = 1;
    std::vector<lt::Array *> arrays;
    std::vector<std::unique_ptr<lt_kernel>> kernels;
    std::vector<std::unique_ptr<lt::RtcKernel>> rtc_kernels;
    std::unordered_map<std::string, std::shared_ptr<lt::Annotation>> annot_cache;

    // planner records (kept until lt_sync)
    lt::IdTable<lt::TaskRec> tasks;
    lt::IdTable<lt::LaunchRec> launches;

    // throttle: staged tasks (completion point, footprint)
    std::deque<std::pair<lt::Fence, int64_t>> staged;
    int64_t staged_bytes = 0;

    // sticky asynchronous error
    lt_status sticky = LT_OK;
    std::string sticky_msg;

    lt_stats stats;
    std::vector<lt_trace_rec> trace;
    int rr = 0;                        // round-robin compute stream
    lt::Group group;                   // tasks awaiting one grouped dispatch
    lt::Batch batch;                   // tasks awaiting the drain kernel
    std::vector<void *> staging_free, staging_used;   // pinned upload buffers
    std::vector<uint64_t> staging_size_free, staging_size_used;
    int32_t *status_host = nullptr;    // drain error flags copied back
    std::vector<int32_t *> graph_status;  // error flags of live graphs
    int status_slots = 0, status_next = 0;
    // the device scratch of lt_batch_end_noalloc on this context's device
    // (looked up at creation; null with scratch_err set if that failed)
    void *scratch = nullptr;
    hipError_t scratch_err = hipSuccess;
    lt::BounceRing *bounce = nullptr;  // created at the first copy out of a pageable home

    // profiling: (kernel name, start, end) awaiting resolution
    int prof = 0;                      // 0 off; k: every k-th dispatch of each body is timed
    std::map<std::string, uint64_t> prof_seen;
    struct ProfPending {
        const char *name;
        hipEvent_t a, b;
        int stream;
        uint64_t count;                // dispatches between a and b
    };
    std::vector<ProfPending> prof_pending;
    std::map<std::string, lt_kernel_prof> prof_acc;
    hipEvent_t prof_base = nullptr;    // time origin of the spans (recorded at enable / reset)
    std::vector<lt_span> prof_spans;   // every timed operation since, on the device clock
    std::vector<hipEvent_t> prof_pool;
    std::vector<void *> host_allocs;
};

namespace lt {
using Ctx = lt_context;

// annotation compiler (annot.cpp)
lt_status compile_annotation(Ctx *ctx, const KernelDef *def, const char *text,
                             std::shared_ptr<Annotation> *out);

// planner helpers (plan.cpp)
struct VarRange {
    int64_t lo[NVAR], hi[NVAR];
};
void var_ranges(int nd, const int64_t *blk_lo, const int64_t *blk_hi,
                const int64_t *block, VarRange *r);
bool access_region(const Access &a, int nd_grid, const int64_t *block,
                   const VarRange &vr, const int64_t *params, const Array *arr,
                   Box *out);
lt_status make_chunks(Ctx *ctx, Array *arr, const lt_dist *dist);
// chunks whose core intersects r (the owners of r's elements)
void chunks_overlapping(const Array *arr, const Box &r, std::vector<Chunk *> *out);
// halo arrays: a chunk whose stored box (core plus halo) contains r, or null
Chunk *enclosing_chunk(const Array *arr, const Box &r);
// halo pieces of c inside `region` that hold an older version than their owner
bool halo_stale(const Chunk *c, const Box &region);

// executor (exec.cpp)
lt_status launch(Ctx *ctx, lt_kernel *k, int nd, const int64_t *grid,
                 const int64_t *block, const int64_t *sb, const char *annotation,
                 const lt_arg *args, int nargs, uint64_t *launch_id);
lt_status sync_all(Ctx *ctx);
lt_status flush_group(Ctx *ctx);
lt_status batch_flush(Ctx *ctx);
lt_status batch_flush_noalloc(Ctx *ctx);
void fold_drain_status(Ctx *ctx);
// Copies a box from pageable host memory to the device through the bounce
// ring (same arguments as copy_box with kind H2D); bounce_release frees it.
lt_status bounce_h2d(Ctx *ctx, int stream, char *dst, const int64_t *ds, const char *src, const int64_t *ss,
                     const int64_t *ext, int nd, int esz);
void bounce_release(Ctx *ctx);
lt_status rtc_define(Ctx *ctx, const char *source, const char *function, const lt_param *params, int32_t nparams,
                     const char *annotation, lt_kernel **out);
const char *rtc_last_error(const KernelDef *def);
void rtc_counters(uint64_t *compiles, uint64_t *loads, double *compile_s);
// Releases the pins of the queued tasks and empties the batch (it stays
// open if it was).
void batch_drop(Ctx *ctx);
lt_status graph_end(Ctx *ctx, lt_graph **out);
lt_status graph_launch(Ctx *ctx, lt_graph *g);
lt_status graph_destroy(Ctx *ctx, lt_graph *g);
lt_status flush_all(Ctx *ctx);
lt_status prof_begin(Ctx *ctx, int s, const char *name, hipEvent_t *a);
lt_status prof_end(Ctx *ctx, int s, const char *name, hipEvent_t a);
void prof_collect(Ctx *ctx);
// step profiling: closes every stream's open interval (before a sync)
lt_status prof_close_steps(Ctx *ctx);
lt_status wait_fence(Ctx *ctx, const Fence &f);
bool fence_done(Ctx *ctx, const Fence &f);
lt_status array_flush_async(Ctx *ctx, Array *arr, Fence *out);
lt_status array_ready_fence(Ctx *ctx, Array *arr, Fence *out);
lt_status array_write(Ctx *ctx, Array *arr, const void *src, bool device_src);
lt_status array_read(Ctx *ctx, Array *arr, void *dst, bool device_dst);
lt_status array_fill(Ctx *ctx, Array *arr, const void *scalar);
lt_status array_destroy(Ctx *ctx, Array *arr);
lt_status ensure_arena(Ctx *ctx);
void ctx_release_all(Ctx *ctx);

// memory manager and streams (memory.cpp)
uint64_t bump(Ctx *ctx, int stream);
lt_status stream_wait(Ctx *ctx, int stream, const Fence &f);
// Records an event at stream s's current end, so that a later wait for what
// has been issued so far waits for exactly that and not for work issued after.
lt_status mark_tail(Ctx *ctx, int s);
// by_kernel: a copy kernel instead of the copy engine (both sides must be
// reachable by kernels: device or pinned host memory)
lt_status copy_box(Ctx *ctx, int stream, char *dst, const int64_t *ds,
                   const char *src, const int64_t *ss, const int64_t *ext,
                   int nd, int esz, hipMemcpyKind kind, bool by_kernel = false);
// copies the elements `sub` between two buffers holding boxes with origins
// dlo / slo and element strides ds / ss
lt_status copy_sub(Ctx *ctx, int stream, char *dst, const int64_t *dlo, const int64_t *ds, const char *src,
                   const int64_t *slo, const int64_t *ss, const Box &sub, int nd, int esz, hipMemcpyKind kind,
                   bool by_kernel = false);
// D2H of a dirty chunk to its host copy on the D2H stream (after its data is
// ready): the core for host-backed arrays (the halo belongs to other
// chunks), the whole stored box for spill buffers.  Returns the D2H seq.
lt_status write_back(Ctx *ctx, Chunk *c, uint64_t *seq);
// brings the halo pieces of c that `region` touches up to their owners'
// versions (copies on the H2D stream); c must be valid on the device
lt_status refresh_halo(Ctx *ctx, Chunk *c, const Box &region);
lt_status alloc_range(Ctx *ctx, int64_t size, int kind, Chunk *owner,
                      int64_t *off, Fence *fence);
lt_status alloc_chunk(Ctx *ctx, Chunk *c, Fence *fence);
bool alloc_slab(Ctx *ctx, Array *arr);
lt_status place_run(Ctx *ctx, const std::vector<Chunk *> &run, Fence *mem);
lt_status evict_chunk(Ctx *ctx, Chunk *c);
lt_status ensure_host_copy(Ctx *ctx, Chunk *c);
// makes the host copy of c readable in memory (reads it back from the disk
// tier when it was moved there); call before using c->host_ptr as a source
lt_status host_resident(Ctx *ctx, Chunk *c);
// releases c's pinned spill buffer (and its disk slot stays reserved)
void free_spill(Ctx *ctx, Chunk *c);
// the first failed spill file read or write since the last call, as an error
lt_status disk_status(Ctx *ctx);
// Unpins every recycled spill buffer (context teardown).
void drain_pin_pool(Ctx *ctx);
char *dev_ptr(Ctx *ctx, const Chunk *c);
void trace_op(Ctx *ctx, int kind, int stream, uint64_t task, uint64_t chunk,
              uint64_t bytes, uint64_t offset);

lt_status set_err(Ctx *ctx, lt_status st, const char *fmt, ...);
lt_status hip_fail(Ctx *ctx, hipError_t e, const char *what);

}  // namespace lt
