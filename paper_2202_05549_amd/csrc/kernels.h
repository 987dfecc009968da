// Interface between the executor and the hand-written HIP kernels.
//
// Every task (superblock) reaches its kernel as a KTask: the superblock's box
// of global thread indices plus one KView per array parameter.  A view's base
// address is pre-offset by the origin of the memory that backs the region
// (a chunk, a run of contiguous chunks, or a temporary), so that the kernel
// addresses elements with their GLOBAL array indices:
//     addr(i0, i1, i2) = base + (i0*s0 + i1*s1 + i2*s2) * sizeof(T).
// This is the paper's wrapper mechanism (Sec. 3.5: the block index is
// offset once, and array handles subtract the chunk offset once at
// construction, so element access costs nothing extra).  Kernels only touch
// elements inside the annotated region of each view.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lt {

constexpr int KMAXD = 3;
constexpr int KMAXARR = 6;   // array parameters per kernel
constexpr int KMAXG = 32;    // tasks per grouped dispatch
constexpr int KMAXP = 8;     // parameters per kernel

struct KView {
    int64_t base;            // byte address of element (0, 0, 0); may lie outside the allocation
    int64_t s[KMAXD];        // element strides
};

struct KTask {
    int64_t lo[KMAXD];       // superblock thread box, global indices, half-open
    int64_t hi[KMAXD];
    KView v[KMAXP];          // indexed by parameter number (scalars unused)
    // reduce(f) parameters whose body writes several partials per task
    // (one per workgroup slot, so float folds stay in a fixed order): the
    // element distance between consecutive slots; 0 = one slot
    int64_t slot[KMAXP];
};

struct KLaunch {
    hipStream_t stream;
    int ndim;
    int ntask;
    const KTask *tasks;
    int64_t iarg[KMAXP];     // int scalar parameters by parameter number
    double farg[KMAXP];
    int64_t block[KMAXD];    // logical block shape of the launch
    int variant;             // tuning variant (0 = default)
    int32_t rop[KMAXP];      // reduce(f) operator per parameter (ROp: 0 +, 1 *, 2 min, 3 max)
    const void *user;        // runtime-compiled kernels: their definition
};

typedef hipError_t (*KernelFn)(const KLaunch &);

// Built-in bodies (kernels.hip).
hipError_t launch_touch_i32(const KLaunch &);
hipError_t launch_stencil1d_f32(const KLaunch &);
hipError_t launch_jacobi2d_f32(const KLaunch &);
hipError_t launch_gemm_f32(const KLaunch &);
hipError_t launch_hist256_i32(const KLaunch &);
hipError_t launch_kmeans_assign_f32(const KLaunch &);
hipError_t launch_rowreduce_f32(const KLaunch &);
hipError_t launch_kmeans_update_f32(const KLaunch &);
hipError_t launch_kmeans_centres_f32(const KLaunch &);
// Runtime-compiled user kernels (rtc.cpp).
hipError_t launch_rtc(const KLaunch &);

// hist256 outside batches: one workgroup and one partial slot per 64 Ki
// elements of a task (at most 1024, at least one); each workgroup stores its
// whole 256-bin histogram into its slot, so no two workgroups add into the
// same words.  (One slot per 16 Ki elements measured slower at 2^24
// elements, 3.88 against 4.16 TB/s, and the same from 2^26 on.)
constexpr int64_t HIST_WG_SPAN = 65536;
constexpr int64_t HIST_MAXSLOTS = 1024;
inline int64_t hist_slots(const int64_t *lo, const int64_t *hi, const int64_t *iarg) {
    const int64_t e = (hi[0] < iarg[0] ? hi[0] : iarg[0]) - lo[0];
    if (e <= 0) return 1;
    const int64_t b = (e + HIST_WG_SPAN - 1) / HIST_WG_SPAN;
    return b < HIST_MAXSLOTS ? b : HIST_MAXSLOTS;
}
// k-means update: points per workgroup tile and the largest number of
// workgroups (= partial slots) per task.  A task of p points gets
// kmu_slots(p, d) workgroups; workgroup w takes tiles w, w + slots, ... in
// order and writes slot w, so the float folds never depend on scheduling.
// The cap is about as many workgroups as fit on the chip at once: 1024 for
// the bodies with one LDS copy per wave, 512 for d = 16 and 32, whose body
// keeps two copies per wave (two workgroups per CU).
constexpr int64_t KMU_TILE = 4096;
constexpr int64_t KMU_MAXSLOTS = 1024;
inline int64_t kmu_slot_cap(int64_t d) { return d == 16 || d == 32 ? 512 : KMU_MAXSLOTS; }
inline int64_t kmu_slots(int64_t points, int64_t d) {
    if (points <= 0) return 1;
    const int64_t t = (points + KMU_TILE - 1) / KMU_TILE, cap = kmu_slot_cap(d);
    return t < cap ? t : cap;
}
constexpr int KMU_MAXD = 32;
constexpr int KMU_MAXK = 256;
constexpr int KMU_MAXKD = 1536;   // K * d limit: four float64 copies stay under 64 KiB of LDS
// partial slots of a k-means update task over points [lo, min(hi, N))
inline int64_t kmeans_update_slots(const int64_t *lo, const int64_t *hi, const int64_t *iarg) {
    const int64_t end = hi[0] < iarg[0] ? hi[0] : iarg[0];
    return kmu_slots(end - lo[0], iarg[1]);
}

// Runtime helpers.
// Copies boxes of elements between device buffers: entry i copies ext[0] x
// ext[1] x ext[2] elements (last axis fastest) from src to dst with the given
// element strides.  One dispatch for many small pieces (halo refreshes).
struct CopyBoxEntry {
    int64_t src, dst;        // byte addresses of the first element
    int64_t ext[3];
    int64_t ss[3], ds[3];
};
hipError_t launch_copy_boxes(hipStream_t s, const CopyBoxEntry *table, int n, int esz, int64_t max_elems);

// Copies `bytes` bytes (a multiple of 16; both pointers 16-byte aligned)
// with a kernel of at most 64 workgroups, sized for the host link: 16-byte
// words, four in flight per lane.  The pointers may be device memory or
// pinned host memory (which kernels reach over the host link).  Returns
// hipErrorInvalidValue for other shapes.
hipError_t launch_copy_linear(hipStream_t s, void *dst, const void *src, int64_t bytes);

// Copies `rows` rows of `width` bytes (source and destination pitches in
// bytes) with a kernel of at most 64 workgroups, sized for the host link;
// either side may be device or pinned host memory.
hipError_t launch_copy_rows(hipStream_t s, void *dst, int64_t dpitch, const void *src, int64_t spitch,
                            int64_t width, int64_t rows);

// Sets `count` elements of size esz (1, 4 or 8 bytes) at dst to *value.
hipError_t launch_fill(hipStream_t s, void *dst, int64_t count, int esz,
                       const void *value);

// Reduction combine: target[e] = identity (+ or * or min or max) of every
// partial p whose box contains e, for e in box `u`.  Partials are dense boxes
// stored at part_base + part_off[p] elements.  `accumulate` = 1 starts from
// the target's current value instead of the identity.
struct CombinePart {
    int64_t off;             // element offset of the partial
    int64_t lo[KMAXD], hi[KMAXD];
    int64_t count;           // slots: dense copies of the box, back to back (0 or 1 = one)
};
constexpr int KMAXPART = 24;
struct CombineArgs {
    int ndim, dtype, op, accumulate;
    int64_t lo[KMAXD], hi[KMAXD];     // union box u
    KView target;
    int64_t part_base;               // byte address of the partial block
    int nparts;
    CombinePart parts[KMAXPART];
};
hipError_t launch_combine(hipStream_t s, const CombineArgs &a);
// Folds the slots of each part into its first slot in a fixed order: up to
// 16 runs of consecutive slots, each folded in slot order, then the runs in
// run order.
hipError_t launch_fold_slots(hipStream_t s, const CombineArgs &a);

}  // namespace lt

namespace lt {

// ------------------------------------------------------------ batched path
// A batch of tasks from many launches, drained by one persistent kernel.
// Work items are (task, tile) pairs handed out in program order by an atomic
// ticket; a task's tiles start once every dependency counter has reached its
// value.  counters[i] counts the finished tiles of task i; a task whose last
// tile finishes also bumps counters[signal] once.
enum DKind { DK_TOUCH = 0, DK_STENCIL1D = 1, DK_JACOBI2D = 2, DK_HIST256 = 3, DK_SUM_PARTIALS = 4 };
constexpr int DMAXDEP = 8;
constexpr int64_t DSPAN = 65536;  // elements per tile of the touch body (and default of the histogram's)
constexpr int64_t DTILE = 16384;  // default elements per tile of the stencil body
constexpr int DJROWS = 128;       // rows per Jacobi tile (marched in groups of 8)

struct DTask {
    int32_t kind;
    int32_t ntiles;
    int64_t tile_begin;
    int32_t ndeps;
    int32_t signal;                // -1 = none
    int32_t dep_ctr[DMAXDEP];
    int32_t dep_val[DMAXDEP];
    int64_t lo0, hi0, lo1, hi1;    // thread box (rows, columns) or range
    int64_t n, m;                  // scalar parameters
    int64_t y, x;                  // pre-offset views (output, input)
    int64_t ys, xs;                // row strides
    int32_t tx;                    // Jacobi column tiles
    int32_t vec;                   // Jacobi float4 layout
    int64_t aux;                   // DK_SUM_PARTIALS: number of partials
    int32_t flags;                 // DF_* below
    int32_t pad;
};

// DTask.flags: what a finished tile must do before counting itself done.
// DF_RELEASE: a later task of the batch reads this task's plain stores:
//   agent-scope release (write back this XCD's L2) before the count.
// DF_ATOMIC: every global write of the body is a device-scope atomic
//   (coherent across XCDs): waiting for their completion is enough.
// Tasks without consumers skip both.
constexpr int32_t DF_RELEASE = 1;
constexpr int32_t DF_ATOMIC = 2;

// counters: ntasks + nsignals task/signal counters, then the ticket, then an
// error flag (bit 0: a dependency wait gave up after spin_limit polls).
// kinds: bit k set when the queue holds a task of body DK k; the drain is
// built once per common set of bodies (a build that carries only the bodies
// it needs uses fewer registers, so more waves fit per SIMD)
// vectors: 16-byte vectors per lane per group of the streaming bodies (2 or
// 4; 0 = 4)
hipError_t launch_drain(hipStream_t s, const DTask *q, int ntasks, int32_t *counters, int ticket_idx,
                        int64_t total_tiles, int nwg, int64_t spin_limit, uint32_t kinds, int vectors);

// Fixed device scratch for issuing a batch without allocating: queue,
// counters and partials of one batch at a time.  drain_scratch_address
// returns its address on `device` (looked up once per device, with that
// device current; later calls return the kept address).
constexpr int64_t NOALLOC_SCRATCH_BYTES = (int64_t)32 << 20;
hipError_t drain_scratch_address(int device, void **out);

}  // namespace lt
