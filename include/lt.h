/*
 * lt.h -- C ABI of the one-GPU annotated-launch runtime (MI355X, gfx950).
 *
 * The runtime implements the single-GPU share of the method of
 * "Lightning: Scaling the GPU Programming Model Beyond a Single GPU"
 * (Heldens et al., arXiv 2202.05549):
 *
 *   - a kernel launch is split into superblocks: disjoint boxes of thread
 *     blocks (Sec. 2.1 "Distributed Kernel Launches");
 *   - arrays of up to three dimensions are split into chunks by a
 *     distribution policy (Sec. 2.2 "Multi-Dimensional Distributed Arrays");
 *   - a data annotation states which elements each thread reads, writes or
 *     reduces (Sec. 2.3 "Data Annotations"); the planner turns it into one
 *     access region per superblock and array, resolves regions to chunks and
 *     adds dependency edges between tasks that conflict on a chunk
 *     (Sec. 2.4 "Execution Planner");
 *   - chunks live in device memory within a byte budget; least-recently used
 *     chunks are spilled to pinned host memory and reloaded with asynchronous
 *     copies that overlap kernels (Sec. 3.2, Sec. 3.4 "Memory Management").
 *
 * Conventions
 *   - Every call returns lt_status: LT_OK (0) or a negative error code.  After
 *     an error, lt_last_error(ctx) holds a message (owned by the context,
 *     valid until the next call on it).
 *   - Calls on one context are not thread-safe: one host thread drives a
 *     context, as the single driver program of Sec. 3.1 does.
 *   - Shapes and indices are int64 element counts.  Arrays are row-major: the
 *     last axis is contiguous.  Axis 0 is the slowest.
 *   - Boxes are half-open per axis: [lo, hi).
 *   - Launches are asynchronous and sequentially consistent: the result equals
 *     running the launches one after another, each over its whole grid
 *     (Sec. 1, Sec. 2.4).  Errors that happen on the device after a call has
 *     returned are sticky and reported by the next lt_sync / lt_wait /
 *     lt_array_read.
 */
#ifndef LT_H
#define LT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lt_status;

#define LT_OK 0
#define LT_ERR_INVALID (-1)     /* bad argument, handle, shape, dtype, arity   */
#define LT_ERR_PARSE (-2)       /* annotation syntax / non-affine / unknown name */
#define LT_ERR_BUDGET (-3)      /* one task needs more device bytes than the budget */
#define LT_ERR_OOM (-4)         /* host or device allocation failed            */
#define LT_ERR_DEVICE (-5)      /* a HIP call failed (message carries the text) */
#define LT_ERR_TIMEOUT (-6)     /* a bounded device wait gave up               */
#define LT_ERR_UNSUPPORTED (-7) /* valid request this build does not implement */
#define LT_ERR_COMPILE (-8)     /* runtime compilation of a user kernel failed
                                   (the compiler's log is in lt_last_error) */

typedef enum lt_dtype {
    LT_F32 = 0,
    LT_I32 = 1,
    LT_F64 = 2,
    LT_I64 = 3,
    LT_U8 = 4
} lt_dtype;

typedef struct lt_context lt_context;
typedef struct lt_array lt_array;
typedef struct lt_kernel lt_kernel;

/* ------------------------------------------------------------------ context
 * Execution modes for the tasks of a launch:
 *   LT_EXEC_PLAIN   one kernel dispatch per task (superblock).
 *   LT_EXEC_GROUPED consecutive tasks of one launch that have no edges among
 *                   each other and run on one stream share one dispatch; each
 *                   workgroup finds its task in a table passed by value.  The
 *                   arithmetic per element is identical to PLAIN.
 */
#define LT_EXEC_PLAIN 0
#define LT_EXEC_GROUPED 1

#define LT_EVICT_NEXT_USE 0
#define LT_EVICT_LRU 1

typedef struct lt_config {
    int32_t device;                 /* HIP device ordinal                      */
    int32_t n_compute_streams;      /* >= 1; default 1                          */
    int32_t exec_mode;              /* LT_EXEC_PLAIN or LT_EXEC_GROUPED         */
    int32_t dry_run;                /* 1: plan and simulate memory only; no
                                       device memory is touched, no kernel runs,
                                       array contents are unavailable          */
    uint64_t device_budget_bytes;   /* cap on device bytes held by chunks and
                                       temporaries (Sec. 3.4); default 8 GiB    */
    uint64_t stage_threshold_bytes; /* cap on the summed footprint of tasks
                                       staged ahead of execution (Sec. 3.4);
                                       default 2e9; one task is always admitted */
    void *device_arena;             /* optional borrowed device buffer to carve
                                       chunks from (e.g. a torch tensor); must
                                       outlive the context; NULL = the runtime
                                       allocates its own on first use           */
    uint64_t arena_bytes;           /* size of device_arena                     */
    int32_t trace;                  /* 1: record a per-operation trace          */
    int32_t sb_order;               /* superblock issue order of 2-D/3-D grids
                                       (the last two axes; earlier axes
                                       outermost): LT_ORDER_ROWMAJOR,
                                       LT_ORDER_SERPENTINE (odd rows of
                                       superblocks reversed, so consecutive
                                       rows reuse the chunks the previous row
                                       touched last) or LT_ORDER_BANDS (bands
                                       of sb_band rows, issued column by
                                       column with the rows of a column
                                       consecutive, odd bands reversed: a chunk
                                       that spans a column is used by sb_band
                                       superblocks in a row).  Changes traffic
                                       only, never results.                   */
    int32_t drain_workgroups;       /* workgroups of the batch drain kernel;
                                       0 = 1024                               */
    int32_t batch_flush_tasks;      /* an open batch issues its queue whenever
                                       it holds this many tasks, so planning
                                       of later launches overlaps the drain of
                                       earlier ones; 0 = only at lt_batch_end */
    int32_t drain_vectors;          /* 16-byte vectors per lane per group in
                                       the drain's streaming bodies (two groups
                                       are in flight): 2 (fewer registers, more
                                       waves) or 4; 0 = 4.  Changes speed
                                       only, never results.                   */
    int32_t evict_policy;           /* which chunks leave the device when the
                                       budget is full (Sec. 3.4 evicts the least
                                       recently used): LT_EVICT_NEXT_USE (0,
                                       default) prefers chunks that the tasks
                                       of the launch being issued need latest
                                       or never, then the least recently used;
                                       LT_EVICT_LRU (1) uses recency only.
                                       Changes traffic only, never results.   */
    int32_t sb_band;                /* LT_ORDER_BANDS: rows of superblocks per
                                       band, >= 0; 0 = 2                      */
    int32_t d2h_kernel;             /* write-backs into pinned home buffers of
                                       host-backed arrays: 0 (default) with
                                       hipMemcpy*Async, 1 with the library's
                                       row-copy kernel over the host link.
                                       Pageable homes always use
                                       hipMemcpy*Async.  Changes
                                       speed only.                            */
    uint64_t host_budget_bytes;     /* cap on the pinned host memory of spill
                                       buffers (chunks of device-home arrays
                                       evicted from the device); beyond it the
                                       least recently used ones move to a file
                                       in spill_dir (Sec. 3.4 disk tier);
                                       0 = no cap, no disk                     */
    const char *spill_dir;          /* directory of the spill file; NULL =
                                       $TMPDIR or /tmp.  The file is unlinked
                                       at creation and vanishes with the
                                       context.                                 */
    int64_t drain_tile;             /* batch drain: elements of a 1-D stencil or
                                       histogram task per ticket, a multiple of
                                       4096 (0 = 16384 for stencils, 65536 for
                                       histograms).  A task's tiles interleave
                                       its 4096-element groups.  Changes speed
                                       only, never results.                   */
} lt_config;

#define LT_ORDER_ROWMAJOR 0
#define LT_ORDER_SERPENTINE 1
#define LT_ORDER_BANDS 2

/* Fills *cfg with defaults. */
void lt_config_init(lt_config *cfg);

/* Creates a context on cfg->device.  cfg may be NULL (defaults).
 * Errors: LT_ERR_INVALID (bad config), LT_ERR_DEVICE (HIP init failed). */
lt_status lt_context_create(const lt_config *cfg, lt_context **out);

/* Waits for all work, releases every array, kernel and pool of the context.
 * Returns the first sticky error, if any. */
lt_status lt_context_destroy(lt_context *ctx);

/* Updates the tunable fields of a live context from *cfg: exec_mode,
 * stage_threshold_bytes, sb_order, sb_band, drain_workgroups, batch_flush_tasks,
 * trace.  Other fields are ignored.  Pending grouped work and an open batch's
 * queue are issued first.  Errors: LT_ERR_INVALID. */
lt_status lt_context_configure(lt_context *ctx, const lt_config *cfg);

/* Message of the last error on ctx; "" if none.  ctx may be NULL for errors
 * of lt_context_create. */
const char *lt_last_error(lt_context *ctx);

/* ------------------------------------------------------------ distributions
 * A distribution policy splits an array's domain into rectangular chunks
 * that cover it (Sec. 2.2):
 *   LT_DIST_BLOCK  chunks of chunk[a] elements along each axis a (0 = whole
 *                  axis): row-wise = {r, 0}, column-wise = {0, c},
 *                  tiled = {r, c}.  Edge chunks may be short.
 *   LT_DIST_CUSTOM nboxes explicit boxes; they must be disjoint, lie inside
 *                  the domain and cover it.
 *   LT_DIST_STENCIL the BLOCK cores of chunk[a], each stored with halo[a]
 *                  extra elements on both sides along axis a (clipped to the
 *                  domain), so neighbouring chunks overlap (Sec. 2.2).  Every
 *                  element is owned by the chunk whose core holds it; the
 *                  copies in other chunks' halos are replicas, kept coherent
 *                  by the runtime: a read whose region fits in one chunk's
 *                  stored box is served from that chunk alone, after any
 *                  replica older than its owner is refreshed from the owner
 *                  (a device-to-device copy of just those elements).  Writes
 *                  go to the owners' cores.  Results never depend on the
 *                  distribution (Sec. 2.4).  Along the last axis the stored
 *                  halo is rounded up to whole 16-byte words, so rows keep
 *                  the alignment of vector loads.
 */
#define LT_DIST_BLOCK 0
#define LT_DIST_CUSTOM 1
#define LT_DIST_STENCIL 2

typedef struct lt_box {
    int64_t lo[3];
    int64_t hi[3];
} lt_box;

typedef struct lt_dist {
    int32_t kind;
    int32_t nboxes;       /* LT_DIST_CUSTOM                          */
    int64_t chunk[3];     /* LT_DIST_BLOCK / _STENCIL; unused axes ignored */
    const lt_box *boxes;  /* LT_DIST_CUSTOM; copied at array creation */
    int64_t halo[3];      /* LT_DIST_STENCIL: halo width per axis (>= 0) */
} lt_dist;

/* ------------------------------------------------------------------- arrays
 * lt_array_create: a device-home array.  Its chunks live in device memory and
 *   spill to runtime-owned pinned host memory when the budget is exceeded.
 *   Contents are undefined until written or filled.  dist NULL = one chunk.
 * lt_array_create_host: a host-backed array whose home is the caller's
 *   buffer host_ptr (row-major, shape[] elements).  host_ptr is BORROWED for
 *   the array's lifetime.  Pinned buffers (lt_host_alloc) are copied
 *   asynchronously; chunks of a pageable buffer are packed by host threads
 *   into pinned bounce buffers and copied from there (the packing runs on the
 *   calling thread's time), and write-backs into a pageable buffer wait for
 *   their copy.  The buffer holds the array's contents after lt_sync; chunks
 *   are loaded on demand and written back when evicted.
 * Errors: LT_ERR_INVALID (ndim not in 1..3, shape <= 0, dtype, dist),
 *         LT_ERR_OOM, LT_ERR_BUDGET (creation of an array whose single chunk
 *         exceeds the device budget is allowed; launching on it is not).
 */
lt_status lt_array_create(lt_context *ctx, lt_dtype dtype, int32_t ndim,
                          const int64_t *shape, const lt_dist *dist,
                          lt_array **out);
lt_status lt_array_create_host(lt_context *ctx, lt_dtype dtype, int32_t ndim,
                               const int64_t *shape, const lt_dist *dist,
                               void *host_ptr, lt_array **out);

/* Releases the array once all launches issued before this call that use it
 * have completed (the release itself does not block). */
lt_status lt_array_destroy(lt_context *ctx, lt_array *arr);

/* Copies the whole array from host memory src (row-major).  Ordered after
 * earlier launches; src is fully consumed when the call returns. */
lt_status lt_array_write(lt_context *ctx, lt_array *arr, const void *src);

/* Copies the whole array into host memory dst (row-major).  Blocks until all
 * earlier launches that write the array have finished. */
lt_status lt_array_read(lt_context *ctx, lt_array *arr, void *dst);

/* Sets every element to *scalar (one element of the array's dtype). */
lt_status lt_array_fill(lt_context *ctx, lt_array *arr, const void *scalar);

/* Device-memory variants of write/read for arrays that live in device memory
 * elsewhere (e.g. a torch tensor): src/dst are device pointers to a
 * row-major buffer of the whole array.  Ordered like write/read; read blocks. */
lt_status lt_array_write_device(lt_context *ctx, lt_array *arr, const void *src);
lt_status lt_array_read_device(lt_context *ctx, lt_array *arr, void *dst);

/* Pinned host memory for host-backed arrays and fast transfers. */
lt_status lt_host_alloc(lt_context *ctx, uint64_t bytes, void **out);
lt_status lt_host_free(lt_context *ctx, void *ptr);

/* ------------------------------------------------------------------ kernels
 * Built-in kernels, each with its parameter list and default annotation
 * (the role of the kernel definition of Sec. 3.6).  Parameter names are what
 * annotations refer to.  Integer parameters are int64 scalars.
 *
 *   touch_i32(n, y)             global i => readwrite y[i]
 *       y[i] += 1 for i < n (exactly-once probe of the superblock split)
 *   stencil1d_f32(n, y, x)      global i => read x[i-1:i+1], write y[i]
 *       y[i] = 0.25*(x[i-1] + x[i+1]) + 0.5*x[i], zero outside [0, n)
 *   jacobi2d_f32(n, m, y, x)    global [r, c] => read x[r-1:r+1, c-1:c+1], write y[r, c]
 *       y = 0.25*((up + down) + (left + right)), zero outside the n x m field
 *   gemm_f32(M, N, K, C, A, B)  global [i, j] => read A[i, :], read B[:, j], write C[i, j]
 *       C = A B, FP32 inputs, FP32 matrix-core accumulation
 *   hist256_i32(n, h, v)        global i => read v[i], reduce(+) h[:]
 *       h[b] = #{i < n : v[i] == b}
 *   kmeans_assign_f32(N, d, K, lab, X, Cen)
 *                               global i => read X[i, :], read Cen[:, :], write lab[i]
 *       lab[i] = argmin_k sum_j (X[i,j] - Cen[k,j])^2, float32 fma chain,
 *       ties to the smallest k
 *   rowreduce_f32(n, m, out, A) global [i, j] => read A[i, j], reduce(+) out[i]
 *       out[i] = f over j of A[i, j], the reduction example of Sec. 2.3; f is
 *       the annotation's operator (+, *, min or max: define the kernel with
 *       e.g. "reduce(max) out[i]").  Each superblock folds its part of a row
 *       in float64 (min/max exact), rounds once to float32, and the partials
 *       of a row are folded in superblock order: the result depends on the
 *       superblock shape, never on scheduling or distributions.
 *   kmeans_update_f32(N, d, K, sums, counts, X, lab)
 *                               global i => read X[i, :], read lab[i],
 *                                           reduce(+) sums[:, :], reduce(+) counts[:]
 *       sums (float64 K x d) and counts (int32 K) of the points with each
 *       label (labels outside [0, K) are skipped): the centre update of the
 *       K-Means benchmark (Sec. 4.1).  Float64 folds in a fixed order, one
 *       partial slot per workgroup.  d <= 32, K <= 256, K*d <= 1536.
 *   kmeans_centres_f32(K, d, Cen, sums, counts)
 *                               global [k, j] => read sums[k, j], read counts[k], readwrite Cen[k, j]
 *       Cen[k, j] = sums[k, j] / counts[k] in float64 rounded once to
 *       float32; clusters with no points keep their centre
 *
 * lt_kernel_get: the built-in with its default annotation.
 * lt_kernel_define: the built-in body `base` under another annotation (it must
 *   still describe every access the body makes; an under-approximating
 *   annotation gives undefined results, as in the paper).
 * Errors: LT_ERR_INVALID (unknown name), LT_ERR_PARSE (annotation).
 */
lt_status lt_kernel_get(lt_context *ctx, const char *name, lt_kernel **out);
lt_status lt_kernel_define(lt_context *ctx, const char *base,
                           const char *annotation, lt_kernel **out);

/* ------------------------------------------------------------ user kernels
 * Runtime kernel compilation (Sec. 3.5 "Runtime Kernel Compilation").  The
 * caller supplies HIP source holding a __device__ function `function` whose
 * arguments are, in order: the virtual block index (a dim3), then one
 * argument per entry of params[]:
 *   LT_ARG_INT   an integer (passed as long long; declare any integer type)
 *   LT_ARG_FLOAT a number (passed as double; declare float or double)
 *   LT_ARG_ARRAY a view of an array of `dtype` with `ndim` axes:
 *                lt::Vector<T>, lt::Matrix<T> or lt::Tensor<T> for 1, 2, 3
 *                axes (T = float, int, double, long long, unsigned char),
 *                indexed with GLOBAL array indices: v[i], m(i, j) or m[i][j],
 *                t(i, j, k) or t[i][j][k]
 * This is the paper's porting recipe: a __global__ kernel becomes a
 * __device__ function, takes the block index as an argument (use it in
 * place of blockIdx; blockDim and threadIdx keep their meaning) and takes
 * views in place of raw pointers.  The grid's axes map to hardware axes
 * fastest first: a 1-D grid runs along x, the axes [i, j] of a 2-D grid
 * along (y, x), [i, j, k] along (z, y, x); block[] is given in the same
 * order as the grid.
 *
 * The runtime generates a wrapper kernel that finds the workgroup's
 * superblock, forms the virtual block index (the superblock's first block
 * plus the workgroup's block within it) and builds the views from base
 * addresses already moved by each region's origin, then calls the function.
 * The wrapper and the function are compiled together with hipRTC for gfx950
 * (-O3, no contraction of multiply-add, no packed FP32), with the block
 * shape, every view's strides and the values of scalars flagged
 * LT_PARAM_CONST baked in as constants: one compiled version per
 * combination, cached for the process, compiled at the first dispatch that
 * needs it.  Up to 16 superblocks share a dispatch in LT_EXEC_GROUPED mode.
 *
 * annotation: required; it names params[] entries and its bound index names
 * fix the rank of the launch grid (1..3).  The source is compiled once here
 * (block of 64, unit strides) so that its errors are reported now.
 * Planning, staging, spilling and reductions are those of built-in bodies;
 * a reduce(f) argument is a view of the superblock's partial, filled with
 * f's identity before the function runs.  User kernels cannot run inside a
 * batch (LT_ERR_UNSUPPORTED).  Blocks hold at most 1024 threads.
 * Errors: LT_ERR_INVALID (parameter list, function name), LT_ERR_PARSE
 * (annotation), LT_ERR_COMPILE (with the compiler's log).  A failure to
 * compile or load a later version is reported by the launch that needs it
 * (LT_ERR_DEVICE).  With the environment variable LT_RTC_DUMP=1 each
 * generated translation unit is printed to stderr before it is compiled. */
#define LT_PARAM_CONST 1
typedef struct lt_param {
    const char *name;   /* the name annotations use                    */
    int32_t kind;       /* LT_ARG_ARRAY / LT_ARG_INT / LT_ARG_FLOAT     */
    int32_t dtype;      /* arrays: element type (lt_dtype)              */
    int32_t ndim;       /* arrays: number of axes, 1..3                 */
    int32_t flags;      /* scalars: LT_PARAM_CONST bakes the value in   */
} lt_param;
lt_status lt_kernel_define_source(lt_context *ctx, const char *source, const char *function,
                                  const lt_param *params, int32_t nparams, const char *annotation,
                                  lt_kernel **out);

/* Process-wide counts of user-kernel versions compiled (including the check
 * build of each definition) and loaded onto a device, and the seconds spent
 * compiling. */
typedef struct lt_rtc_stats {
    uint64_t compiles;
    uint64_t loads;
    double compile_seconds;
} lt_rtc_stats;
lt_status lt_rtc_stats_get(lt_rtc_stats *out);

/* Selects a tuning variant of a built-in body for later launches through
 * this handle (0 = default).  Variants change only the work mapping, never
 * the per-element arithmetic (but see kmeans_update_f32 below for the order
 * of its float64 sums).  jacobi2d_f32 takes:
 *   8, 16 or 32: tiles of 1024 columns and that many rows, all loaded at once;
 *   132, 164 or 228: tiles of 1024 columns and 32, 64 or 128 rows, marched in
 *     groups of 8 (each input row loaded once per tile);
 *   302, 304 or 308: tiles of 256 columns and 4 bands of 2, 4 or 8 rows, one
 *     band per wave, the rows between bands exchanged on chip.
 * Unknown variants fall back to the default (304).  kmeans_assign_f32 at
 * d of 4, 8, 16 or 32 takes 1 to broadcast the centres from LDS instead of
 * reading them through scalar loads, and at d = 16 2 for two points per
 * lane; the labels are identical.  kmeans_update_f32 takes 1 for four features per lane (d of 16
 * or 32: the default there is one feature per lane with two LDS copies per
 * wave) and 2 for two features per lane (d of 8, 16 or 32).  Its variants
 * add each cell's points in different fixed orders: every variant gives the
 * same bits on every run, each within the float64 rounding bound of the
 * exact sums, but two variants may differ in the last bits. */
lt_status lt_kernel_tune(lt_context *ctx, lt_kernel *k, int32_t variant);

/* ------------------------------------------------------------------- launch */
#define LT_ARG_ARRAY 0
#define LT_ARG_INT 1
#define LT_ARG_FLOAT 2

typedef struct lt_arg {
    const char *name;   /* parameter name; NULL = positional          */
    int32_t kind;       /* LT_ARG_ARRAY / LT_ARG_INT / LT_ARG_FLOAT    */
    int32_t pad;
    lt_array *array;
    int64_t i;
    double f;
} lt_arg;

/* Launches kernel k over an ndim-D grid of grid[] threads (rounded up to
 * whole blocks of block[] threads), split into superblocks of superblock[]
 * threads (multiples of block[]; 0 = whole axis) (Sec. 2.1).  annotation
 * NULL = the kernel's own.  Returns immediately; *launch_id (may be NULL)
 * names the launch for lt_wait.
 * Errors (synchronous): LT_ERR_PARSE, LT_ERR_INVALID (grid/block/superblock,
 * arity, dtype, rank), LT_ERR_BUDGET (a task's chunks cannot all be held in
 * the device budget at once, Sec. 3.4). */
lt_status lt_launch(lt_context *ctx, lt_kernel *k, int32_t ndim,
                    const int64_t *grid, const int64_t *block,
                    const int64_t *superblock, const char *annotation,
                    const lt_arg *args, int32_t nargs, uint64_t *launch_id);

/* count launches in one call, exactly as count successive lt_launch calls:
 * launch i runs kernels[i] over grids[i*ndim ...] with blocks[i*ndim ...],
 * superblocks[i*ndim ...] (NULL = whole grid) and args[i*nargs ...]; all
 * launches share ndim, nargs and the annotation (NULL = each kernel's own).
 * launch_ids (may be NULL) receives count ids.  Stops at the first failing
 * launch and returns its error; the launches before it stay issued. */
lt_status lt_launch_many(lt_context *ctx, lt_kernel *const *kernels, int32_t count,
                         int32_t ndim, const int64_t *grids, const int64_t *blocks,
                         const int64_t *superblocks, const char *annotation,
                         const lt_arg *args, int32_t nargs, uint64_t *launch_ids);

/* Blocks until every issued launch has finished and host-backed arrays hold
 * their contents (Sec. 3.6 "synchronize").  Returns and clears the first
 * sticky device error. */
lt_status lt_sync(lt_context *ctx);

/* Blocks until launch `launch_id` has finished. */
lt_status lt_wait(lt_context *ctx, uint64_t launch_id);

/* ------------------------------------------------------------------ batching
 * lt_batch_begin opens a batch: later launches are planned as usual, but
 * their tasks become entries of a device task table instead of dispatches.
 * lt_batch_end (or any call that needs the results: lt_sync, lt_wait,
 * lt_array_read/write/fill/destroy) issues the table with one upload, one
 * clear of its counters and ONE persistent drain dispatch; the batch stays
 * open for further launches until lt_batch_end.  Edges between tasks of the
 * batch become counter waits inside the drain; edges to earlier work become
 * stream waits before it.  Results are identical to the unbatched path.
 * Supported bodies: touch_i32, stencil1d_f32, jacobi2d_f32, hist256_i32
 * (int32 reduce(+) with equal partial boxes).  Every chunk a batched task
 * touches must be resident: LT_ERR_UNSUPPORTED otherwise (and for other
 * bodies).  A dependency wait inside the drain that exceeds its poll limit
 * reports LT_ERR_TIMEOUT at the next lt_sync. */
lt_status lt_batch_begin(lt_context *ctx);
lt_status lt_batch_end(lt_context *ctx);

/* lt_batch_end without allocating, for callers that cannot allocate device
 * or pinned memory at this point (tight serving loops, code that runs
 * between allocation-free checkpoints).  It issues the open batch like
 * lt_batch_end, but the queue, counters and partials go to a fixed device
 * scratch of 32 MiB (one per GPU, held until the process ends) instead of an
 * arena range, so nothing is evicted; the queue is uploaded from the
 * planner's host copy instead of a pinned staging buffer; and the drain's
 * error flag reuses one of the context's preallocated slots (when all are
 * pending, the call first waits for compute stream 0).  No hipMalloc,
 * hipFree or hipHostMalloc is called.  Tasks that lt_launch issued before
 * (a batch that filled up, or launches that needed an earlier issue) went
 * through the usual path.  Errors, each leaving the batch open and
 * unissued (lt_batch_end can still issue it): LT_ERR_BUDGET if the batch
 * needs more than 32 MiB of scratch (192 bytes per task, 4 per counter, the
 * partials: about 160k tasks without partials), LT_ERR_DEVICE if the
 * scratch could not be found on the context's device, LT_ERR_UNSUPPORTED
 * for dry-run contexts; LT_ERR_INVALID while a graph is recorded.  A failure
 * of the issue itself is sticky until lt_sync, as for lt_batch_end.  Every
 * call on one GPU shares
 * that GPU's scratch and keeps its last contents (the counters are cleared
 * per call): calls from one context are ordered on its compute stream 0,
 * but calls from different contexts or processes on one GPU that overlap
 * in time race and give wrong results. */
lt_status lt_batch_end_noalloc(lt_context *ctx);

/* Graphs: a batch planned once and replayed.  lt_graph_begin opens a batch
 * whose queue is not issued; lt_graph_end turns it into a HIP graph (queue
 * upload, counter clear, drain) that owns its device queue and keeps every
 * chunk it touches pinned in HBM at its current place.  lt_graph_launch
 * replays it, ordered after earlier work on those chunks like any launch;
 * each replay recomputes the same tasks on the arrays' current contents.
 * lt_graph_destroy releases it (after its last replay completes).  Arrays a
 * graph uses cannot be destroyed while it exists (LT_ERR_INVALID). */
typedef struct lt_graph lt_graph;
lt_status lt_graph_begin(lt_context *ctx);
lt_status lt_graph_end(lt_context *ctx, lt_graph **out);
lt_status lt_graph_launch(lt_context *ctx, lt_graph *g);
lt_status lt_graph_destroy(lt_context *ctx, lt_graph *g);

/* ------------------------------------------------------------------ serving
 * A request loop with continuous batching on one context.  Requests are
 * queued by lt_server_submit and admitted in arrival order (or, with a
 * lookahead, cached datasets first) as soon as an active slot is free and
 * their device footprint fits next to the admitted ones (a request larger
 * than the budget is admitted alone and runs out of core through the memory
 * manager).  An admitted request's launches are
 * issued at once, so the work of all admitted requests overlaps on the
 * device.  Inputs are host-backed arrays over the caller's buffers, cached
 * per (kind, dataset, size): a later request on the same dataset finds its
 * chunks still in HBM unless they were spilled for other work.  Results are
 * written to the caller's output buffer; a request completes when they are
 * there.  lt_server_poll advances admission and reports completions without
 * blocking; lt_server_drain blocks until every submitted request is done.
 *
 * Request kinds (host buffers are row-major; pinned memory is faster):
 *   LT_REQ_JACOBI  n x n float32 field in0, `sweeps` Jacobi sweeps, out = the
 *                  final field (n x n float32)
 *   LT_REQ_KMEANS  N x d float32 points in0, K x d float32 centres in1,
 *                  out = N int32 labels (d <= 32, K <= 256)
 *   LT_REQ_GEMM    n x n float32 A in0 and B in1, out = C = A B (n x n)
 * Input buffers of a cached dataset must stay valid and unchanged while the
 * server lives. */
#define LT_REQ_JACOBI 0
#define LT_REQ_KMEANS 1
#define LT_REQ_GEMM 2

typedef struct lt_server lt_server;

typedef struct lt_server_config {
    int32_t max_active;        /* admitted requests at once (>= 1)            */
    int32_t keep_resident;     /* 1: cache dataset arrays across requests     */
    uint64_t admit_bytes;      /* cap on the summed footprint of admitted
                                  requests; 0 = the device budget            */
    int64_t chunk_rows;        /* row chunk / superblock for Jacobi and
                                  k-means (0 = 512 rows / 2^20 points)        */
    int64_t gemm_tile;         /* GEMM superblock edge (0 = 4096)            */
    int32_t lookahead;         /* 0: admit in arrival order.  k > 0: when a
                                  slot frees, the oldest of the first k queued
                                  requests whose dataset is already cached
                                  goes first (its inputs may still be in HBM),
                                  else the oldest that fits; a request passed
                                  over max_bypass times blocks admission
                                  until it is admitted                       */
    int32_t max_bypass;        /* with lookahead: 0 = 4 * lookahead          */
    int32_t reserved[2];
} lt_server_config;

typedef struct lt_request {
    int32_t kind;              /* LT_REQ_*                                   */
    int32_t dataset;           /* cache key with kind and size               */
    int64_t size;              /* n (Jacobi, GEMM) or N points (k-means)     */
    int64_t d, K;              /* k-means                                    */
    int32_t sweeps;            /* Jacobi                                     */
    int32_t pad;
    const void *in0, *in1;
    void *out;
} lt_request;

typedef struct lt_completion {
    uint64_t id;
    int32_t status;            /* LT_OK or the request's error               */
    int32_t kind;
    double t_submit, t_admit, t_done;   /* seconds, steady clock             */
    uint64_t footprint;
    int32_t cache_hit;         /* inputs were already cached                 */
    int32_t pad;
} lt_completion;

lt_status lt_server_create(lt_context *ctx, const lt_server_config *cfg, lt_server **out);
lt_status lt_server_submit(lt_server *srv, const lt_request *req, uint64_t *id);
lt_status lt_server_poll(lt_server *srv, lt_completion *out, int32_t cap, int32_t *n);
lt_status lt_server_drain(lt_server *srv, lt_completion *out, int32_t cap, int32_t *n);
lt_status lt_server_destroy(lt_server *srv);
/* Seconds on the clock that lt_completion times use. */
double lt_now(void);

/* ----------------------------------------------------------- introspection
 * Planner output of a launch, for tests and tools.  Task records are kept
 * until the next lt_sync. */
#define LT_TASK_EXEC 0
#define LT_TASK_COMBINE 1
#define LT_TASK_IO 2

typedef struct lt_task_info {
    uint64_t id;          /* global task number (program order)           */
    uint64_t launch;      /* launch id                                    */
    int32_t kind;         /* LT_TASK_*                                     */
    int32_t stream;       /* compute stream index it was issued on         */
    int32_t ndeps;        /* number of predecessor tasks                   */
    int32_t nregions;     /* number of (array, region) accesses            */
    int64_t sb_lo[3];     /* superblock thread box (EXEC)                  */
    int64_t sb_hi[3];
} lt_task_info;

typedef struct lt_region_info {
    int32_t arg;          /* kernel parameter index                        */
    int32_t mode;         /* 0 read, 1 write, 2 readwrite, 3 reduce         */
    int32_t op;           /* reduce op: 0 +, 1 *, 2 min, 3 max             */
    int32_t resolved;     /* 0 direct view, 1 assembled/scattered temp,
                             2 reduction partial                            */
    uint64_t array_id;
    int64_t lo[3];        /* clipped access region, half-open             */
    int64_t hi[3];
} lt_region_info;

lt_status lt_plan_tasks(lt_context *ctx, uint64_t launch_id,
                        lt_task_info *out, int32_t cap, int32_t *n);
lt_status lt_plan_regions(lt_context *ctx, uint64_t task_id,
                          lt_region_info *out, int32_t cap, int32_t *n);
lt_status lt_plan_deps(lt_context *ctx, uint64_t task_id, uint64_t *out,
                       int32_t cap, int32_t *n);

/* Unique id of an array (stable for its lifetime). */
uint64_t lt_array_id(lt_array *arr);

/* ------------------------------------------------------------------- stats */
typedef struct lt_stats {
    uint64_t launches, tasks, dispatches;
    uint64_t bytes_h2d, bytes_d2h, bytes_d2d;
    uint64_t copies_h2d, copies_d2h, copies_d2d;
    uint64_t evictions_clean, evictions_dirty;
    uint64_t resident_bytes, peak_resident_bytes;
    uint64_t staged_peak_bytes;    /* high-water mark of the staged footprint */
    uint64_t throttle_waits;
    uint64_t assembled_regions, direct_regions;
    double plan_seconds;           /* host time spent planning and issuing */
    uint64_t halo_copies;          /* replica refreshes of halo distributions */
    uint64_t bytes_disk_write;     /* spill buffers moved to the disk tier  */
    uint64_t bytes_disk_read;      /* ... and read back                      */
    uint64_t host_spill_bytes;     /* pinned spill memory held now          */
} lt_stats;

lt_status lt_stats_get(lt_context *ctx, lt_stats *out);
lt_status lt_stats_reset(lt_context *ctx);

/* ------------------------------------------------------------------- trace
 * With cfg.trace = 1 every device operation is recorded in order:
 * kind 0 kernel dispatch, 1 H2D, 2 D2H, 3 D2D, 4 fill, 5 evict (no copy),
 * 6 alloc, 7 free, 8 spill buffer written to the disk tier, 9 read back.  `task` is the task id (or ~0), `a`/`b` carry
 * kind-specific values (bytes, arena offset, chunk id), resident is the
 * device bytes held after the operation. */
typedef struct lt_trace_rec {
    int32_t kind;
    int32_t stream;
    uint64_t task;
    uint64_t chunk;
    uint64_t bytes;
    uint64_t offset;
    uint64_t resident;
} lt_trace_rec;

lt_status lt_trace_get(lt_context *ctx, lt_trace_rec *out, uint64_t cap,
                       uint64_t *n);
lt_status lt_trace_clear(lt_context *ctx);

/* ----------------------------------------------------------------- profile
 * With profiling on, every kernel dispatch is bracketed by timing events on
 * the stream it runs on; durations are summed per built-in body and collected
 * at lt_sync.  Batch drains are entered as "drain" and graph replays as
 * "graph" (the whole replay).  Meant for measurement runs (the events add a
 * little overhead).  lt_profile_enable(ctx, k): 0 off, 1 every dispatch, k > 1
 * every k-th dispatch of each body (a sample with 1/k of the overhead; the
 * returned counts and totals cover the sampled dispatches), -1 whole steps:
 * each stream's dispatches between two lt_sync calls are timed as one
 * interval, entered under the first body dispatched with the number of
 * dispatches in it (two events per stream and step instead of two per
 * dispatch; the average includes the gaps between the dispatches, and
 * copies are not timed).  Copies between
 * host and device memory are timed the same way, as "copy_h2d" and
 * "copy_d2h" (copy-engine copies and copy kernels alike).
 *
 * lt_profile_spans returns every timed operation since profiling was
 * enabled or reset, as (name, stream, start, end) on the device clock in
 * milliseconds from an event recorded then on compute stream 0 (starts
 * before it are negative): copy/compute overlap is measured from these
 * (Sec. 3.4 overlaps staging with execution).  Spans become available at
 * lt_sync; at most 2^22 are kept.
 */
typedef struct lt_kernel_prof {
    char name[32];
    uint64_t dispatches;
    double total_ms;      /* summed device time between the bracketing events */
    double max_ms;
} lt_kernel_prof;

typedef struct lt_span {
    char name[32];
    int32_t stream;       /* stream index: compute 0..n-1, then H2D, then D2H */
    int32_t pad;
    double start_ms, end_ms;
} lt_span;

lt_status lt_profile_enable(lt_context *ctx, int32_t on);
lt_status lt_profile_spans(lt_context *ctx, lt_span *out, uint64_t cap, uint64_t *n);
lt_status lt_profile_get(lt_context *ctx, lt_kernel_prof *out, int32_t cap,
                         int32_t *n);
lt_status lt_profile_reset(lt_context *ctx);

#ifdef __cplusplus
}
#endif
#endif /* LT_H */
