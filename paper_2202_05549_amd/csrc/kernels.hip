// Hand-written CDNA4 (gfx950) kernels for the built-in task bodies.
//
// Every body receives a table of tasks (superblocks).  A dispatch covers one
// or more tasks; each workgroup locates its task by a search over the
// per-task block offsets, then works on global indices through pre-offset
// views (the wrapper scheme of Sec. 3.5).  All float arithmetic is IEEE
// float32 with round-to-nearest; this file is built with -ffp-contract=off
// so no multiply-add is fused unless written as fmaf.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>

#include "bodies.h"
#include "kernels.h"

namespace lt {

using namespace body;

namespace {

inline unsigned grid_of(int64_t blocks) { return (unsigned)blocks; }

}  // namespace

// ==================================================================== touch
struct TouchTask {
    int64_t lo, hi;
    int64_t y;
};
struct TouchArgs {
    int64_t n;
    int ntask;
    int begin[KMAXG + 1];
    TouchTask t[KMAXG];
};

__global__ __launch_bounds__(256) void k_touch(TouchArgs a) {
    int ti = find_task(a.begin, a.ntask, blockIdx.x);
    const TouchTask &t = a.t[ti];
    touch_span(t.y, a.n, t.lo, t.hi, t.lo + (int64_t)(blockIdx.x - a.begin[ti]) * 256);
}

hipError_t launch_touch_i32(const KLaunch &L) {
    TouchArgs a;
    a.n = L.iarg[0];
    a.ntask = L.ntask;
    int64_t nb = 0;
    for (int i = 0; i < L.ntask; ++i) {
        a.begin[i] = (int)nb;
        a.t[i].lo = L.tasks[i].lo[0];
        a.t[i].hi = L.tasks[i].hi[0];
        a.t[i].y = L.tasks[i].v[1].base;
        nb += (a.t[i].hi - a.t[i].lo + 255) / 256;
    }
    a.begin[L.ntask] = (int)nb;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_touch, dim3(grid_of(nb)), dim3(256), 0, L.stream, a);
    return hipGetLastError();
}

// ================================================================ stencil1d
// y[i] = 0.25*(x[i-1] + x[i+1]) + 0.5*x[i], zero outside [0, n).
// Each thread produces 4 consecutive outputs; neighbours across lanes come
// from the adjacent lane's registers, the two wave-edge lanes load theirs.
struct StTask {
    int64_t lo, hi;
    int64_t y, x;
    int64_t span;     // outputs per workgroup: 1024 (one pass) or 8192 (streamed)
};
struct StArgs {
    int64_t n;
    int ntask;
    int begin[KMAXG + 1];
    StTask t[KMAXG];
};

// Small tasks (up to 2^21 outputs) take one span of 1024 outputs per
// workgroup, so even a 2^17-element chunk spreads over 128 workgroups;
// large ones stream 8192 outputs per workgroup with loads kept in flight,
// which measured faster for tasks of 2^24 elements.
__global__ __launch_bounds__(256) void k_stencil1d(StArgs a) {
    int ti = find_task(a.begin, a.ntask, blockIdx.x);
    const StTask &t = a.t[ti];
    const int64_t s0 = t.lo + (int64_t)(blockIdx.x - a.begin[ti]) * t.span;
    if (t.span == 1024) stencil_span(t.x, t.y, a.n, t.lo, t.hi, s0);
    else stencil_stream<4>(t.x, t.y, a.n, t.lo, t.hi, s0, s0 + t.span);
}

hipError_t launch_stencil1d_f32(const KLaunch &L) {
    StArgs a;
    a.n = L.iarg[0];
    a.ntask = L.ntask;
    int64_t nb = 0;
    for (int i = 0; i < L.ntask; ++i) {
        a.begin[i] = (int)nb;
        a.t[i].lo = L.tasks[i].lo[0];
        a.t[i].hi = L.tasks[i].hi[0];
        a.t[i].y = L.tasks[i].v[1].base;
        a.t[i].x = L.tasks[i].v[2].base;
        int64_t e = std::min(a.t[i].hi, a.n) - a.t[i].lo;
        a.t[i].span = e > (1 << 21) ? 8192 : 1024;
        nb += e > 0 ? (e + a.t[i].span - 1) / a.t[i].span : 0;
    }
    a.begin[L.ntask] = (int)nb;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_stencil1d, dim3(grid_of(nb)), dim3(256), 0, L.stream, a);
    return hipGetLastError();
}

// ================================================================= jacobi2d
// y[r][c] = 0.25*((x[r-1][c] + x[r+1][c]) + (x[r][c-1] + x[r][c+1])), zero
// outside the n x m field.  Each lane computes 4 adjacent columns and takes
// its horizontal neighbours from the adjacent lanes.  A workgroup owns a
// tile of either 1024 columns x RB rows (jacobi_tile, jacobi_march) or 256
// columns x 4 RB rows, one RB-row band per wave (jacobi_stack, the default).
struct JTask {
    JView v;
    int tx;           // column tiles
};
struct JArgs {
    int64_t n, m;
    int ntask, rows, nblocks;
    int begin[KMAXG + 1];
    JTask t[KMAXG];
};

template <int RB>
__global__ __launch_bounds__(256) void k_jacobi2d(JArgs a) {
    const int b = xcd_remap(blockIdx.x, a.nblocks);
    const int ti = find_task(a.begin, a.ntask, b);
    const JTask &t = a.t[ti];
    const int local = b - a.begin[ti];
    const int tyi = local / t.tx, txi = local - tyi * t.tx;
    jacobi_tile<RB>(t.v, a.n, a.m, t.v.r0 + (int64_t)tyi * RB, txi);
}

// Marching tiles of 8 NG rows (jacobi_march).
template <int NG>
__global__ __launch_bounds__(256) void k_jacobi2d_march(JArgs a) {
    const int b = xcd_remap(blockIdx.x, a.nblocks);
    const int ti = find_task(a.begin, a.ntask, b);
    const JTask &t = a.t[ti];
    const int local = b - a.begin[ti];
    const int tyi = local / t.tx, txi = local - tyi * t.tx;
    jacobi_march<NG>(t.v, a.n, a.m, t.v.r0 + (int64_t)tyi * 8 * NG, txi);
}

// Stacked tiles of 4 RB rows x 256 columns (jacobi_stack).
template <int RB>
__global__ __launch_bounds__(256) void k_jacobi2d_stack(JArgs a) {
    const int b = xcd_remap(blockIdx.x, a.nblocks);
    const int ti = find_task(a.begin, a.ntask, b);
    const JTask &t = a.t[ti];
    const int local = b - a.begin[ti];
    const int tyi = local / t.tx, txi = local - tyi * t.tx;
    jacobi_stack<RB>(t.v, a.n, a.m, t.v.r0 + (int64_t)tyi * 4 * RB, txi);
}

hipError_t launch_jacobi2d_f32(const KLaunch &L) {
    JArgs a;
    a.n = L.iarg[0];
    a.m = L.iarg[1];
    a.ntask = L.ntask;
    // tiles of 1024 columns and 8, 16 or 32 rows (all rows loaded at once),
    // or 32, 64 or 128 rows marched in groups of 8 (variants 132, 164, 228:
    // 100 + rows); or 256 columns and 4 waves of 2, 4 (default) or 8 rows
    // (variants 302, 304, 308: 300 + rows per wave)
    const bool march = L.variant == 132 || L.variant == 164 || L.variant == 228;
    const bool plain = L.variant == 8 || L.variant == 16 || L.variant == 32;
    const bool stack = !march && !plain;
    const int wrows = L.variant == 302 ? 2 : L.variant == 308 ? 8 : 4;
    a.rows = march ? L.variant - 100 : plain ? L.variant : 4 * wrows;
    const int64_t tcols = stack ? 256 : 1024;
    int64_t nb = 0;
    for (int i = 0; i < L.ntask; ++i) {
        const KTask &k = L.tasks[i];
        JTask &jt = a.t[i];
        JView &t = jt.v;
        t.r0 = k.lo[0];
        t.r1 = std::min(k.hi[0], a.n);
        t.c0 = k.lo[1];
        t.c1 = std::min(k.hi[1], a.m);
        t.y = k.v[2].base;
        t.x = k.v[3].base;
        t.ys = k.v[2].s[0];
        t.xs = k.v[3].s[0];
        t.vec = ((t.x + t.c0 * 4) & 15) == 0 && ((t.y + t.c0 * 4) & 15) == 0 && (t.xs & 3) == 0 &&
                (t.ys & 3) == 0 && ((t.c1 - t.c0) & 3) == 0;
        int64_t cols = t.c1 - t.c0, rows = t.r1 - t.r0;
        jt.tx = cols > 0 ? (int)((cols + tcols - 1) / tcols) : 0;
        int64_t ty = rows > 0 ? (rows + a.rows - 1) / a.rows : 0;
        a.begin[i] = (int)nb;
        nb += (int64_t)jt.tx * ty;
    }
    a.begin[L.ntask] = (int)nb;
    a.nblocks = (int)nb;
    if (nb == 0) return hipSuccess;
    if (stack) {
        if (wrows == 2)
            hipLaunchKernelGGL(k_jacobi2d_stack<2>, dim3(grid_of(nb)), dim3(256), 0, L.stream, a);
        else if (wrows == 8)
            hipLaunchKernelGGL(k_jacobi2d_stack<8>, dim3(grid_of(nb)), dim3(256), 0, L.stream, a);
        else
            hipLaunchKernelGGL(k_jacobi2d_stack<4>, dim3(grid_of(nb)), dim3(256), 0, L.stream, a);
    } else if (march) {
        if (a.rows == 32)
            hipLaunchKernelGGL(k_jacobi2d_march<4>, dim3(grid_of(nb)), dim3(256), 0, L.stream, a);
        else if (a.rows == 64)
            hipLaunchKernelGGL(k_jacobi2d_march<8>, dim3(grid_of(nb)), dim3(256), 0, L.stream, a);
        else
            hipLaunchKernelGGL(k_jacobi2d_march<16>, dim3(grid_of(nb)), dim3(256), 0, L.stream, a);
    } else if (a.rows == 8)
        hipLaunchKernelGGL(k_jacobi2d<8>, dim3(grid_of(nb)), dim3(256), 0, L.stream, a);
    else if (a.rows == 32)
        hipLaunchKernelGGL(k_jacobi2d<32>, dim3(grid_of(nb)), dim3(256), 0, L.stream, a);
    else
        hipLaunchKernelGGL(k_jacobi2d<16>, dim3(grid_of(nb)), dim3(256), 0, L.stream, a);
    return hipGetLastError();
}

// ================================================================ hist256
// Slot w of the superblock's partial = #{i in the workgroup's 4096-element
// groups (w, w + slots, ...) : v[i] == b} for every bin b.  Each wave counts into its own LDS
// sub-histograms (skewed data hammers few bins); the workgroup sums them and
// stores the whole slot, so no two workgroups add into the same words.  The
// slots are folded afterwards (integers: exact in any order).
struct HTask {
    int64_t lo, hi;
    int64_t h, v;
    int64_t slot;     // element distance between slots
};
// Stores the sum of the sub-histograms as the 256 bins at hb (no other
// workgroup writes them).
__device__ __forceinline__ void hist_store(int64_t hb, const int *sh) {
    __syncthreads();
    LT_GLOBAL int32_t *H = gp<int32_t>(hb);
    const int b = threadIdx.x;
    int s = 0;
#pragma unroll
    for (int k = 0; k < HIST_COPIES; ++k) s += sh[k * HIST_STRIDE + b];
    H[b] = s;
}

struct HArgs {
    int64_t n;
    int ntask;
    int per_task;
    int begin[KMAXG + 1];
    HTask t[KMAXG];
};

__global__ __launch_bounds__(256) void k_hist256(HArgs a) {
    __shared__ int sh[HIST_WORDS];
    int ti = find_task(a.begin, a.ntask, blockIdx.x);
    const HTask &t = a.t[ti];
    for (int i = threadIdx.x; i < HIST_WORDS; i += 256) sh[i] = 0;
    __syncthreads();
    const int64_t end = t.hi < a.n ? t.hi : a.n;
    const int w = blockIdx.x - a.begin[ti];
    const int nblk = a.begin[ti + 1] - a.begin[ti];
    hist_span(t.v, t.lo + (int64_t)w * 4096, end, (int64_t)nblk * 4096, sh);
    hist_store(t.h + (int64_t)w * t.slot * 4, sh);
}

hipError_t launch_hist256_i32(const KLaunch &L) {
    HArgs a;
    a.n = L.iarg[0];
    a.ntask = L.ntask;
    int64_t nb = 0;
    for (int i = 0; i < L.ntask; ++i) {
        a.t[i].lo = L.tasks[i].lo[0];
        a.t[i].hi = L.tasks[i].hi[0];
        a.t[i].h = L.tasks[i].v[1].base;
        a.t[i].v = L.tasks[i].v[2].base;
        a.t[i].slot = L.tasks[i].slot[1];
        // one workgroup per slot, as the planner sized the partial (every
        // slot is stored whole, empty tasks included)
        const int64_t blocks = hist_slots(L.tasks[i].lo, L.tasks[i].hi, L.iarg);
        if (blocks > 1 && a.t[i].slot <= 0) return hipErrorInvalidValue;
        a.begin[i] = (int)nb;
        nb += blocks;
    }
    a.begin[L.ntask] = (int)nb;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hist256, dim3(grid_of(nb)), dim3(256), 0, L.stream, a);
    return hipGetLastError();
}

// ========================================================== kmeans assign
// lab[p] = argmin_k sum_j (X[p][j] - C[k][j])^2 with the float32 chain
// acc = fmaf(d, d, acc) over j in order from 0, strict < (ties keep the
// smaller k).  Centres are staged in LDS once per workgroup.
struct KTaskK {
    int64_t lo, hi;
    int64_t lab, x, c;
    int64_t xs, cs;   // row strides
};
struct KArgs {
    int64_t N, d, K;
    int ntask;
    int begin[KMAXG + 1];
    KTaskK t[KMAXG];
};

constexpr int KM_MAXD = 32;
constexpr int KM_MAXK = 256;

template <int D>
__global__ __launch_bounds__(256) void k_kmeans(KArgs a) {
    __shared__ float cen[KM_MAXK * KM_MAXD];
    int ti = find_task(a.begin, a.ntask, blockIdx.x);
    const KTaskK &t = a.t[ti];
    const int d = D > 0 ? D : (int)a.d;
    const int K = (int)a.K;
    const LT_GLOBAL float *C = gp<const float>(t.c);
    for (int i = threadIdx.x; i < K * d; i += 256) cen[i] = C[(i / d) * t.cs + (i % d)];
    __syncthreads();
    const int64_t end = t.hi < a.N ? t.hi : a.N;
    int64_t p = t.lo + (int64_t)(blockIdx.x - a.begin[ti]) * 256 + threadIdx.x;
    if (p >= end) return;
    const LT_GLOBAL float *X = gp<const float>(t.x) + p * t.xs;
    float x[KM_MAXD];
#pragma unroll
    for (int j = 0; j < (D > 0 ? D : KM_MAXD); ++j)
        if (D > 0 || j < d) x[j] = X[j];
    float best = INFINITY;
    int arg = 0;
    for (int k = 0; k < K; ++k) {
        const float *ck = cen + k * d;
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < (D > 0 ? D : KM_MAXD); ++j) {
            if (D > 0 || j < d) {
                float df = x[j] - ck[j];
                acc = fmaf(df, df, acc);
            }
        }
        if (acc < best) {
            best = acc;
            arg = k;
        }
    }
    *at<int32_t>(t.lab, p) = arg;
}

// The same with the centres read through scalar loads into SGPRs (every lane
// of a wave needs the same centre value at the same time), not broadcast
// from LDS: a 16-byte LDS broadcast fills 1 KiB of VGPRs for 8 VALU
// instructions, and the four SIMDs of a CU share one LDS.  The centre loop
// is unrolled UK times (2: two centres' loads share one wait and their FMA
// chains interleave).  A lane takes PP points, 256 apart (a
// workgroup covers 256 PP points): each centre load then serves PP points,
// and their chains are independent.
template <int D, int PP, int UK>
__global__ __launch_bounds__(256) void k_kmeans_s(KArgs a) {
    const int ti = find_task(a.begin, a.ntask, blockIdx.x);
    const KTaskK &t = a.t[ti];
    const int K = (int)a.K;
    const int64_t end = t.hi < a.N ? t.hi : a.N;
    const int64_t p0 = t.lo + (int64_t)(blockIdx.x - a.begin[ti]) * (256 * PP) + threadIdx.x;
    if (p0 >= end) return;
    float x[PP][D];
#pragma unroll
    for (int u = 0; u < PP; ++u) {
        // a point past the end repeats the lane's first point (not stored)
        const int64_t p = p0 + u * 256 < end ? p0 + u * 256 : p0;
        const LT_GLOBAL float *X = gp<const float>(t.x) + p * t.xs;
#pragma unroll
        for (int j = 0; j < D; ++j) x[u][j] = X[j];
    }
    const LT_GLOBAL float *__restrict__ C = gp<const float>(t.c);
    const int64_t cs = t.cs;
    float best[PP];
    int arg[PP];
#pragma unroll
    for (int u = 0; u < PP; ++u) {
        best[u] = INFINITY;
        arg[u] = 0;
    }
#pragma unroll UK
    for (int k = 0; k < K; ++k) {
        const LT_GLOBAL float *ck = C + k * cs;
        float c[D];
#pragma unroll
        for (int j = 0; j < D; ++j) c[j] = ck[j];
#pragma unroll
        for (int u = 0; u < PP; ++u) {
            float acc = 0.f;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                float df = x[u][j] - c[j];
                acc = fmaf(df, df, acc);
            }
            if (acc < best[u]) {
                best[u] = acc;
                arg[u] = k;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < PP; ++u)
        if (p0 + u * 256 < end) *at<int32_t>(t.lab, p0 + u * 256) = arg[u];
}

hipError_t launch_kmeans_assign_f32(const KLaunch &L) {
    KArgs a;
    a.N = L.iarg[0];
    a.d = L.iarg[1];
    a.K = L.iarg[2];
    if (a.d < 1 || a.d > KM_MAXD || a.K < 1 || a.K > KM_MAXK) return hipErrorInvalidValue;
    a.ntask = L.ntask;
    // points per lane: 2 for variant 2 at d = 16, else 1
    const int pp = a.d == 16 && L.variant == 2 ? 2 : 1;
    int64_t nb = 0;
    for (int i = 0; i < L.ntask; ++i) {
        const KTask &k = L.tasks[i];
        a.t[i].lo = k.lo[0];
        a.t[i].hi = k.hi[0];
        a.t[i].lab = k.v[3].base;
        a.t[i].x = k.v[4].base;
        a.t[i].xs = k.v[4].s[0];
        a.t[i].c = k.v[5].base;
        a.t[i].cs = k.v[5].s[0];
        int64_t e = std::min(a.t[i].hi, a.N) - a.t[i].lo;
        a.begin[i] = (int)nb;
        nb += e > 0 ? (e + 256 * pp - 1) / (256 * pp) : 0;
    }
    a.begin[L.ntask] = (int)nb;
    if (nb == 0) return hipSuccess;
    // d = 4, 8, 16 and 32: centres in SGPRs, the centre loop unrolled by 2
    // (default); variant 1 broadcasts them from LDS (the earlier body); at
    // d = 16 variant 2 takes two points per lane
    if (pp == 2)
        hipLaunchKernelGGL((k_kmeans_s<16, 2, 1>), dim3(grid_of(nb)), dim3(256), 0, L.stream, a);
    else if (a.d == 16 && L.variant != 1)
        hipLaunchKernelGGL((k_kmeans_s<16, 1, 2>), dim3(grid_of(nb)), dim3(256), 0, L.stream, a);
    else if (a.d == 32 && L.variant != 1)
        hipLaunchKernelGGL((k_kmeans_s<32, 1, 2>), dim3(grid_of(nb)), dim3(256), 0, L.stream, a);
    else if (a.d == 8 && L.variant != 1)
        hipLaunchKernelGGL((k_kmeans_s<8, 1, 2>), dim3(grid_of(nb)), dim3(256), 0, L.stream, a);
    else if (a.d == 4 && L.variant != 1)
        hipLaunchKernelGGL((k_kmeans_s<4, 1, 2>), dim3(grid_of(nb)), dim3(256), 0, L.stream, a);
    else if (a.d == 16)
        hipLaunchKernelGGL(k_kmeans<16>, dim3(grid_of(nb)), dim3(256), 0, L.stream, a);
    else
        hipLaunchKernelGGL(k_kmeans<0>, dim3(grid_of(nb)), dim3(256), 0, L.stream, a);
    return hipGetLastError();
}

// ============================================================== copy boxes
// blockIdx.y = entry; threads stride over the entry's elements.
template <class T>
__global__ __launch_bounds__(256) void k_copy_boxes(const CopyBoxEntry *table) {
    const CopyBoxEntry &e = table[blockIdx.y];
    const int64_t n2 = e.ext[2], n1 = e.ext[1];
    const int64_t total = e.ext[0] * n1 * n2;
    const LT_GLOBAL T *S = gp<const T>(e.src);
    LT_GLOBAL T *D = gp<T>(e.dst);
    for (int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x; f < total; f += (int64_t)gridDim.x * 256) {
        const int64_t i2 = f % n2, r = f / n2;
        const int64_t i1 = r % n1, i0 = r / n1;
        D[i0 * e.ds[0] + i1 * e.ds[1] + i2 * e.ds[2]] = S[i0 * e.ss[0] + i1 * e.ss[1] + i2 * e.ss[2]];
    }
}

hipError_t launch_copy_boxes(hipStream_t s, const CopyBoxEntry *table, int n, int esz, int64_t max_elems) {
    if (n <= 0 || max_elems <= 0) return hipSuccess;
    if (n > 65535) return hipErrorInvalidValue;
    const int64_t bx = std::min<int64_t>((max_elems + 255) / 256, 64);
    const dim3 grid((unsigned)bx, (unsigned)n);
    if (esz == 4)
        hipLaunchKernelGGL(k_copy_boxes<uint32_t>, grid, dim3(256), 0, s, table);
    else if (esz == 8)
        hipLaunchKernelGGL(k_copy_boxes<uint64_t>, grid, dim3(256), 0, s, table);
    else if (esz == 1)
        hipLaunchKernelGGL(k_copy_boxes<uint8_t>, grid, dim3(256), 0, s, table);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// ============================================================ linear copy
// Copies over the host link (write-backs into pinned host memory) run on few
// workgroups: the link, not the compute units, is the limit, and a narrow
// grid leaves the CUs to the workload's kernels.  64 workgroups with four
// 16-byte loads in flight per lane reach the link rate for device-to-host
// copies (55 GB/s; 16 workgroups 53, 8 workgroups 47).
constexpr int COPY_WG = 64;
constexpr int COPY_U = 4;

__global__ __launch_bounds__(256) void k_copy16(int4 *__restrict__ dst, const int4 *__restrict__ src,
                                                int64_t words) {
    const int64_t stride = (int64_t)gridDim.x * 256 * COPY_U;
    for (int64_t base = (int64_t)blockIdx.x * 256 * COPY_U + threadIdx.x; base < words; base += stride) {
        int4 v[COPY_U];
#pragma unroll
        for (int u = 0; u < COPY_U; ++u) {
            const int64_t i = base + (int64_t)u * 256;
            if (i < words) v[u] = src[i];
        }
#pragma unroll
        for (int u = 0; u < COPY_U; ++u) {
            const int64_t i = base + (int64_t)u * 256;
            if (i < words) dst[i] = v[u];
        }
    }
}

hipError_t launch_copy_linear(hipStream_t s, void *dst, const void *src, int64_t bytes) {
    if (bytes <= 0) return hipSuccess;
    if ((bytes & 15) || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15)) return hipErrorInvalidValue;
    const int64_t words = bytes / 16;
    const int64_t blocks = std::min<int64_t>(COPY_WG, (words + 256 * COPY_U - 1) / (256 * COPY_U));
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, s, (int4 *)dst, (const int4 *)src, words);
    return hipGetLastError();
}

// Rows of `width` bytes: row r from src + r * spitch to dst + r * dpitch.
// Each row is cut into segments of at most 4096 T-sized words (16, 4 or 1
// bytes, the widest that every address, pitch and the width allow);
// workgroup b copies segments b, b + gridDim.x, ... of the rows x segments,
// with COPY_U loads in flight per lane.
template <class T>
__global__ __launch_bounds__(256) void k_copy_rows(char *__restrict__ dst, int64_t dpitch,
                                                   const char *__restrict__ src, int64_t spitch, int64_t words,
                                                   int64_t rows, int64_t segs) {
    for (int64_t b = blockIdx.x; b < rows * segs; b += gridDim.x) {
        const int64_t r = b / segs, w0 = (b - r * segs) * 4096;
        const int64_t w1 = w0 + 4096 < words ? w0 + 4096 : words;
        T *d = reinterpret_cast<T *>(dst + r * dpitch);
        const T *s = reinterpret_cast<const T *>(src + r * spitch);
        for (int64_t i0 = w0 + threadIdx.x; i0 < w1; i0 += 256 * COPY_U) {
            T v[COPY_U];
#pragma unroll
            for (int u = 0; u < COPY_U; ++u) {
                const int64_t i = i0 + (int64_t)u * 256;
                if (i < w1) v[u] = s[i];
            }
#pragma unroll
            for (int u = 0; u < COPY_U; ++u) {
                const int64_t i = i0 + (int64_t)u * 256;
                if (i < w1) d[i] = v[u];
            }
        }
    }
}

template <class T>
static void copy_rows_as(hipStream_t s, char *d, int64_t dpitch, const char *c, int64_t spitch, int64_t width,
                         int64_t rows) {
    const int64_t words = width / (int64_t)sizeof(T);
    const int64_t segs = (words + 4095) / 4096;
    const int64_t blocks = std::min<int64_t>(rows * segs, COPY_WG);
    hipLaunchKernelGGL(k_copy_rows<T>, dim3((unsigned)blocks), dim3(256), 0, s, d, dpitch, c, spitch, words, rows,
                       segs);
}

hipError_t launch_copy_rows(hipStream_t s, void *dst, int64_t dpitch, const void *src, int64_t spitch,
                            int64_t width, int64_t rows) {
    if (width <= 0 || rows <= 0) return hipSuccess;
    const uintptr_t all = (uintptr_t)dst | (uintptr_t)src | (uintptr_t)width |
                          (uintptr_t)(rows > 1 ? (dpitch | spitch) : 0);
    char *d = static_cast<char *>(dst);
    const char *c = static_cast<const char *>(src);
    if ((all & 15) == 0) copy_rows_as<int4>(s, d, dpitch, c, spitch, width, rows);
    else if ((all & 3) == 0) copy_rows_as<int>(s, d, dpitch, c, spitch, width, rows);
    else copy_rows_as<char>(s, d, dpitch, c, spitch, width, rows);
    return hipGetLastError();
}

// =================================================================== fill
template <class T>
__global__ __launch_bounds__(256) void k_fill(T *p, int64_t count, T v) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) p[i] = v;
}

hipError_t launch_fill(hipStream_t s, void *dst, int64_t count, int esz, const void *value) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = std::min<int64_t>((count + 255) / 256, 65536);
    if (esz == 4) {
        uint32_t v;
        std::memcpy(&v, value, 4);
        hipLaunchKernelGGL(k_fill<uint32_t>, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t *)dst, count, v);
    } else if (esz == 8) {
        uint64_t v;
        std::memcpy(&v, value, 8);
        hipLaunchKernelGGL(k_fill<uint64_t>, dim3((unsigned)blocks), dim3(256), 0, s, (uint64_t *)dst, count, v);
    } else if (esz == 1) {
        uint8_t v;
        std::memcpy(&v, value, 1);
        hipLaunchKernelGGL(k_fill<uint8_t>, dim3((unsigned)blocks), dim3(256), 0, s, (uint8_t *)dst, count, v);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lt
