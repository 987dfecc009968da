// Reductions: reduce(f) bodies, the slot fold and the combine (Sec. 2.3
// "reduce", Sec. 2.4: each superblock writes block-level partial results to
// a private temporary, which are then reduced level by level -- first within
// the superblock, then across superblocks).
//
// Float folds never use atomics.  Every fold has a fixed order that depends
// only on the launch (its grid, superblocks and the body's tiling), never on
// scheduling, stream assignment or spilling:
//   - in a body, each wave folds its elements in index order and waves are
//     folded in wave order;
//   - a body that spreads one superblock over several workgroups writes one
//     partial slot per workgroup, and k_fold_slots folds the slots in a
//     fixed order (runs of consecutive slots, then the runs in order);
//   - k_combine folds the superblocks' partials in superblock order.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>

#include "bodies.h"
#include "kernels.h"

namespace lt {

using namespace body;

namespace {

template <class T>
__device__ __forceinline__ T rop(int op, T a, T b) {
    switch (op) {
        case 0: return a + b;
        case 1: return a * b;
        case 2: return b < a ? b : a;
        default: return b > a ? b : a;
    }
}

template <class T>
__device__ __forceinline__ T identity(int op);
template <>
__device__ __forceinline__ float identity<float>(int op) {
    return op == 0 ? 0.f : op == 1 ? 1.f : op == 2 ? INFINITY : -INFINITY;
}
template <>
__device__ __forceinline__ double identity<double>(int op) {
    return op == 0 ? 0. : op == 1 ? 1. : op == 2 ? INFINITY : -INFINITY;
}
template <>
__device__ __forceinline__ int32_t identity<int32_t>(int op) {
    return op == 0 ? 0 : op == 1 ? 1 : op == 2 ? INT_MAX : INT_MIN;
}
template <>
__device__ __forceinline__ int64_t identity<int64_t>(int op) {
    return op == 0 ? 0 : op == 1 ? 1 : op == 2 ? LLONG_MAX : LLONG_MIN;
}

// element offset of global index g inside the dense box of part q
__device__ __forceinline__ int64_t part_offset(const CombinePart &q, int ndim, const int64_t *g) {
    int64_t s1 = ndim > 2 ? q.hi[2] - q.lo[2] : 1;
    int64_t s0 = ndim > 1 ? (q.hi[1] - q.lo[1]) * s1 : 1;
    int64_t off = (g[0] - q.lo[0]) * s0;
    if (ndim > 1) off += (g[1] - q.lo[1]) * s1;
    if (ndim > 2) off += g[2] - q.lo[2];
    return off;
}

__device__ __forceinline__ int64_t box_volume(const CombinePart &q, int ndim) {
    int64_t v = 1;
    for (int x = 0; x < ndim; ++x) v *= q.hi[x] - q.lo[x];
    return v;
}

inline unsigned blocks_for(int64_t total, int64_t cap) {
    int64_t b = (total + 255) / 256;
    return (unsigned)(b < cap ? (b > 0 ? b : 1) : cap);
}

}  // namespace

// ================================================================ combine
template <class T>
__global__ __launch_bounds__(256) void k_combine(CombineArgs a) {
    int64_t e1 = a.hi[1] - a.lo[1], e2 = a.hi[2] - a.lo[2];
    int64_t total = (a.hi[0] - a.lo[0]) * e1 * e2;
    for (int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x; f < total; f += (int64_t)gridDim.x * 256) {
        int64_t i2 = f % e2, r = f / e2;
        int64_t i1 = r % e1, i0 = r / e1;
        int64_t g[3] = {a.lo[0] + i0, a.lo[1] + i1, a.lo[2] + i2};
        LT_GLOBAL T *tp = gp<T>(a.target.base) + g[0] * a.target.s[0] + g[1] * a.target.s[1] +
                g[2] * a.target.s[2];
        T acc = a.accumulate ? *tp : identity<T>(a.op);
        // parts in groups of 8: a group's loads are issued together, then
        // folded in part order
        for (int p0 = 0; p0 < a.nparts; p0 += 8) {
            T v[8];
            bool ok[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int p = p0 + u;
                ok[u] = false;
                v[u] = T(0);
                if (p < a.nparts) {
                    const CombinePart &q = a.parts[p];
                    bool in = true;
                    for (int x = 0; x < a.ndim; ++x)
                        if (g[x] < q.lo[x] || g[x] >= q.hi[x]) in = false;
                    if (in) {
                        ok[u] = true;
                        v[u] = gp<const T>(a.part_base)[q.off + part_offset(q, a.ndim, g)];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (ok[u]) acc = rop<T>(a.op, acc, v[u]);
        }
        *tp = acc;
    }
}

hipError_t launch_combine(hipStream_t s, const CombineArgs &a) {
    int64_t total = 1;
    for (int x = 0; x < KMAXD; ++x) total *= (a.hi[x] - a.lo[x]);
    if (total <= 0) return hipSuccess;
    unsigned blocks = blocks_for(total, 4096);
    switch (a.dtype) {
        case 0: hipLaunchKernelGGL(k_combine<float>, dim3(blocks), dim3(256), 0, s, a); break;
        case 1: hipLaunchKernelGGL(k_combine<int32_t>, dim3(blocks), dim3(256), 0, s, a); break;
        case 2: hipLaunchKernelGGL(k_combine<double>, dim3(blocks), dim3(256), 0, s, a); break;
        case 3: hipLaunchKernelGGL(k_combine<int64_t>, dim3(blocks), dim3(256), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ============================================================= slot fold
// Folds the slots of each part into its first slot.  A workgroup takes 16
// elements of one part (blockIdx.y); its 16 thread groups each fold a
// contiguous run of slots in slot order (loads eight at a time), and the
// runs are then folded in run order.  The order depends only on the slot
// count, so the result is the same on every run.
constexpr int FS_E = 16, FS_G = 16;

template <class T>
__global__ __launch_bounds__(256) void k_fold_slots(CombineArgs a) {
    __shared__ T run[FS_G][FS_E];
    const CombinePart &q = a.parts[blockIdx.y];
    if (q.count <= 1) return;
    const int64_t vol = box_volume(q, a.ndim);
    const int el = threadIdx.x % FS_E, gr = threadIdx.x / FS_E;
    const int64_t per = (q.count + FS_G - 1) / FS_G;
    const int nruns = (int)((q.count + per - 1) / per);
    const int64_t s0 = gr * per, s1 = s0 + per < q.count ? s0 + per : q.count;
    LT_GLOBAL T *P = gp<T>(a.part_base) + q.off;
    for (int64_t eb = blockIdx.x; eb * FS_E < vol; eb += gridDim.x) {
        const int64_t e = eb * FS_E + el;
        if (e < vol && gr < nruns) {
            T acc = P[s0 * vol + e];
            int64_t s = s0 + 1;
            for (; s + 8 <= s1; s += 8) {
                T v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = P[(s + u) * vol + e];
#pragma unroll
                for (int u = 0; u < 8; ++u) acc = rop<T>(a.op, acc, v[u]);
            }
            for (; s < s1; ++s) acc = rop<T>(a.op, acc, P[s * vol + e]);
            run[gr][el] = acc;
        }
        __syncthreads();
        if (gr == 0 && e < vol) {
            T acc = run[0][el];
            for (int g = 1; g < nruns; ++g) acc = rop<T>(a.op, acc, run[g][el]);
            P[e] = acc;
        }
        __syncthreads();
    }
}

hipError_t launch_fold_slots(hipStream_t s, const CombineArgs &a) {
    if (a.nparts <= 0) return hipSuccess;
    int64_t vmax = 0;
    for (int p = 0; p < a.nparts; ++p) {
        int64_t v = 1;
        for (int x = 0; x < a.ndim; ++x) v *= a.parts[p].hi[x] - a.parts[p].lo[x];
        vmax = v > vmax ? v : vmax;
    }
    if (vmax <= 0) return hipSuccess;
    const int64_t eblocks = (vmax + FS_E - 1) / FS_E;
    dim3 grid((unsigned)(eblocks < 4096 ? eblocks : 4096), (unsigned)a.nparts);
    switch (a.dtype) {
        case 0: hipLaunchKernelGGL(k_fold_slots<float>, grid, dim3(256), 0, s, a); break;
        case 1: hipLaunchKernelGGL(k_fold_slots<int32_t>, grid, dim3(256), 0, s, a); break;
        case 2: hipLaunchKernelGGL(k_fold_slots<double>, grid, dim3(256), 0, s, a); break;
        case 3: hipLaunchKernelGGL(k_fold_slots<int64_t>, grid, dim3(256), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ========================================================== row reduction
// The Sec. 2.3 example "global [i, j] => read A[i,j], reduce(f) out[i]":
// out[i] = f over j of A[i][j].  One wave per row of the superblock.  Lane l
// folds the columns c0 + 256k + 4l + q (k = 0, 1, ...; q = 0..3) in that
// order in float64 (+ and * round once at the end; min and max are exact),
// then the 64 lane values are folded by a butterfly, which leaves the same
// value in every lane (each level combines x with y and y with x).  The
// superblock's partial gets the result rounded to float32.
struct RTask {
    int64_t r0, r1, c0, c1;   // rows and columns of the task, clipped to n, m
    int64_t out, a;           // partial view base, A base
    int64_t as;               // A row stride
    int vec;                  // float4 loads usable
};
struct RArgs {
    int op;
    int ntask;
    int begin[KMAXG + 1];
    RTask t[KMAXG];
};

__device__ __forceinline__ double rfold(int op, double acc, float v) { return rop<double>(op, acc, (double)v); }

__global__ __launch_bounds__(256) void k_rowreduce(RArgs a) {
    const int ti = find_task(a.begin, a.ntask, blockIdx.x);
    const RTask &t = a.t[ti];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t row = t.r0 + (int64_t)(blockIdx.x - a.begin[ti]) * 4 + wave;
    if (row >= t.r1) return;
    const int op = a.op;
    const LT_GLOBAL float *A = gp<const float>(t.a) + row * t.as;
    double acc = identity<double>(op);
    int64_t c = t.c0 + 4 * lane;
    if (t.vec) {
        // four float4 loads in flight per lane
        for (; c + 3 * 256 + 3 < t.c1; c += 4 * 256) {
            float4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = ld4<float4>(A + c + u * 256);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                acc = rfold(op, acc, v[u].x);
                acc = rfold(op, acc, v[u].y);
                acc = rfold(op, acc, v[u].z);
                acc = rfold(op, acc, v[u].w);
            }
        }
        for (; c + 3 < t.c1; c += 256) {
            float4 v = ld4<float4>(A + c);
            acc = rfold(op, acc, v.x);
            acc = rfold(op, acc, v.y);
            acc = rfold(op, acc, v.z);
            acc = rfold(op, acc, v.w);
        }
    } else {
        for (; c + 3 < t.c1; c += 256) {
            float x0 = A[c], x1 = A[c + 1], x2 = A[c + 2], x3 = A[c + 3];
            acc = rfold(op, acc, x0);
            acc = rfold(op, acc, x1);
            acc = rfold(op, acc, x2);
            acc = rfold(op, acc, x3);
        }
    }
    for (int q = 0; q < 4; ++q)
        if (c + q < t.c1) acc = rfold(op, acc, A[c + q]);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) acc = rop<double>(op, acc, __shfl_xor(acc, off));
    if (lane == 0) *at<float>(t.out, row) = (float)acc;
}

hipError_t launch_rowreduce_f32(const KLaunch &L) {
    RArgs a;
    const int64_t n = L.iarg[0], m = L.iarg[1];
    a.op = L.rop[2];
    a.ntask = L.ntask;
    int64_t nb = 0;
    for (int i = 0; i < L.ntask; ++i) {
        const KTask &k = L.tasks[i];
        RTask &r = a.t[i];
        r.r0 = k.lo[0];
        r.r1 = k.hi[0] < n ? k.hi[0] : n;
        r.c0 = k.lo[1];
        r.c1 = k.hi[1] < m ? k.hi[1] : m;
        r.out = k.v[2].base;
        r.a = k.v[3].base;
        r.as = k.v[3].s[0];
        const int64_t first = r.a + (r.r0 * r.as + r.c0) * 4;
        r.vec = (first % 16 == 0) && (r.as % 4 == 0);
        a.begin[i] = (int)nb;
        if (r.r1 > r.r0 && r.c1 > r.c0) nb += (r.r1 - r.r0 + 3) / 4;
    }
    a.begin[L.ntask] = (int)nb;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rowreduce, dim3((unsigned)nb), dim3(256), 0, L.stream, a);
    return hipGetLastError();
}

// ======================================================== k-means update
// sums[k][j] = sum of X[p][j] and counts[k] = number of points p with
// lab[p] = k (labels outside [0, K) are skipped), over the superblock's
// points.  The task's points are cut into tiles of KMU_TILE; workgroup w
// (w < slots) takes tiles w, w + slots, ... and each of its four waves a
// quarter of every tile, in order.  A wave accumulates in its own float64
// LDS copy of sums and counts: the wave's lanes cover P = 64 / DP points at
// a step (DP = d rounded up to a power of two, one feature per lane), and
// lanes whose points share a cluster add in rounds, in point order, so every
// cell of the wave's copy is a sequential sum in point order.  The workgroup
// then adds its four copies in wave order and writes partial slot w.
struct KUTask {
    int64_t lo, hi;           // points, clipped to N
    int64_t sums, counts;     // slot-0 partial views (pre-offset, element (0, 0) / (0))
    int64_t ss0, ss1, sslot;  // sums view strides and slot stride (elements)
    int64_t cs0, cslot;       // counts view stride and slot stride
    int64_t x, xs, lab;       // X base and row stride, lab base
    int nslots;
};
struct KUArgs {
    int d, K, dp;
    int ntask;
    int begin[KMAXG + 1];
    KUTask t[KMAXG];
};

constexpr int KMU_U = 8;  // steps per load batch; two batches are in flight

// Loads one batch of KMU_U steps: lane (q, j) gets feature j of point
// pb + u*P + q and that point's label (-1 when out of range or inactive).
template <int DP>
__device__ __forceinline__ void kmu_load(const LT_GLOBAL float *X, int64_t xs, const LT_GLOBAL int32_t *LB,
                                         int64_t pb, int64_t p1, int q, int j, int d, int K, float *xv, int *kv) {
    constexpr int P = 64 / DP;
#pragma unroll
    for (int u = 0; u < KMU_U; ++u) {
        const int64_t p = pb + (int64_t)u * P + q;
        const bool act = p < p1;
        xv[u] = (act && j < d) ? X[p * xs + j] : 0.f;
        const int k = act ? LB[p] : -1;
        kv[u] = (k >= 0 && k < K) ? k : -1;
    }
}

// Rank of this lane's point among the step's P = 64 / LP points: the number
// of earlier points of the step (point q holds lanes q LP .. q LP + LP - 1)
// with the same cluster.  With LP >= 4 the comparisons are spread over the
// point's lanes: lane (q, c) compares with points c, c + LP, ... (fetched by
// lane permutes) and the LP lanes add their counts, so a step costs P / LP
// permutes per lane instead of P scalar reads.  Labels of -1 never add, so
// their ranks do not matter.
template <int LP>
__device__ __forceinline__ int kmu_rank(int k, int q, int c) {
    constexpr int P = 64 / LP;
    int rank = 0;
    if constexpr (LP >= 4) {
#pragma unroll
        for (int q2 = c; q2 < P; q2 += LP) {
            const int k2 = __shfl(k, q2 * LP);
            rank += (q2 < q && k2 == k) ? 1 : 0;
        }
#pragma unroll
        for (int off = 1; off < LP; off <<= 1) rank += __shfl_xor(rank, off);
    } else if constexpr (P <= 32) {
#pragma unroll
        for (int q2 = 0; q2 < P; ++q2) {
            const int k2 = __builtin_amdgcn_readlane(k, q2 * LP);
            rank += (q2 < q && k2 == k) ? 1 : 0;
        }
    } else {
        // one lane per point: a rolled loop keeps the scalar registers in bounds
#pragma unroll 1
        for (int q2 = 0; q2 < P; ++q2) {
            const int k2 = __builtin_amdgcn_readlane(k, q2 * LP);
            rank += (q2 < q && k2 == k) ? 1 : 0;
        }
    }
    return rank;
}

// LDS adds that return nothing (ds_add_f64, ds_add_u32): the wave issues
// them without waiting for the old value.  No two of them ever touch the
// same word concurrently (each wave owns its copy, and the rounds below
// keep equal clusters out of one instruction), so the atomicity is never
// exercised: they are ordinary read-add-writes, each correctly rounded, and
// a wave's LDS operations complete in issue order.
__device__ __forceinline__ void lds_add(double *p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add(int *p, int v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Adds one step's points into the wave's copy.  Lanes whose points share a
// cluster add in rounds, in point order: round r adds the points of rank r.
// The ranks of one cluster are 0, 1, 2, ..., so the first round with no
// point ends the step.  A wave's LDS operations complete in issue order, so
// round r + 1 adds after round r; the empty asm only stops the compiler
// from moving LDS operations across rounds.
template <int DP>
__device__ __forceinline__ void kmu_step(double *acc, int *cnt, int d, int ks, int q, int j, float x, int k) {
    const int rank = kmu_rank<DP>(k, q, j);
    for (int r = 0;; ++r) {
        const bool mine = k >= 0 && rank == r;
        if (!__ballot(mine)) break;
        if (mine) {
            if (j < d) lds_add(&acc[k * ks + j], (double)x);
            if (j == 0) lds_add(&cnt[k], 1);
        }
        asm volatile("" ::: "memory");
    }
}

// The task's fields, copied to registers once: the compiler barrier between
// rounds would otherwise make it re-read them from memory at every step.
struct KUReg {
    int64_t lo, hi, xs, sslot, cslot, ss0, ss1, cs0;
    const LT_GLOBAL float *X;
    const LT_GLOBAL int32_t *LB;
    LT_GLOBAL double *S;
    LT_GLOBAL int32_t *C;
    int nslots;
};

__device__ __forceinline__ KUReg kmu_regs(const KUTask &t) {
    KUReg r;
    r.lo = t.lo;
    r.hi = t.hi;
    r.xs = t.xs;
    r.sslot = t.sslot;
    r.cslot = t.cslot;
    r.ss0 = t.ss0;
    r.ss1 = t.ss1;
    r.cs0 = t.cs0;
    r.X = gp<const float>(t.x);
    r.LB = gp<const int32_t>(t.lab);
    r.S = gp<double>(t.sums);
    r.C = gp<int32_t>(t.counts);
    r.nslots = t.nslots;
    return r;
}

// A wave's copy holds cluster k's sums at k * KS .. k * KS + d - 1 with the
// odd stride KS = d | 1: in one LDS instruction the lanes of different
// points then spread over the banks instead of all landing on the bank of
// feature j (an even stride of 16 doubles maps every cluster to one bank).
__device__ __forceinline__ int kmu_stride(int d) { return d | 1; }

__device__ __forceinline__ void kmu_clear(double *lds, int KDP, int K) {
    int *cnt_all = reinterpret_cast<int *>(lds + 4 * KDP);
    for (int i = threadIdx.x; i < 4 * KDP; i += 256) lds[i] = 0.0;
    for (int i = threadIdx.x; i < 4 * K; i += 256) cnt_all[i] = 0;
    __syncthreads();
}

// Adds the four wave copies in wave order and writes partial slot w.
__device__ __forceinline__ void kmu_flush(const double *lds, int d, int K, const KUReg &t, int w) {
    const int ks = kmu_stride(d), KDP = K * ks;
    const int *cnt_all = reinterpret_cast<const int *>(lds + 4 * KDP);
    __syncthreads();
    LT_GLOBAL double *S = t.S + (int64_t)w * t.sslot;
    for (int e = threadIdx.x; e < K * d; e += 256) {
        const int k = e / d, jj = e - (e / d) * d;
        const int i = k * ks + jj;
        double s = lds[i];
        s += lds[KDP + i];
        s += lds[2 * KDP + i];
        s += lds[3 * KDP + i];
        S[k * t.ss0 + jj * t.ss1] = s;
    }
    LT_GLOBAL int32_t *Cn = t.C + (int64_t)w * t.cslot;
    for (int k = threadIdx.x; k < K; k += 256)
        Cn[k * t.cs0] = cnt_all[k] + cnt_all[K + k] + cnt_all[2 * K + k] + cnt_all[3 * K + k];
}

// Any d: one feature per lane (DP lanes per point).
template <int DP>
__global__ __launch_bounds__(256) void k_kmeans_update(KUArgs a) {
    constexpr int P = 64 / DP;
    extern __shared__ double lds[];
    const int ti = find_task(a.begin, a.ntask, blockIdx.x);
    const KUReg t = kmu_regs(a.t[ti]);
    const int w = blockIdx.x - a.begin[ti];
    const int d = a.d, K = a.K, ks = kmu_stride(d), KDP = K * ks;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    kmu_clear(lds, KDP, K);
    double *acc = lds + wave * KDP;
    int *cnt = reinterpret_cast<int *>(lds + 4 * KDP) + wave * K;
    const int q = lane / DP, j = lane % DP;
    constexpr int64_t QUARTER = KMU_TILE / 4;
    constexpr int64_t BATCH = (int64_t)KMU_U * P;
    for (int64_t tile = w; t.lo + tile * KMU_TILE < t.hi; tile += t.nslots) {
        const int64_t p0 = t.lo + tile * KMU_TILE + wave * QUARTER;
        const int64_t p1 = p0 + QUARTER < t.hi ? p0 + QUARTER : t.hi;
        if (p0 >= p1) continue;
        float xv[KMU_U], xn[KMU_U];
        int kv[KMU_U], kn[KMU_U];
        kmu_load<DP>(t.X, t.xs, t.LB, p0, p1, q, j, d, K, xv, kv);
        for (int64_t pb = p0; pb < p1; pb += BATCH) {
            const bool more = pb + BATCH < p1;
            if (more) kmu_load<DP>(t.X, t.xs, t.LB, pb + BATCH, p1, q, j, d, K, xn, kn);
#pragma unroll
            for (int u = 0; u < KMU_U; ++u) kmu_step<DP>(acc, cnt, d, ks, q, j, xv[u], kv[u]);
            if (more) {
#pragma unroll
                for (int u = 0; u < KMU_U; ++u) {
                    xv[u] = xn[u];
                    kv[u] = kn[u];
                }
            }
        }
    }
    kmu_flush(lds, d, K, t, w);
}

// d = VD in {4, 8, 16, 32} with dense, 16-byte aligned rows: lane l holds
// features FPL c .. FPL c + FPL - 1 (c = l % LP, LP = VD / FPL) of point
// l / LP, so one FPL-float load per lane brings 64 / LP whole points; the
// additions per element are the same as in the one-feature-per-lane body,
// and in the same order (point order), whatever FPL is.
constexpr int KMV_U = 4;  // steps per load batch; two batches are in flight

template <int FPL>
struct KmvVec;
template <>
struct KmvVec<4> {
    using T = float4;
    static __device__ __forceinline__ float get(const T &v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }
    static __device__ __forceinline__ T zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
};
template <>
struct KmvVec<2> {
    using T = float2;
    static __device__ __forceinline__ float get(const T &v, int i) { return i == 0 ? v.x : v.y; }
    static __device__ __forceinline__ T zero() { return make_float2(0.f, 0.f); }
};

template <int VD, int FPL>
__device__ __forceinline__ void kmv_load(const KUReg &t, int64_t pb, int64_t p1, int lane, int q, int K, bool full,
                                         typename KmvVec<FPL>::T *xv, int *kv) {
    using V = KmvVec<FPL>;
    constexpr int LP = VD / FPL, P = 64 / LP;
#pragma unroll
    for (int u = 0; u < KMV_U; ++u) {
        const int64_t pu = pb + (int64_t)u * P;
        const int64_t p = pu + q;
        int k;
        if (full) {
            xv[u] = ld4<typename V::T>(t.X + pu * VD + FPL * lane);
            k = t.LB[p];
        } else {
            const bool act = p < p1;
            xv[u] = act ? ld4<typename V::T>(t.X + pu * VD + FPL * lane) : V::zero();
            k = act ? t.LB[p] : -1;
        }
        kv[u] = (k >= 0 && k < K) ? k : -1;
    }
}

template <int VD, int FPL>
__device__ __forceinline__ void kmv_step(double *acc, int *cnt, int q, int c, const typename KmvVec<FPL>::T &x,
                                         int k) {
    using V = KmvVec<FPL>;
    constexpr int LP = VD / FPL;
    const int rank = kmu_rank<LP>(k, q, c);
    for (int r = 0;; ++r) {
        const bool mine = k >= 0 && rank == r;
        if (!__ballot(mine)) break;
        if (mine) {
            double *e = acc + k * (VD | 1) + FPL * c;
#pragma unroll
            for (int i = 0; i < FPL; ++i) lds_add(e + i, (double)V::get(x, i));
            if (c == 0) lds_add(&cnt[k], 1);
        }
        asm volatile("" ::: "memory");
    }
}

template <int VD, int FPL>
__global__ __launch_bounds__(256) void k_kmeans_update_v(KUArgs a) {
    using VT = typename KmvVec<FPL>::T;
    constexpr int LP = VD / FPL, P = 64 / LP;
    extern __shared__ double lds[];
    const int ti = find_task(a.begin, a.ntask, blockIdx.x);
    const KUReg t = kmu_regs(a.t[ti]);
    const int w = blockIdx.x - a.begin[ti];
    const int K = a.K, KDP = K * (VD | 1);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    kmu_clear(lds, KDP, K);
    double *acc = lds + wave * KDP;
    int *cnt = reinterpret_cast<int *>(lds + 4 * KDP) + wave * K;
    const int q = lane / LP, c = lane % LP;
    constexpr int64_t QUARTER = KMU_TILE / 4;
    constexpr int64_t BATCH = (int64_t)KMV_U * P;
    for (int64_t tile = w; t.lo + tile * KMU_TILE < t.hi; tile += t.nslots) {
        const int64_t p0 = t.lo + tile * KMU_TILE + wave * QUARTER;
        const int64_t p1 = p0 + QUARTER < t.hi ? p0 + QUARTER : t.hi;
        if (p0 >= p1) continue;
        VT xv[KMV_U], xn[KMV_U];
        int kv[KMV_U], kn[KMV_U];
        kmv_load<VD, FPL>(t, p0, p1, lane, q, K, p0 + BATCH <= p1, xv, kv);
        for (int64_t pb = p0; pb < p1; pb += BATCH) {
            const int64_t nb = pb + BATCH;
            const bool more = nb < p1;
            if (more) kmv_load<VD, FPL>(t, nb, p1, lane, q, K, nb + BATCH <= p1, xn, kn);
#pragma unroll
            for (int u = 0; u < KMV_U; ++u) kmv_step<VD, FPL>(acc, cnt, q, c, xv[u], kv[u]);
            if (more) {
#pragma unroll
                for (int u = 0; u < KMV_U; ++u) {
                    xv[u] = xn[u];
                    kv[u] = kn[u];
                }
            }
        }
    }
    kmu_flush(lds, VD, K, t, w);
}

// d = VD in {16, 32} with dense rows: one feature per lane, P = 64 / VD
// points per step (point q on lanes q VD .. q VD + VD - 1).  Each wave has
// two LDS copies of the sums, interleaved by cluster: row k holds copy 0's
// VD doubles and then copy 1's (double k 2VD + c VD + j), and point q of a
// step adds into copy q % 2.  A row is 4 VD dwords, a multiple of 64, so
// copy 0 of every cluster starts on one bank and copy 1 VD doubles further:
// the two points that share an LDS half-instruction (32 lanes) fall on
// disjoint banks whatever their clusters.  Only points q and q + 2 share a
// copy; when their clusters agree, the add of point q + 2 waits for the
// end of its batch, so no two lanes of one instruction add into one cell
// and the order of every cell's adds is fixed by the data alone.  Counts
// are integer adds in one copy per wave, exact in any order.
//
// Loads one batch of U steps: lane (q, j) gets feature j of point
// pb + u P + q and that point's raw label.  With FULL every point of the
// batch is in range and the loads take immediate offsets from one scalar
// base; otherwise points at or past p1 read point p1 - 1 instead.  Either
// way every load is issued and none of the loaded values is inspected here,
// so the wave does not wait for a batch until it adds it.
template <int VD, int U, bool FULL>
__device__ __forceinline__ void kmc_load(const KUReg &t, int64_t pb, int64_t p1, int lane, float *xv, int *kv) {
    constexpr int P = 64 / VD;
    const int q = lane / VD, j = lane % VD;
    if constexpr (FULL) {
        const LT_GLOBAL float *x = t.X + pb * VD + lane;
        const LT_GLOBAL int32_t *lb = t.LB + pb + q;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            xv[u] = __builtin_nontemporal_load(x + u * 64);
            kv[u] = lb[u * P];
        }
    } else {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int64_t p = pb + (int64_t)u * P + q;
            p = p < p1 ? p : p1 - 1;
            xv[u] = t.X[p * VD + j];
            kv[u] = t.LB[p];
        }
    }
}

// Adds one loaded batch; nleft = points of the batch inside the range
// (unchecked with FULL).  Point q + 2 of a step finds the cluster of point
// q, its copy-mate, 32 lanes down with one lane swap of the two wave halves.
// A point whose copy-mate has its cluster is held back: the clashing adds of
// the batch's U steps follow the others, step by step, so each cell's order
// is fixed by the data alone.  The batch's counts go in one integer LDS add
// after its U steps: lane (q, j) with j < U counts point q of step j
// (integer adds need no order, and the atomic keeps equal clusters in one
// instruction correct).
template <int VD, int U, bool FULL>
__device__ __forceinline__ void kmc_add(double *acc, int *cnt, const float *xv, const int *kv, int64_t nleft, int q,
                                        int j, int K) {
    constexpr int P = 64 / VD;
    static_assert(U <= VD, "one count lane per step");
    const int krow = 2 * VD;
    bool late[U];
    bool any_late = false;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int k = kv[u];
        const bool ok = (unsigned)k < (unsigned)K && (FULL || (int64_t)(u * P + q) < nleft);
        late[u] = false;
        if constexpr (P == 4) {
            // lanes 32..63 receive lanes 0..31 of k: the copy-mate's cluster
            const int mate = __builtin_amdgcn_permlane32_swap(k, k, false, false)[0];
            late[u] = ok && q >= 2 && k == mate;
            any_late |= late[u];
        }
        if (ok && !late[u]) lds_add(acc + k * krow, (double)xv[u]);
    }
    if constexpr (P == 4) {
        if (__builtin_amdgcn_ballot_w64(any_late)) {
            asm volatile("" ::: "memory");
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (late[u]) lds_add(acc + kv[u] * krow, (double)xv[u]);
        }
    }
    asm volatile("" ::: "memory");
    int kc = -1;
#pragma unroll
    for (int u = 0; u < U; ++u) kc = j == u ? kv[u] : kc;
    if (j < U && (unsigned)kc < (unsigned)K && (FULL || (int64_t)(j * P + q) < nleft)) lds_add(&cnt[kc], 1);
}

// Points [p0, p1) of one wave: two register batches, A and B, alternate, so
// the next batch is in flight while the current one is added.  With FULL,
// p1 - p0 is a whole number of batch pairs (a whole quarter tile).
template <int VD, int U, bool FULL>
__device__ __forceinline__ void kmc_range(const KUReg &t, double *acc, int *cnt, int64_t p0, int64_t p1, int lane,
                                          int K) {
    constexpr int P = 64 / VD;
    constexpr int64_t BATCH = (int64_t)U * P;
    const int q = lane / VD, j = lane % VD;
    float xa[U], xb[U];
    int ka[U], kb[U];
    kmc_load<VD, U, FULL>(t, p0, p1, lane, xa, ka);
    for (int64_t pb = p0;; pb += 2 * BATCH) {
        if (!FULL && pb + BATCH >= p1) {
            kmc_add<VD, U, FULL>(acc, cnt, xa, ka, p1 - pb, q, j, K);
            break;
        }
        kmc_load<VD, U, FULL>(t, pb + BATCH, p1, lane, xb, kb);
        kmc_add<VD, U, FULL>(acc, cnt, xa, ka, p1 - pb, q, j, K);
        if (pb + 2 * BATCH >= p1) {
            kmc_add<VD, U, FULL>(acc, cnt, xb, kb, p1 - pb - BATCH, q, j, K);
            break;
        }
        kmc_load<VD, U, FULL>(t, pb + 2 * BATCH, p1, lane, xa, ka);
        kmc_add<VD, U, FULL>(acc, cnt, xb, kb, p1 - pb - BATCH, q, j, K);
    }
}

template <int VD, int U>
__global__ __launch_bounds__(256) void k_kmeans_update_c(KUArgs a) {
    constexpr int P = 64 / VD;
    static_assert(P == 2 || P == 4, "two or four points per step");
    constexpr int64_t QUARTER = KMU_TILE / 4;
    static_assert(QUARTER % (2 * U * P) == 0, "a quarter tile is a whole number of batch pairs");
    extern __shared__ double lds[];
    const int ti = find_task(a.begin, a.ntask, blockIdx.x);
    const KUReg t = kmu_regs(a.t[ti]);
    const int w = blockIdx.x - a.begin[ti];
    // each wave: its two copies, K rows of 2 VD doubles
    const int K = a.K, KROW = 2 * VD, KD2 = K * KROW;
    // the wave index is uniform: readfirstlane keeps the point ranges, and
    // the branches on them, scalar
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    int *cnt_all = reinterpret_cast<int *>(lds + 4 * KD2);
    for (int i = threadIdx.x; i < 4 * KD2; i += 256) lds[i] = 0.0;
    for (int i = threadIdx.x; i < 4 * K; i += 256) cnt_all[i] = 0;
    __syncthreads();
    const int q = lane / VD, j = lane % VD;
    double *acc = lds + wave * KD2 + (q & 1) * VD + j;
    int *cnt = cnt_all + wave * K;
    for (int64_t tile = w; t.lo + tile * KMU_TILE < t.hi; tile += t.nslots) {
        const int64_t p0 = t.lo + tile * KMU_TILE + wave * QUARTER;
        const int64_t p1 = p0 + QUARTER < t.hi ? p0 + QUARTER : t.hi;
        if (p1 - p0 == QUARTER) kmc_range<VD, U, true>(t, acc, cnt, p0, p1, lane, K);
        else if (p0 < p1) kmc_range<VD, U, false>(t, acc, cnt, p0, p1, lane, K);
    }
    // the eight copies in wave order, copy 0 before copy 1, into slot w
    __syncthreads();
    LT_GLOBAL double *S = t.S + (int64_t)w * t.sslot;
    for (int e = threadIdx.x; e < K * VD; e += 256) {
        const int k = e / VD, jj = e % VD;
        const int i = k * KROW + jj;
        double s = lds[i];
        s += lds[i + VD];
#pragma unroll
        for (int v = 1; v < 4; ++v) {
            s += lds[v * KD2 + i];
            s += lds[v * KD2 + i + VD];
        }
        S[k * t.ss0 + jj * t.ss1] = s;
    }
    LT_GLOBAL int32_t *Cn = t.C + (int64_t)w * t.cslot;
    for (int k = threadIdx.x; k < K; k += 256)
        Cn[k * t.cs0] = cnt_all[k] + cnt_all[K + k] + cnt_all[2 * K + k] + cnt_all[3 * K + k];
}

hipError_t launch_kmeans_update_f32(const KLaunch &L) {
    // parameters: N, d, K, sums, counts, X, lab
    KUArgs a;
    const int64_t N = L.iarg[0];
    a.d = (int)L.iarg[1];
    a.K = (int)L.iarg[2];
    if (a.d < 1 || a.d > KMU_MAXD || a.K < 1 || a.K > KMU_MAXK || (int64_t)a.K * a.d > KMU_MAXKD)
        return hipErrorInvalidValue;
    a.dp = 1;
    while (a.dp < a.d) a.dp <<= 1;
    a.ntask = L.ntask;
    int64_t nb = 0;
    for (int i = 0; i < L.ntask; ++i) {
        const KTask &k = L.tasks[i];
        KUTask &u = a.t[i];
        u.lo = k.lo[0];
        u.hi = k.hi[0] < N ? k.hi[0] : N;
        u.sums = k.v[3].base;
        u.ss0 = k.v[3].s[0];
        u.ss1 = k.v[3].s[1];
        u.sslot = k.slot[3];
        u.counts = k.v[4].base;
        u.cs0 = k.v[4].s[0];
        u.cslot = k.slot[4];
        u.x = k.v[5].base;
        u.xs = k.v[5].s[0];
        u.lab = k.v[6].base;
        const int64_t e = u.hi - u.lo;
        u.nslots = (int)kmu_slots(e, a.d);
        // a task with several slots needs the slot strides from the planner
        if (u.nslots > 1 && (u.sslot <= 0 || u.cslot <= 0)) return hipErrorInvalidValue;
        // every slot gets its workgroup, empty tasks included: the partials
        // are not filled beforehand, each slot is written whole
        a.begin[i] = (int)nb;
        nb += u.nslots;
    }
    a.begin[L.ntask] = (int)nb;
    if (nb == 0) return hipSuccess;
    // four wave copies of K x (d | 1) float64 sums and K int32 counts: at
    // most 4 x (1536 + 256) x 8 + 4 x 256 x 4 = 61,440 bytes
    const size_t lds = (size_t)4 * a.K * (a.d | 1) * sizeof(double) + (size_t)4 * a.K * sizeof(int);
    const dim3 g((unsigned)nb), b(256);
    bool vec = a.d == a.dp && a.d >= 4;  // d in {4, 8, 16, 32}
    for (int i = 0; i < L.ntask && vec; ++i)
        vec = a.t[i].xs == a.d && a.t[i].x % 16 == 0 && (a.t[i].lo * a.d * 4) % 16 == 0;
    if (vec && a.d >= 16 && L.variant == 0) {
        // d in {16, 32}: one feature per lane with two interleaved copies per
        // wave: 4 x K x 2d float64 sums and K int32 counts per wave, at most
        // 4 x 1536 x 2 x 8 + 4 x 96 x 4 bytes
        const size_t lc = (size_t)4 * a.K * 2 * a.d * sizeof(double) + (size_t)4 * a.K * sizeof(int);
        void (*f)(KUArgs) = a.d == 16 ? k_kmeans_update_c<16, 8> : k_kmeans_update_c<32, 8>;
        if (lc > 65536) {
            // more than 64 KiB of dynamic LDS (up to 160 KiB per workgroup on gfx950)
            const hipError_t e = hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lc);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(f, g, b, lc, L.stream, a);
        return hipGetLastError();
    }
    if (vec) {
        switch (a.d) {
            // four features per lane (d in {4, 8}, and variant 1 for d in
            // {16, 32}); variant 2 takes two (d >= 8): fewer add rounds per
            // point, but measured slower (3.24 against 3.45 TB/s at d = 16,
            // K = 64), the LDS being bound by lanes, not instructions
            case 4: hipLaunchKernelGGL((k_kmeans_update_v<4, 4>), g, b, lds, L.stream, a); break;
            case 8:
                if (L.variant == 2) hipLaunchKernelGGL((k_kmeans_update_v<8, 2>), g, b, lds, L.stream, a);
                else hipLaunchKernelGGL((k_kmeans_update_v<8, 4>), g, b, lds, L.stream, a);
                break;
            case 16:
                if (L.variant == 2) hipLaunchKernelGGL((k_kmeans_update_v<16, 2>), g, b, lds, L.stream, a);
                else hipLaunchKernelGGL((k_kmeans_update_v<16, 4>), g, b, lds, L.stream, a);
                break;
            default:
                if (L.variant == 2) hipLaunchKernelGGL((k_kmeans_update_v<32, 2>), g, b, lds, L.stream, a);
                else hipLaunchKernelGGL((k_kmeans_update_v<32, 4>), g, b, lds, L.stream, a);
                break;
        }
        return hipGetLastError();
    }
    switch (a.dp) {
        case 1: hipLaunchKernelGGL(k_kmeans_update<1>, g, b, lds, L.stream, a); break;
        case 2: hipLaunchKernelGGL(k_kmeans_update<2>, g, b, lds, L.stream, a); break;
        case 4: hipLaunchKernelGGL(k_kmeans_update<4>, g, b, lds, L.stream, a); break;
        case 8: hipLaunchKernelGGL(k_kmeans_update<8>, g, b, lds, L.stream, a); break;
        case 16: hipLaunchKernelGGL(k_kmeans_update<16>, g, b, lds, L.stream, a); break;
        default: hipLaunchKernelGGL(k_kmeans_update<32>, g, b, lds, L.stream, a); break;
    }
    return hipGetLastError();
}

// ========================================================= k-means centres
// cen[k][j] = sums[k][j] / counts[k] in float64, rounded once to float32;
// clusters with no points keep their centre.
struct KCTask {
    int64_t k0, k1, j0, j1;
    int64_t cen, sums, counts;
    int64_t c0, s0, s1, n0;   // strides: cen row, sums row and column, counts
};
struct KCArgs {
    int ntask;
    int begin[KMAXG + 1];
    KCTask t[KMAXG];
};

__global__ __launch_bounds__(256) void k_kmeans_centres(KCArgs a) {
    const int ti = find_task(a.begin, a.ntask, blockIdx.x);
    const KCTask &t = a.t[ti];
    const int64_t w = t.j1 - t.j0;
    const int64_t e = (int64_t)(blockIdx.x - a.begin[ti]) * 256 + threadIdx.x;
    if (e >= (t.k1 - t.k0) * w) return;
    const int64_t k = t.k0 + e / w, j = t.j0 + e % w;
    const int32_t c = *at<const int32_t>(t.counts, k * t.n0);
    if (c <= 0) return;
    const double s = *at<const double>(t.sums, k * t.s0 + j * t.s1);
    *at<float>(t.cen, k * t.c0 + j) = (float)(s / (double)c);
}

hipError_t launch_kmeans_centres_f32(const KLaunch &L) {
    // parameters: K, d, cen, sums, counts
    KCArgs a;
    const int64_t K = L.iarg[0], d = L.iarg[1];
    a.ntask = L.ntask;
    int64_t nb = 0;
    for (int i = 0; i < L.ntask; ++i) {
        const KTask &k = L.tasks[i];
        KCTask &c = a.t[i];
        c.k0 = k.lo[0];
        c.k1 = k.hi[0] < K ? k.hi[0] : K;
        c.j0 = k.lo[1];
        c.j1 = k.hi[1] < d ? k.hi[1] : d;
        c.cen = k.v[2].base;
        c.c0 = k.v[2].s[0];
        c.sums = k.v[3].base;
        c.s0 = k.v[3].s[0];
        c.s1 = k.v[3].s[1];
        c.counts = k.v[4].base;
        c.n0 = k.v[4].s[0];
        a.begin[i] = (int)nb;
        const int64_t e = (c.k1 - c.k0) * (c.j1 - c.j0);
        if (c.k1 > c.k0 && c.j1 > c.j0) nb += (e + 255) / 256;
    }
    a.begin[L.ntask] = (int)nb;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_kmeans_centres, dim3((unsigned)nb), dim3(256), 0, L.stream, a);
    return hipGetLastError();
}

}  // namespace lt
