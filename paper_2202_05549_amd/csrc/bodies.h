// Device bodies shared by the one-dispatch-per-task kernels (kernels.hip)
// and the persistent drain kernel (drain.hip).  Each body works on one tile
// of one task with 256 threads and global indices through pre-offset views,
// so both execution paths perform exactly the same arithmetic per element.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lt {
namespace body {

constexpr int WAVE = 64;
constexpr int THREADS = 256;

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Views arrive as integer addresses.  Turning them into pointers in the
// global address space (not generic ones) makes the compiler emit global
// loads and stores: generic (flat) accesses also count against the LDS
// counter, so every lane shuffle or LDS read would wait for all global loads
// still in flight and defeat any prefetching.
#if defined(__HIP_DEVICE_COMPILE__)
#define LT_GLOBAL __attribute__((address_space(1)))
#else
#define LT_GLOBAL
#endif

// Task lookup in a dispatch that covers several tasks: the task t with
// begin[t] <= b < begin[t+1].
__device__ __forceinline__ int find_task(const int *begin, int ntask, int b) {
    int lo = 0, hi = ntask - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (begin[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <class T>
__device__ __forceinline__ LT_GLOBAL T *gp(int64_t base) {
    return (LT_GLOBAL T *)base;
}

template <class T>
__device__ __forceinline__ LT_GLOBAL T *at(int64_t base, int64_t idx) {
    return gp<T>(base) + idx;
}

template <class T>
__device__ __forceinline__ T ld4(const LT_GLOBAL void *p) {
    return *(const LT_GLOBAL T *)p;
}

// 16-byte store without cache retention (streaming output)
__device__ __forceinline__ void nt_store4(LT_GLOBAL float *p, float4 v) {
    f32x4 w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, (LT_GLOBAL f32x4 *)p);
}

// Physical workgroups are dealt round-robin to the 8 XCDs.  Remap so each
// XCD receives a contiguous range of logical tiles; identity on the tail
// that is not a multiple of 8.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    int per = nb >> 3;
    if (b >= (per << 3)) return b;
    return (b & 7) * per + (b >> 3);
}

// ------------------------------------------------------------------ touch
// y[i] += 1 for i in [i0, i0 + 256) within [lo, hi) and [0, n).
__device__ __forceinline__ void touch_span(int64_t y, int64_t n, int64_t lo, int64_t hi, int64_t i0) {
    int64_t i = i0 + threadIdx.x;
    if (i >= lo && i < hi && i < n && i >= 0) *at<int32_t>(y, i) += 1;
}

// -------------------------------------------------------------- stencil1d
// y[i] = 0.25*(x[i-1] + x[i+1]) + 0.5*x[i], zero outside [0, n).
__device__ __forceinline__ float st_point(float l, float m, float r) {
    float s = l + r;
    float t = 0.25f * s;
    float u = 0.5f * m;
    return t + u;
}

// The 1024 outputs starting at span0 (4 per thread) of the task [lo, hi).
// Neighbours across lanes come from the adjacent lane's registers; the two
// wave-edge lanes load theirs.  Must be called by all 256 threads.
__device__ __forceinline__ void stencil_span(int64_t xb, int64_t yb, int64_t n, int64_t lo, int64_t hi,
                                             int64_t span0) {
    const int64_t end = hi < n ? hi : n;               // outputs [lo, end)
    const int64_t rend = end + 1 < n ? end + 1 : n;    // inputs read: [lo-1, rend)
    const int64_t i0 = span0 + threadIdx.x * 4;
    const LT_GLOBAL float *X = gp<const float>(xb);
    LT_GLOBAL float *Y = gp<float>(yb);
    const bool aligned = ((xb + lo * 4) & 15) == 0 && ((yb + lo * 4) & 15) == 0 && ((span0 - lo) & 3) == 0;
    float v[4];
    if (aligned && i0 + 3 < end) {
        float4 q = ld4<float4>(X + i0);
        v[0] = q.x;
        v[1] = q.y;
        v[2] = q.z;
        v[3] = q.w;
    } else {
        for (int j = 0; j < 4; ++j) v[j] = (i0 + j < rend) ? X[i0 + j] : 0.f;
    }
    const int lane = threadIdx.x & (WAVE - 1);
    float left = __shfl_up(v[3], 1);
    float right = __shfl_down(v[0], 1);
    if (i0 >= end) return;
    if (lane == 0) left = (i0 - 1 >= 0) ? X[i0 - 1] : 0.f;
    if (lane == WAVE - 1 && i0 + 3 < end) right = (i0 + 4 < n) ? X[i0 + 4] : 0.f;
    float o[4];
    o[0] = st_point(left, v[0], v[1]);
    o[1] = st_point(v[0], v[1], v[2]);
    o[2] = st_point(v[1], v[2], v[3]);
    o[3] = st_point(v[2], v[3], right);
    if (aligned && i0 + 3 < end) {
        *(LT_GLOBAL float4 *)(Y + i0) = make_float4(o[0], o[1], o[2], o[3]);
    } else {
        for (int j = 0; j < 4; ++j)
            if (i0 + j < end) Y[i0 + j] = o[j];
    }
}

// Streaming form for long ranges: outputs [s0, s1) of the task [lo, hi) in
// groups of G spans of 1024.  A group's loads (the lane's G float4 plus the
// two wave-edge neighbours) are issued before the previous group is computed
// and stored, so 2G independent 16-byte loads per lane stay in flight.  The
// input and output arrays must not overlap (they never do for a stencil:
// the annotation reads x and writes y).  Ragged ends use stencil_span.
template <int G>
struct StGroup {
    float4 v[G];
    float l[G], r[G];
};

template <int G>
__device__ __forceinline__ void st_load(const LT_GLOBAL float *__restrict__ X, int64_t n, int64_t g0, int lane,
                                        StGroup<G> &q) {
#pragma unroll
    for (int u = 0; u < G; ++u) {
        const int64_t i0 = g0 + u * 1024 + threadIdx.x * 4;
        q.v[u] = ld4<float4>(X + i0);
        q.l[u] = (lane == 0 && i0 - 1 >= 0) ? X[i0 - 1] : 0.f;
        q.r[u] = (lane == WAVE - 1 && i0 + 4 < n) ? X[i0 + 4] : 0.f;
    }
}

template <int G>
__device__ __forceinline__ void st_store(LT_GLOBAL float *__restrict__ Y, int64_t g0, int lane,
                                         const StGroup<G> &q) {
#pragma unroll
    for (int u = 0; u < G; ++u) {
        const int64_t i0 = g0 + u * 1024 + threadIdx.x * 4;
        float left = __shfl_up(q.v[u].w, 1);
        float right = __shfl_down(q.v[u].x, 1);
        if (lane == 0) left = q.l[u];
        if (lane == WAVE - 1) right = q.r[u];
        float4 o;
        o.x = st_point(left, q.v[u].x, q.v[u].y);
        o.y = st_point(q.v[u].x, q.v[u].y, q.v[u].z);
        o.z = st_point(q.v[u].y, q.v[u].z, q.v[u].w);
        o.w = st_point(q.v[u].z, q.v[u].w, right);
        nt_store4(Y + i0, o);
    }
}

template <int G>
__device__ __forceinline__ void stencil_stream(int64_t xb, int64_t yb, int64_t n, int64_t lo, int64_t hi,
                                               int64_t s0, int64_t s1) {
    const int64_t end = hi < n ? hi : n;
    if (s1 > end) s1 = end;
    const bool aligned = ((xb + lo * 4) & 15) == 0 && ((yb + lo * 4) & 15) == 0 && ((s0 - lo) & 3) == 0;
    int64_t g = s0;
    if (aligned) {
        const int64_t step = (int64_t)G * 1024;
        const int64_t full = s0 + (s1 - s0) / step * step;
        const LT_GLOBAL float *X = gp<const float>(xb);
        LT_GLOBAL float *Y = gp<float>(yb);
        const int lane = threadIdx.x & (WAVE - 1);
        if (full > s0) {
            StGroup<G> cur;
            st_load<G>(X, n, g, lane, cur);
            for (; g < full; g += step) {
                StGroup<G> nxt;
                const bool more = g + step < full;
                if (more) st_load<G>(X, n, g + step, lane, nxt);
                st_store<G>(Y, g, lane, cur);
                if (more) cur = nxt;
            }
        }
    }
    for (; g < s1; g += 1024) stencil_span(xb, yb, n, lo, hi, g);
}

// Outputs of the task [lo, hi) in the groups of G spans of 1024 that start at
// g0, g0 + stride, g0 + 2 stride, ... (stride a multiple of G * 1024).  The
// batch drain gives tile j of a task with T tiles the groups j, j + T, ...:
// tiles handed out together then work on neighbouring groups, so the
// workgroups in flight stream through one region of memory instead of T
// separate ones.  Pipelined like stencil_stream; a ragged last group goes
// span by span.
template <int G>
__device__ __forceinline__ void stencil_strided(int64_t xb, int64_t yb, int64_t n, int64_t lo, int64_t hi,
                                                int64_t g0, int64_t stride) {
    constexpr int64_t GS = (int64_t)G * 1024;
    const int64_t end = hi < n ? hi : n;
    const bool aligned = ((xb + lo * 4) & 15) == 0 && ((yb + lo * 4) & 15) == 0 && ((g0 - lo) & 3) == 0;
    int64_t g = g0;
    if (aligned && g + GS <= end) {
        const LT_GLOBAL float *X = gp<const float>(xb);
        LT_GLOBAL float *Y = gp<float>(yb);
        const int lane = threadIdx.x & (WAVE - 1);
        StGroup<G> cur;
        st_load<G>(X, n, g, lane, cur);
        for (;;) {
            const int64_t gn = g + stride;
            const bool more = gn + GS <= end;
            StGroup<G> nxt;
            if (more) st_load<G>(X, n, gn, lane, nxt);
            st_store<G>(Y, g, lane, cur);
            g = gn;
            if (!more) break;
            cur = nxt;
        }
    }
    for (; g < end; g += stride)
        for (int64_t s = g; s < g + GS && s < end; s += 1024) stencil_span(xb, yb, n, lo, hi, s);
}

// ---------------------------------------------------------------- jacobi2d
// y[r][c] = 0.25*((x[r-1][c] + x[r+1][c]) + (x[r][c-1] + x[r][c+1])), zero
// outside the n x m field.
__device__ __forceinline__ float jpoint(float u, float d, float l, float r) {
    float v = u + d;
    float h = l + r;
    float s = v + h;
    return 0.25f * s;
}

struct JView {
    int64_t r0, r1, c0, c1;   // task box, clipped to the field
    int64_t y, x;             // pre-offset bases
    int64_t ys, xs;           // row strides
    int vec;                  // float4 layout usable
};

// Sliding three-row window over rows [r0, r1) for the lane's four columns
// starting at col (consecutive lanes hold consecutive column groups); any
// tile shape, alignment or raggedness.  Lanes past the last output column
// still load the halo column cend (read by their left neighbour lane) when
// it lies inside the field.
__device__ __forceinline__ void jacobi_window(const JView &t, int64_t n, int64_t m, int64_t col, int64_t r0,
                                              int64_t r1) {
    const int64_t cend = t.c1 < m ? t.c1 : m;
    const int64_t rcend = cend + 1 < m ? cend + 1 : m;
    const bool active = col < cend;
    const LT_GLOBAL float *X = gp<const float>(t.x);
    LT_GLOBAL float *Y = gp<float>(t.y);
    const int lane = threadIdx.x & (WAVE - 1);
    auto load4 = [&](int64_t r, float *v) {
        if (r < 0 || r >= n || col >= rcend) {
            v[0] = v[1] = v[2] = v[3] = 0.f;
            return;
        }
        const LT_GLOBAL float *p = X + r * t.xs + col;
        if (t.vec && active) {
            float4 q = ld4<float4>(p);
            v[0] = q.x;
            v[1] = q.y;
            v[2] = q.z;
            v[3] = q.w;
        } else {
            for (int j = 0; j < 4; ++j) v[j] = (col + j < rcend) ? p[j] : 0.f;
        }
    };
    float up[4], mid[4], dn[4];
    load4(r0 - 1, up);
    load4(r0, mid);
    for (int64_t r = r0; r < r1; ++r) {
        load4(r + 1, dn);
        float left = __shfl_up(mid[3], 1);
        float right = __shfl_down(mid[0], 1);
        const LT_GLOBAL float *row = X + r * t.xs;
        if (active && lane == 0) left = (col - 1 >= 0) ? row[col - 1] : 0.f;
        if (active && lane == WAVE - 1 && col + 3 < cend) right = (col + 4 < m) ? row[col + 4] : 0.f;
        if (active) {
            // columns at or past m were loaded as zero
            float o0 = jpoint(up[0], dn[0], left, mid[1]);
            float o1 = jpoint(up[1], dn[1], mid[0], mid[2]);
            float o2 = jpoint(up[2], dn[2], mid[1], mid[3]);
            float o3 = jpoint(up[3], dn[3], mid[2], right);
            LT_GLOBAL float *q = Y + r * t.ys + col;
            if (t.vec) {
                *(LT_GLOBAL float4 *)q = make_float4(o0, o1, o2, o3);
            } else {
                float o[4] = {o0, o1, o2, o3};
                for (int j = 0; j < 4; ++j)
                    if (col + j < cend) q[j] = o[j];
            }
        }
        for (int j = 0; j < 4; ++j) {
            up[j] = mid[j];
            mid[j] = dn[j];
        }
    }
}

// Rows [tr0, tr0 + RB) (within the task) of the 1024-column tile txi.
// Full tiles load all RB + 2 rows of the lane's four columns before any
// arithmetic (RB + 2 independent 16-byte loads in flight per lane) and write
// with non-temporal stores; ragged tiles slide a three-row window.
template <int RB>
__device__ __forceinline__ void jacobi_tile(const JView &t, int64_t n, int64_t m, int64_t tr0, int txi) {
    const int64_t r0 = tr0;
    const int64_t r1e = r0 + RB < t.r1 ? r0 + RB : t.r1;
    const int64_t r1 = r1e < n ? r1e : n;
    const int64_t cend = t.c1 < m ? t.c1 : m;            // outputs [c0, cend)
    const int64_t col = t.c0 + ((int64_t)txi * THREADS + threadIdx.x) * 4;
    const bool active = col < cend;
    const LT_GLOBAL float *X = gp<const float>(t.x);
    LT_GLOBAL float *Y = gp<float>(t.y);
    const int lane = threadIdx.x & (WAVE - 1);

    if (t.vec && r1 - r0 == RB) {
        float4 v[RB + 2];
#pragma unroll
        for (int i = 0; i < RB + 2; ++i) {
            const int64_t r = r0 - 1 + i;
            if (active && r >= 0 && r < n)
                v[i] = ld4<float4>(X + r * t.xs + col);
            else
                v[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        // the columns beside the wave's end lanes, before any store
        float el[RB], er[RB];
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const LT_GLOBAL float *row = X + (r0 + i) * t.xs;
            el[i] = active && lane == 0 && col - 1 >= 0 ? row[col - 1] : 0.f;
            er[i] = active && (lane == WAVE - 1 || col + 4 >= cend) && col + 4 < m ? row[col + 4] : 0.f;
        }
#pragma unroll
        for (int i = 1; i <= RB; ++i) {
            const int64_t r = r0 - 1 + i;
            const float4 up = v[i - 1], mid = v[i], dn = v[i + 1];
            float left = __shfl_up(mid.w, 1);
            float right = __shfl_down(mid.x, 1);
            if (lane == 0) left = el[i - 1];
            if (lane == WAVE - 1 || col + 4 >= cend) right = er[i - 1];
            if (active) {
                float4 o;
                o.x = jpoint(up.x, dn.x, left, mid.y);
                o.y = jpoint(up.y, dn.y, mid.x, mid.z);
                o.z = jpoint(up.z, dn.z, mid.y, mid.w);
                o.w = jpoint(up.w, dn.w, mid.z, right);
                nt_store4(Y + r * t.ys + col, o);
            }
        }
        return;
    }

    jacobi_window(t, n, m, col, r0, r1);
}

// Tiles of 256 columns and 4 RB rows starting at row tr0: wave w owns rows
// [tr0 + w RB, tr0 + (w + 1) RB) of its lanes' four columns each.  In a full
// tile only the two halo rows outside the tile come from memory; the rows
// between waves pass through LDS, so a tile loads 4 RB + 2 rows rather than
// 4 (RB + 2).  Ragged tiles slide a window per wave.  Called once per
// workgroup (the LDS rows are not reused).
template <int RB>
__device__ __forceinline__ void jacobi_stack(const JView &t, int64_t n, int64_t m, int64_t tr0, int txi) {
    const int w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    const int64_t rend = t.r1 < n ? t.r1 : n;
    const int64_t cend = t.c1 < m ? t.c1 : m;
    const int64_t cw = t.c0 + (int64_t)txi * (WAVE * 4);
    const int64_t col = cw + lane * 4;
    const int64_t r0 = tr0 + (int64_t)w * RB;
    // the branch is uniform over the workgroup: the full path has a barrier
    if (!t.vec || tr0 + 4 * RB > rend || cw + WAVE * 4 > cend) {
        const int64_t r1 = r0 + RB < rend ? r0 + RB : rend;
        if (r0 < r1) jacobi_window(t, n, m, col, r0, r1);
        return;
    }
    const LT_GLOBAL float *X = gp<const float>(t.x);
    LT_GLOBAL float *Y = gp<float>(t.y);
    __shared__ float4 s_first[THREADS / WAVE][WAVE], s_last[THREADS / WAVE][WAVE];
    constexpr int NW = THREADS / WAVE;
    float4 v[RB + 2];
#pragma unroll
    for (int i = 1; i <= RB; ++i) v[i] = ld4<float4>(X + (r0 - 1 + i) * t.xs + col);
    v[0] = make_float4(0.f, 0.f, 0.f, 0.f);
    v[RB + 1] = v[0];
    if (w == 0 && r0 >= 1) v[0] = ld4<float4>(X + (r0 - 1) * t.xs + col);
    if (w == NW - 1 && r0 + RB < n) v[RB + 1] = ld4<float4>(X + (r0 + RB) * t.xs + col);
    // the neighbouring columns of the wave's end lanes, loaded with the rows
    // (before any store, so no row waits for a load of its own)
    float el[RB], er[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) {
        const LT_GLOBAL float *row = X + (r0 + i) * t.xs;
        el[i] = lane == 0 && col - 1 >= 0 ? row[col - 1] : 0.f;
        er[i] = lane == WAVE - 1 && col + 4 < m ? row[col + 4] : 0.f;
    }
    s_first[w][lane] = v[1];
    s_last[w][lane] = v[RB];
    __syncthreads();
    if (w > 0) v[0] = s_last[w - 1][lane];
    if (w < NW - 1) v[RB + 1] = s_first[w + 1][lane];
#pragma unroll
    for (int i = 1; i <= RB; ++i) {
        const int64_t r = r0 - 1 + i;
        const float4 up = v[i - 1], mid = v[i], dn = v[i + 1];
        float left = __shfl_up(mid.w, 1);
        float right = __shfl_down(mid.x, 1);
        if (lane == 0) left = el[i - 1];
        if (lane == WAVE - 1) right = er[i - 1];
        float4 o;
        o.x = jpoint(up.x, dn.x, left, mid.y);
        o.y = jpoint(up.y, dn.y, mid.x, mid.z);
        o.z = jpoint(up.z, dn.z, mid.y, mid.w);
        o.w = jpoint(up.w, dn.w, mid.z, right);
        nt_store4(Y + r * t.ys + col, o);
    }
}

// Rows [tr0, tr0 + 8 NG) of the 1024-column tile txi, marched down in groups
// of 8 rows: the two rows above a group are carried over in registers from
// the group before, so each input row is loaded once per tile and only the
// tile's first group reads a halo row above it (plus one below the last).
// A group's 8 loads per lane, and the columns beside the wave's, are issued
// together before its arithmetic.
// Ragged tiles fall back to jacobi_tile per group.
template <int NG>
__device__ __forceinline__ void jacobi_march(const JView &t, int64_t n, int64_t m, int64_t tr0, int txi) {
    constexpr int RB = 8;
    const int64_t rend = t.r1 < n ? t.r1 : n;
    const int64_t r1 = tr0 + RB * NG < rend ? tr0 + RB * NG : rend;
    if (!t.vec || r1 - tr0 != RB * NG) {
        for (int g = 0; g < NG; ++g) {
            if (tr0 + g * RB >= rend) break;
            jacobi_tile<RB>(t, n, m, tr0 + g * RB, txi);
        }
        return;
    }
    const int64_t cend = t.c1 < m ? t.c1 : m;
    const int64_t col = t.c0 + ((int64_t)txi * THREADS + threadIdx.x) * 4;
    const bool active = col < cend;
    const LT_GLOBAL float *X = gp<const float>(t.x);
    LT_GLOBAL float *Y = gp<float>(t.y);
    const int lane = threadIdx.x & (WAVE - 1);
    auto load = [&](int64_t r) {
        return (active && r >= 0 && r < n) ? ld4<float4>(X + r * t.xs + col) : make_float4(0.f, 0.f, 0.f, 0.f);
    };
    // the lanes at a wave's ends (and at the tile's last column) take the
    // neighbouring columns from memory; they are loaded with the group's rows,
    // before its stores, so no row waits for a load of its own
    const bool need_l = active && lane == 0 && col - 1 >= 0;
    const bool need_r = active && (lane == WAVE - 1 || col + 4 >= cend) && col + 4 < m;
    float4 v[RB + 2];
    float el[RB], er[RB];
    v[0] = load(tr0 - 1);
    v[1] = load(tr0);
    for (int g = 0; g < NG; ++g) {
        const int64_t rb = tr0 + (int64_t)g * RB;
#pragma unroll
        for (int i = 0; i < RB; ++i) v[i + 2] = load(rb + 1 + i);
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const LT_GLOBAL float *row = X + (rb + i) * t.xs;
            el[i] = need_l ? row[col - 1] : 0.f;
            er[i] = need_r ? row[col + 4] : 0.f;
        }
#pragma unroll
        for (int i = 1; i <= RB; ++i) {
            const int64_t r = rb - 1 + i;
            const float4 up = v[i - 1], mid = v[i], dn = v[i + 1];
            float left = __shfl_up(mid.w, 1);
            float right = __shfl_down(mid.x, 1);
            if (lane == 0) left = el[i - 1];
            if (lane == WAVE - 1 || col + 4 >= cend) right = er[i - 1];
            if (active) {
                float4 o;
                o.x = jpoint(up.x, dn.x, left, mid.y);
                o.y = jpoint(up.y, dn.y, mid.x, mid.z);
                o.z = jpoint(up.z, dn.z, mid.y, mid.w);
                o.w = jpoint(up.w, dn.w, mid.z, right);
                nt_store4(Y + r * t.ys + col, o);
            }
        }
        v[0] = v[RB];
        v[1] = v[RB + 1];
    }
}

// ---------------------------------------------------------------- hist256
// Counts v[i] into LDS sub-histograms for the 4096-element chunks of [s0, s1)
// that start at s0, s0 + stride, s0 + 2*stride, ...; values outside [0, 256)
// are ignored.  Full aligned chunks load four 16-byte groups per lane before
// counting; ragged chunks go one by one.
//
// There are HIST_COPIES sub-histograms per workgroup: each wave has four,
// and lane l counts into copy l % 4, so lanes that see the same value (a
// skewed distribution puts a fifth of all values in one bin) are spread over
// four addresses.  Copies are HIST_STRIDE = 257 words apart, so one bin's
// copies sit in different LDS banks.
constexpr int HIST_COPIES = 16;
constexpr int HIST_STRIDE = 257;
constexpr int HIST_WORDS = HIST_COPIES * HIST_STRIDE;
__device__ __forceinline__ void hist_count(int *mine, int32_t b) {
    if ((uint32_t)b < 256u) atomicAdd(&mine[b], 1);
}

__device__ __forceinline__ void hist_span(int64_t vb, int64_t s0, int64_t s1, int64_t stride, int *sh) {
    const LT_GLOBAL int32_t *V = gp<const int32_t>(vb);
    int *mine = sh + ((threadIdx.x >> 6) * 4 + (threadIdx.x & 3)) * HIST_STRIDE;
    // the workgroup owns the 4096-element chunks starting at s0, s0 + stride,
    // ...; full aligned chunks are pipelined: the next chunk's four 16-byte
    // loads per lane are issued before the current chunk is counted
    const bool vec = ((vb + s0 * 4) & 15) == 0 && (stride % 4096) == 0;
    int64_t c = s0;
    if (vec && c + 4096 <= s1) {
        int4 cur[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) cur[u] = ld4<int4>(V + c + u * 1024 + threadIdx.x * 4);
        for (;;) {
            const int64_t cn = c + stride;
            const bool more = cn + 4096 <= s1;
            int4 nxt[4];
            if (more) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    nxt[u] = ld4<int4>(V + cn + u * 1024 + threadIdx.x * 4);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                hist_count(mine, cur[u].x);
                hist_count(mine, cur[u].y);
                hist_count(mine, cur[u].z);
                hist_count(mine, cur[u].w);
            }
            c = cn;
            if (!more) break;
#pragma unroll
            for (int u = 0; u < 4; ++u) cur[u] = nxt[u];
        }
    }
    // ragged or unaligned chunks, one element per lane at a time
    for (; c < s1; c += stride) {
        const int64_t ce = c + 4096 < s1 ? c + 4096 : s1;
        for (int64_t j = c + threadIdx.x; j < ce; j += THREADS) hist_count(mine, V[j]);
    }
}

// Adds the sub-histograms into the partial h (integer atomics: exact and
// order-free) and clears them.
__device__ __forceinline__ void hist_flush(int64_t hb, int *sh) {
    __syncthreads();
    LT_GLOBAL int32_t *H = gp<int32_t>(hb);
    const int b = threadIdx.x;
    int s = 0;
#pragma unroll
    for (int k = 0; k < HIST_COPIES; ++k) {
        s += sh[k * HIST_STRIDE + b];
        sh[k * HIST_STRIDE + b] = 0;
    }
    if (s) __hip_atomic_fetch_add(H + b, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
}

}  // namespace body
}  // namespace lt
