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

template <class T>
__device__ __forceinline__ T *at(int64_t base, int64_t idx) {
    return reinterpret_cast<T *>(base) + idx;
}

// 16-byte store without cache retention (streaming output)
__device__ __forceinline__ void nt_store4(float *p, float4 v) {
    f32x4 w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<f32x4 *>(p));
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
    const float *X = reinterpret_cast<const float *>(xb);
    float *Y = reinterpret_cast<float *>(yb);
    const bool aligned = ((xb + lo * 4) & 15) == 0 && ((yb + lo * 4) & 15) == 0 && ((span0 - lo) & 3) == 0;
    float v[4];
    if (aligned && i0 + 3 < end) {
        float4 q = *reinterpret_cast<const float4 *>(X + i0);
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
        *reinterpret_cast<float4 *>(Y + i0) = make_float4(o[0], o[1], o[2], o[3]);
    } else {
        for (int j = 0; j < 4; ++j)
            if (i0 + j < end) Y[i0 + j] = o[j];
    }
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
    const int64_t rcend = cend + 1 < m ? cend + 1 : m;     // inputs read up to rcend
    const int64_t col = t.c0 + ((int64_t)txi * THREADS + threadIdx.x) * 4;
    const bool active = col < cend;
    const float *X = reinterpret_cast<const float *>(t.x);
    float *Y = reinterpret_cast<float *>(t.y);
    const int lane = threadIdx.x & (WAVE - 1);

    if (t.vec && r1 - r0 == RB) {
        float4 v[RB + 2];
#pragma unroll
        for (int i = 0; i < RB + 2; ++i) {
            const int64_t r = r0 - 1 + i;
            if (active && r >= 0 && r < n)
                v[i] = *reinterpret_cast<const float4 *>(X + r * t.xs + col);
            else
                v[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int i = 1; i <= RB; ++i) {
            const int64_t r = r0 - 1 + i;
            const float4 up = v[i - 1], mid = v[i], dn = v[i + 1];
            float left = __shfl_up(mid.w, 1);
            float right = __shfl_down(mid.x, 1);
            const float *row = X + r * t.xs;
            if (active && lane == 0) left = (col - 1 >= 0) ? row[col - 1] : 0.f;
            if (active && (lane == WAVE - 1 || col + 4 >= cend)) right = (col + 4 < m) ? row[col + 4] : 0.f;
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

    // lanes past the last output column still load the halo column cend
    // (read by their left neighbour lane) when it lies inside the field
    auto load4 = [&](int64_t r, float *v) {
        if (r < 0 || r >= n || col >= rcend) {
            v[0] = v[1] = v[2] = v[3] = 0.f;
            return;
        }
        const float *p = X + r * t.xs + col;
        if (t.vec && active) {
            float4 q = *reinterpret_cast<const float4 *>(p);
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
        const float *row = X + r * t.xs;
        if (active && lane == 0) left = (col - 1 >= 0) ? row[col - 1] : 0.f;
        if (active && lane == WAVE - 1 && col + 3 < cend) right = (col + 4 < m) ? row[col + 4] : 0.f;
        if (active) {
            // columns at or past m were loaded as zero
            float o0 = jpoint(up[0], dn[0], left, mid[1]);
            float o1 = jpoint(up[1], dn[1], mid[0], mid[2]);
            float o2 = jpoint(up[2], dn[2], mid[1], mid[3]);
            float o3 = jpoint(up[3], dn[3], mid[2], right);
            float *q = Y + r * t.ys + col;
            if (t.vec) {
                *reinterpret_cast<float4 *>(q) = make_float4(o0, o1, o2, o3);
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

// ---------------------------------------------------------------- hist256
// Counts v[i] for i in [s0, s1) into the wave's LDS sub-histogram sh[wave];
// values outside [0, 256) are ignored.  Grid-stride over `stride` elements.
__device__ __forceinline__ void hist_span(int64_t vb, int64_t s0, int64_t s1, int64_t stride, int *sh) {
    const int32_t *V = reinterpret_cast<const int32_t *>(vb);
    int *mine = sh + (threadIdx.x >> 6) * 256;
    for (int64_t i = s0 + threadIdx.x; i < s1; i += stride) {
        int32_t b = V[i];
        if ((uint32_t)b < 256u) atomicAdd(&mine[b], 1);
    }
}

// Adds the four sub-histograms into the partial h (integer atomics: exact
// and order-free) and clears them.
__device__ __forceinline__ void hist_flush(int64_t hb, int *sh) {
    __syncthreads();
    int32_t *H = reinterpret_cast<int32_t *>(hb);
    const int b = threadIdx.x;
    int s = sh[b] + sh[256 + b] + sh[512 + b] + sh[768 + b];
    if (s) atomicAdd(H + b, s);
    sh[b] = sh[256 + b] = sh[512 + b] = sh[768 + b] = 0;
    __syncthreads();
}

}  // namespace body
}  // namespace lt
