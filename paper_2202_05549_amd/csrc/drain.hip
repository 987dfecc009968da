// Persistent drain kernel: executes a queue of tasks from many launches in
// one dispatch.  Each workgroup takes the next (task, tile) ticket, waits
// until the task's dependency counters are reached (a bounded poll: after
// spin_limit polls it gives up, flags the error and skips the tile, so every
// wave exits), runs the tile with the same device body as the per-task
// kernels, and publishes completion with a release fence and a counter
// increment.  Tickets are handed out in program order and dependencies point
// to earlier tasks only, so a waiting workgroup always waits on tiles that
// running workgroups already hold: the drain makes progress.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "bodies.h"
#include "kernels.h"

namespace lt {

using namespace body;

template <int G, uint32_t KINDS>
__device__ __forceinline__ void run_tile(const DTask &t, int64_t local, int *sh) {
    // a build only carries the bodies in KINDS (the host never queues others)
    switch (t.kind) {
        case DK_TOUCH: {
            if constexpr (!(KINDS & (1u << DK_TOUCH))) break;
            const int64_t s0 = t.lo0 + local * DSPAN;
            for (int64_t sp = 0; sp < DSPAN; sp += THREADS) touch_span(t.y, t.n, t.lo0, t.hi0, s0 + sp);
            break;
        }
        case DK_STENCIL1D: {
            if constexpr (!(KINDS & (1u << DK_STENCIL1D))) break;
            // tile `local` of ntiles: the groups local, local + ntiles, ...
            constexpr int64_t GS = (int64_t)G * 1024;
            stencil_strided<G>(t.x, t.y, t.n, t.lo0, t.hi0, t.lo0 + local * GS, (int64_t)t.ntiles * GS);
            break;
        }
        case DK_JACOBI2D: {
            if constexpr (!(KINDS & (1u << DK_JACOBI2D))) break;
            JView v;
            v.r0 = t.lo0;
            v.r1 = t.hi0;
            v.c0 = t.lo1;
            v.c1 = t.hi1;
            v.y = t.y;
            v.x = t.x;
            v.ys = t.ys;
            v.xs = t.xs;
            v.vec = t.vec;
            const int tyi = (int)(local / t.tx), txi = (int)(local - (int64_t)tyi * t.tx);
            // the tile's DJROWS rows marched in groups of 8 (each input row
            // loaded once); jacobi_march clips at the task's last row
            jacobi_march<DJROWS / 8>(v, t.n, t.m, t.lo0 + (int64_t)tyi * DJROWS, txi);
            break;
        }
        case DK_HIST256: {
            if constexpr (!(KINDS & (1u << DK_HIST256))) break;
            // tile `local` of ntiles: the 4096-element chunks local,
            // local + ntiles, ... (neighbouring tiles read neighbouring chunks)
            const int64_t end = t.hi0 < t.n ? t.hi0 : t.n;
            hist_span(t.x, t.lo0 + local * 4096, end, (int64_t)t.ntiles * 4096, sh);
            hist_flush(t.y, sh);
            break;
        }
        case DK_SUM_PARTIALS: {
            if constexpr (!(KINDS & (1u << DK_SUM_PARTIALS))) break;
            // y[e] = sum over p of partial p at element e, e in [lo0, hi0);
            // partials are dense blocks of m elements starting at x
            const LT_GLOBAL int32_t *P = gp<const int32_t>(t.x);
            for (int64_t e = t.lo0 + threadIdx.x; e < t.hi0; e += THREADS) {
                int32_t acc = 0;
                for (int64_t p = 0; p < t.aux; ++p) acc += P[p * t.m + (e - t.lo0)];
                *at<int32_t>(t.y, e) = acc;
            }
            break;
        }
        default:
            break;
    }
}

template <int G, uint32_t KINDS>
__device__ __forceinline__ void drain_loop(const DTask *q, int ntasks, int32_t *ctr, int ticket_idx,
                                           int64_t total, int64_t spin_limit) {
    __shared__ int sh[HIST_WORDS];
    __shared__ int s_tile, s_task, s_ok;
    for (int i = threadIdx.x; i < HIST_WORDS; i += THREADS) sh[i] = 0;
    int cur = 0;
    int next = 0;
    if (threadIdx.x == 0) next = atomicAdd(&ctr[ticket_idx], 1);
    for (;;) {
        if (threadIdx.x == 0) {
            const int tile = next;
            // claim the following ticket now; its latency overlaps this tile
            if (tile < total) next = atomicAdd(&ctr[ticket_idx], 1);
            s_tile = tile;
        }
        __syncthreads();
        const int64_t tile = __builtin_amdgcn_readfirstlane(s_tile);
        if (tile >= total) break;
        if (threadIdx.x < WAVE) {
            // the task holding `tile`: the last one whose first tile is at
            // most `tile`.  First tiles grow with the task index and a
            // workgroup's tickets only grow, so the search starts at its
            // previous task.  The first wave tests 64 candidates per step
            // (one memory round trip): tasks cur + 1 .. cur + 64, galloping
            // to strides of 64 and 4096 while every candidate is passed,
            // then narrowing back to stride 1.  Passed candidates form a
            // prefix, so their count is the step.
            const int lane = threadIdx.x;
            int stride = 1;
            for (;;) {
                const int64_t idx = (int64_t)cur + (int64_t)(lane + 1) * stride;
                const bool passed = idx < ntasks && q[idx].tile_begin <= tile;
                const int adv = __popcll(__ballot(passed));
                cur += adv * stride;
                if (adv < WAVE) {
                    if (stride == 1) break;
                    stride >>= 6;
                } else if (stride < 4096) {
                    stride <<= 6;
                }
            }
        }
        if (threadIdx.x == 0) {
            const DTask &t = q[cur];
            int ok = 1;
            for (int d = 0; d < t.ndeps && ok; ++d) {
                int64_t spins = 0;
                while (__hip_atomic_load(&ctr[t.dep_ctr[d]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                       t.dep_val[d]) {
                    __builtin_amdgcn_s_sleep(2);
                    if (++spins > spin_limit) {
                        ok = 0;
                        atomicOr(&ctr[ticket_idx + 1], 1);
                        break;
                    }
                }
            }
            // acquire at device scope: invalidates this XCD's caches so the
            // predecessors' writes are seen (a full fence would also write
            // back the whole L2, which only a release needs)
            if (t.ndeps) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            s_task = cur;
            s_ok = ok;
        }
        __syncthreads();
        const int task = __builtin_amdgcn_readfirstlane(s_task);
        const DTask &t = q[task];
        if (__builtin_amdgcn_readfirstlane(s_ok)) run_tile<G, KINDS>(t, tile - t.tile_begin, sh);
        __syncthreads();
        if (threadIdx.x == 0) {
            const int32_t fl = t.flags;
            // release at device scope: the workgroup's plain stores (complete
            // at the barrier above) are written back from this XCD's L2
            if (fl & DF_RELEASE) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            else if (fl & DF_ATOMIC) __builtin_amdgcn_s_waitcnt(0);  // atomics performed
            int prev = atomicAdd(&ctr[task], 1);
            if (prev == t.ntiles - 1 && t.signal >= 0) atomicAdd(&ctr[t.signal], 1);
        }
    }
}

// Builds of the same loop for common sets of bodies and group sizes.  Each
// is a separate kernel so that its register allocation covers only the
// bodies it can meet: the 1-D streaming bodies with 2-vector groups fit in
// 64 VGPRs (eight waves per SIMD); with 4-vector groups, or with every
// body, a build takes 82-93 (five waves) but keeps more loads in flight.
constexpr uint32_t KB_TOUCH = 1u << DK_TOUCH, KB_ST = 1u << DK_STENCIL1D, KB_JAC = 1u << DK_JACOBI2D,
                   KB_HIST = 1u << DK_HIST256, KB_SUM = 1u << DK_SUM_PARTIALS;
constexpr uint32_t KB_1D = KB_TOUCH | KB_ST | KB_HIST | KB_SUM;
constexpr uint32_t KB_ALL = KB_1D | KB_JAC;

template <uint32_t KINDS, int G>
__global__ __launch_bounds__(256) void k_drain(const DTask *q, int ntasks, int32_t *ctr, int ticket_idx,
                                               int64_t total, int64_t spin_limit) {
    drain_loop<G, KINDS>(q, ntasks, ctr, ticket_idx, total, spin_limit);
}

hipError_t launch_drain(hipStream_t s, const DTask *q, int ntasks, int32_t *counters, int ticket_idx,
                        int64_t total_tiles, int nwg, int64_t spin_limit, uint32_t kinds, int vectors) {
    if (total_tiles <= 0 || ntasks <= 0) return hipSuccess;
    if (nwg < 1) nwg = 1;
    if ((int64_t)nwg > total_tiles) nwg = (int)total_tiles;
    const bool one_d = (kinds & ~KB_1D) == 0;
    if (vectors == 0) vectors = 4;
    void (*k)(const DTask *, int, int32_t *, int, int64_t, int64_t);
    if (one_d) k = vectors == 2 ? k_drain<KB_1D, 2> : k_drain<KB_1D, 4>;
    else if ((kinds & ~(KB_JAC | KB_SUM)) == 0) k = k_drain<KB_JAC | KB_SUM, 4>;
    else k = vectors == 2 ? k_drain<KB_ALL, 2> : k_drain<KB_ALL, 4>;
    hipLaunchKernelGGL(k, dim3((unsigned)nwg), dim3(256), 0, s, q, ntasks, counters, ticket_idx, total_tiles,
                       spin_limit);
    return hipGetLastError();
}

// Device scratch of the no-allocation batch issue: one copy per GPU, held
// until the process ends.  Host code never passes this name to a kernel or a
// copy (on the host it is only a stand-in for the symbol); it uses the
// address drain_scratch_address() looks up on each device.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

hipError_t drain_scratch_address(int device, void **out) {
    static std::mutex mu;
    static void *addr[64] = {};
    *out = nullptr;
    if (device < 0 || device >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t r = hipGetDevice(&cur);
        if (r != hipSuccess) return r;
        if (cur != device && (r = hipSetDevice(device)) != hipSuccess) return r;
        void *p = nullptr;
        r = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (r != hipSuccess) return r;
        addr[device] = p;
    }
    *out = addr[device];
    return hipSuccess;
}

}  // namespace lt
