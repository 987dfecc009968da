// C = A * B in float32 on the CDNA4 matrix cores (v_mfma_f32_32x32x2f32).
//
// One task is one superblock of C (thread (i, j) owns C[i][j]; annotation
// read A[i, :], read B[:, j], write C[i, j]).  A workgroup of 512 threads
// computes a 256 x 256 block of C: its eight waves (two per SIMD, so one
// hides the other's LDS reads) each own 128 x 64 as 4 x 2 MFMA blocks of
// 32 x 32 (128 accumulators per lane).  K advances in
// tiles of 32 staged in LDS: A transposed to [k][m] (odd row stride, so the
// transposing stores do not collide on banks), B as [k][n].  The LDS tile is
// double-buffered and the next tile's global loads are in flight while the
// current one feeds the matrix cores.  Rows/columns/K beyond the operands are
// read as zero and C is written only inside the task and the matrix.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "bodies.h"
#include "kernels.h"

namespace lt {

namespace {

constexpr int BM = 256, BN = 256, BK = 32;
constexpr int LDA = BM + 1;   // As[k][m]
constexpr int LDB = BN + 4;   // Bs[k][n]
constexpr int GMAX = 8;       // tasks per dispatch
constexpr int GM = 8;         // block rows per group of the block order

typedef float f32x16 __attribute__((ext_vector_type(16)));

struct GTask {
    int64_t i0, i1, j0, j1;   // C rows / columns of the task, clipped to M, N
    int64_t a, b, c;          // pre-offset bases
    int64_t as, bs, cs;       // row strides
    int tn;                   // column tiles
    int vec;                  // 16-byte loads usable for A and B
};

struct GArgs {
    int64_t K;
    int ntask, nblocks;
    int begin[GMAX + 1];
    GTask t[GMAX];
};


}  // namespace

// The fields of one task, held in registers for the whole block.
struct GReg {
    int64_t i1, j1, as, bs, cs, K;
    const LT_GLOBAL float *A;
    const LT_GLOBAL float *B;
    LT_GLOBAL float *C;
};

// One 256 x 256 block of C.  FULL: the block lies inside the matrix, K is a
// multiple of 32 and 16-byte loads are usable, so the loads carry no guards.
template <bool FULL>
__device__ __forceinline__ void gemm_block(const GReg &t, int64_t m0, int64_t n0, float (*As)[BK][LDA],
                                           float (*Bs)[BK][LDB], int vec) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 2) * 128, wn = (wave & 3) * 64;
    const int64_t K = t.K;

    // global -> register staging of one K tile
    // A: thread covers rows tid/8 + 64*j, k4 = tid%8 (4 float4)
    // B: thread covers k = tid/64 + 8*j, n4 = tid%64 (4 float4)
    float4 ra[4], rb[4];
    const int a_row = tid >> 3, a_k4 = tid & 7;
    const int b_k = tid >> 6, b_n4 = tid & 63;
    const LT_GLOBAL float *Ab = t.A + (m0 + a_row) * t.as + a_k4 * 4;
    const LT_GLOBAL float *Bb = t.B + (int64_t)b_k * t.bs + n0 + b_n4 * 4;

    auto load_tile = [&](int64_t k0) {
        if constexpr (FULL) {
#pragma unroll
            for (int j = 0; j < 4; ++j) ra[j] = body::ld4<float4>(Ab + 64 * j * t.as + k0);
#pragma unroll
            for (int j = 0; j < 4; ++j) rb[j] = body::ld4<float4>(Bb + (k0 + 8 * j) * t.bs);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t r = m0 + a_row + 64 * j;
                const int64_t k = k0 + a_k4 * 4;
                if (vec && r < t.i1 && k + 3 < K) {
                    ra[j] = body::ld4<float4>(t.A + r * t.as + k);
                } else {
                    float v[4];
                    for (int q = 0; q < 4; ++q) v[q] = (r < t.i1 && k + q < K) ? t.A[r * t.as + k + q] : 0.f;
                    ra[j] = make_float4(v[0], v[1], v[2], v[3]);
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t k = k0 + b_k + 8 * j;
                const int64_t c = n0 + b_n4 * 4;
                if (vec && k < K && c + 3 < t.j1) {
                    rb[j] = body::ld4<float4>(t.B + k * t.bs + c);
                } else {
                    float v[4];
                    for (int q = 0; q < 4; ++q) v[q] = (k < K && c + q < t.j1) ? t.B[k * t.bs + c + q] : 0.f;
                    rb[j] = make_float4(v[0], v[1], v[2], v[3]);
                }
            }
        }
    };
    auto store_tile = [&](int buf) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = a_row + 64 * j;
            As[buf][a_k4 * 4 + 0][m] = ra[j].x;
            As[buf][a_k4 * 4 + 1][m] = ra[j].y;
            As[buf][a_k4 * 4 + 2][m] = ra[j].z;
            As[buf][a_k4 * 4 + 3][m] = ra[j].w;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) *reinterpret_cast<float4 *>(&Bs[buf][b_k + 8 * j][b_n4 * 4]) = rb[j];
    };

    f32x16 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

    const int nk = (int)((K + BK - 1) / BK);
    load_tile(0);
    store_tile(0);
    __syncthreads();
    const int half = lane >> 5, l32 = lane & 31;
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        const bool more = kt + 1 < nk;
        if (more) load_tile((int64_t)(kt + 1) * BK);
        // fragments of k-step s + 1 are read from LDS before the matrix-core
        // instructions of step s are issued, so their latency is hidden
        float av[2][4], bv[2][2];
#pragma unroll
        for (int i = 0; i < 4; ++i) av[0][i] = As[buf][half][wm + 32 * i + l32];
#pragma unroll
        for (int j = 0; j < 2; ++j) bv[0][j] = Bs[buf][half][wn + 32 * j + l32];
#pragma unroll
        for (int s = 0; s < BK / 2; ++s) {
            const int cur = s & 1;
            if (s + 1 < BK / 2) {
                const int k = 2 * (s + 1) + half;
#pragma unroll
                for (int i = 0; i < 4; ++i) av[cur ^ 1][i] = As[buf][k][wm + 32 * i + l32];
#pragma unroll
                for (int j = 0; j < 2; ++j) bv[cur ^ 1][j] = Bs[buf][k][wn + 32 * j + l32];
            }
            // the next tile goes into the other LDS buffer half-way through
            // this one, so its stores overlap the matrix-core work
            if (s == BK / 4 && more) store_tile(buf ^ 1);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[cur][i], bv[cur][j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }

    // accumulator v of a 32 x 32 block holds row 8*(v/4) + 4*(lane/32) + v%4,
    // column lane%32
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t col = n0 + wn + 32 * j + l32;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int64_t row = m0 + wm + 32 * i + 8 * (v >> 2) + 4 * half + (v & 3);
                if (FULL || (row < t.i1 && col < t.j1)) t.C[row * t.cs + col] = acc[i][j][v];
            }
        }
}

__global__ __launch_bounds__(512, 1) void k_gemm(GArgs g) {
    __shared__ float As[2][BK][LDA];
    __shared__ float Bs[2][BK][LDB];

    const int b = body::xcd_remap(blockIdx.x, g.nblocks);
    const int ti = body::find_task(g.begin, g.ntask, b);
    const GTask &tk = g.t[ti];
    // Blocks of a task go in groups of GM block rows, column by column within
    // a group, so that a run of 32 consecutive blocks (one XCD's share of a
    // 16 x 16 task after xcd_remap) covers 8 x 4 blocks: the XCD's L2 then
    // serves 12 operand strips instead of the 18 of two whole block rows.
    // A bijection onto the task's blocks for any shape.
    const int local = b - g.begin[ti];
    const int tm = (g.begin[ti + 1] - g.begin[ti]) / tk.tn;
    const int grp = local / (GM * tk.tn);
    const int first = grp * GM;
    const int gsz = tm - first < GM ? tm - first : GM;
    const int r = local - grp * GM * tk.tn;
    const int tmi = first + r % gsz, tni = r / gsz;
    const int64_t m0 = tk.i0 + (int64_t)tmi * BM;
    const int64_t n0 = tk.j0 + (int64_t)tni * BN;
    // global-address-space pointers: global (not flat) loads do not hold up
    // the LDS reads that feed the matrix cores
    GReg t;
    t.i1 = tk.i1;
    t.j1 = tk.j1;
    t.as = tk.as;
    t.bs = tk.bs;
    t.cs = tk.cs;
    t.K = g.K;
    t.A = body::gp<const float>(tk.a);
    t.B = body::gp<const float>(tk.b);
    t.C = body::gp<float>(tk.c);
    const int vec = tk.vec;
    if (vec && m0 + BM <= t.i1 && n0 + BN <= t.j1 && t.K % BK == 0)
        gemm_block<true>(t, m0, n0, As, Bs, vec);
    else
        gemm_block<false>(t, m0, n0, As, Bs, vec);
}

hipError_t launch_gemm_f32(const KLaunch &L) {
    GArgs g;
    const int64_t M = L.iarg[0], N = L.iarg[1];
    g.K = L.iarg[2];
    if (L.ntask > GMAX) return hipErrorInvalidValue;
    g.ntask = L.ntask;
    int64_t nb = 0;
    for (int i = 0; i < L.ntask; ++i) {
        const KTask &k = L.tasks[i];
        GTask &t = g.t[i];
        t.i0 = k.lo[0];
        t.i1 = k.hi[0] < M ? k.hi[0] : M;
        t.j0 = k.lo[1];
        t.j1 = k.hi[1] < N ? k.hi[1] : N;
        t.c = k.v[3].base;
        t.cs = k.v[3].s[0];
        t.a = k.v[4].base;
        t.as = k.v[4].s[0];
        t.b = k.v[5].base;
        t.bs = k.v[5].s[0];
        // 16-byte loads need every row start of A (from column 0) and of B
        // (from the task's first column) on a 16-byte boundary
        t.vec = (t.as % 4 == 0) && (t.bs % 4 == 0) && (t.a % 16 == 0) && ((t.b + t.j0 * 4) % 16 == 0) &&
                (t.j0 % 4 == 0);
        int64_t rows = t.i1 - t.i0, cols = t.j1 - t.j0;
        int64_t tm = rows > 0 ? (rows + BM - 1) / BM : 0;
        t.tn = cols > 0 ? (int)((cols + BN - 1) / BN) : 0;
        g.begin[i] = (int)nb;
        nb += tm * t.tn;
    }
    g.begin[L.ntask] = (int)nb;
    g.nblocks = (int)nb;
    if (nb == 0) return hipSuccess;  // K = 0 still runs: C becomes the empty sum, 0
    hipLaunchKernelGGL(k_gemm, dim3((unsigned)nb), dim3(512), 0, L.stream, g);
    return hipGetLastError();
}

}  // namespace lt
