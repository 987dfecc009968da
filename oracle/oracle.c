/*
 * CPU oracle for the annotated-launch workloads -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load this library.  The product path never calls it and shares no code
 * with it.
 *
 * What it computes.  The method (Lightning, Sec. 2.4 "Execution Planner")
 * promises that a launch split into superblocks, with its arrays split into
 * chunks, spilled and reordered, gives the result of running the kernel body
 * for every thread index of the whole grid on whole arrays, launches in
 * program order (sequential consistency, Sec. 1 and Sec. 2.4; distributions
 * change only performance, Sec. 2.4).  So each routine below is the kernel
 * body applied to every index of the unchunked domain.  There are no chunks,
 * regions or DAGs here.
 *
 * Arithmetic.  The workloads store float32 data, and each body fixes its
 * operation order (stated per routine), so float32 results are reproducible
 * operation by operation.  Products by 0.25 and 0.5 are exact, so only the
 * additions round.  The GEMM reference accumulates in float64.  Build with
 * -ffp-contract=off so the compiler does not fuse a multiply and an add.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

/* ------------------------------------------------------------------ stencils
 * 1-D three-point stencil (the Sec. 3.5 example kernel with the workload's
 * weights 1/4, 1/2, 1/4):
 *     y[i] = 0.25 * (x[i-1] + x[i+1]) + 0.5 * x[i],   0 <= i < n,
 * with x[-1] = x[n] = 0 (the example kernel's guard reads 0 outside the
 * array).  Order: the two neighbours are added first, then scaled, then the
 * scaled centre is added.
 */
void or_stencil1d_f32(int64_t n, const float *x, float *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        float left = (i - 1 >= 0) ? x[i - 1] : 0.0f;
        float mid = x[i];
        float right = (i + 1 < n) ? x[i + 1] : 0.0f;
        float s = left + right;
        float t = 0.25f * s;
        float u = 0.5f * mid;
        y[i] = t + u;
    }
}

/* One 2-D Jacobi sweep of the five-point Laplace stencil on an n x m
 * row-major field: every cell is an unknown and neighbours outside the field
 * are held at zero (Dirichlet zero boundary):
 *     y[r][c] = 0.25 * ((x[r-1][c] + x[r+1][c]) + (x[r][c-1] + x[r][c+1])).
 * The centre value does not enter.  Order: vertical pair, horizontal pair,
 * their sum, then the exact scaling by 1/4.
 */
void or_jacobi2d_sweep_f32(int64_t n, int64_t m, const float *x, float *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        for (int64_t c = 0; c < m; ++c) {
            float up = (r - 1 >= 0) ? x[(r - 1) * m + c] : 0.0f;
            float down = (r + 1 < n) ? x[(r + 1) * m + c] : 0.0f;
            float left = (c - 1 >= 0) ? x[r * m + c - 1] : 0.0f;
            float right = (c + 1 < m) ? x[r * m + c + 1] : 0.0f;
            float v = up + down;
            float h = left + right;
            float s = v + h;
            y[r * m + c] = 0.25f * s;
        }
    }
}

/* `sweeps` ping-pong sweeps: sweep t reads buffer t%2 and writes (t+1)%2,
 * with buffer 0 = a and buffer 1 = b, as in the host sample of Sec. 3.6 that
 * swaps input and output after every launch.  Returns the index (0 or 1) of
 * the buffer holding the last result; a has the input on entry.
 */
int or_jacobi2d_f32(int64_t n, int64_t m, int sweeps, float *a, float *b)
{
    float *buf[2] = {a, b};
    for (int t = 0; t < sweeps; ++t)
        or_jacobi2d_sweep_f32(n, m, buf[t & 1], buf[(t + 1) & 1]);
    return sweeps & 1;
}

/* --------------------------------------------------------------------- GEMM
 * C = A * B for row-major A (M x K, leading dimension lda) and B (K x N, ldb),
 * accumulated in float64 from the float32 inputs (the workload's matrix
 * product, Sec. 4.2 "GEMM", as the thread-(i,j) definition of Sec. 2.3).
 * The plain dot product over k = 0..K-1 in order.
 */
void or_gemm_f64(int64_t M, int64_t N, int64_t K, const float *A, int64_t lda,
                 const float *B, int64_t ldb, double *C, int64_t ldc)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
        double *ci = C + i * ldc;
        for (int64_t j = 0; j < N; ++j)
            ci[j] = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            double a = (double)A[i * lda + k];
            const float *bk = B + k * ldb;
            for (int64_t j = 0; j < N; ++j)
                ci[j] += a * (double)bk[j];
        }
    }
}

/* Selected entries C[ii[s]][jj[s]] of A * B in float64, and the matching
 * entries of |A| * |B| (the scale of the componentwise error bound).
 */
void or_gemm_entries_f64(int64_t K, const float *A, int64_t lda, const float *B,
                         int64_t ldb, int64_t count, const int64_t *ii,
                         const int64_t *jj, double *val, double *absval)
{
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < count; ++s) {
        double acc = 0.0, aacc = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            double p = (double)A[ii[s] * lda + k] * (double)B[k * ldb + jj[s]];
            acc += p;
            aacc += fabs(p);
        }
        val[s] = acc;
        absval[s] = aacc;
    }
}

/* y = op(A) x in float64 for a row-major float32 M x K matrix A, where op
 * takes |a| when `absval` is non-zero.  Used for randomized product checks
 * (Freivalds): C r against A (B r).
 */
void or_matvec_f64(int64_t M, int64_t K, const float *A, int64_t lda,
                   const double *x, double *y, int absval)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
        const float *ai = A + i * lda;
        double acc = 0.0;
        if (absval) {
            for (int64_t k = 0; k < K; ++k)
                acc += fabs((double)ai[k]) * x[k];
        } else {
            for (int64_t k = 0; k < K; ++k)
                acc += (double)ai[k] * x[k];
        }
        y[i] = acc;
    }
}

/* Y = op(A) X in float64 for a row-major float32 M x K matrix A and a
 * row-major float64 K x m matrix X with few columns (m of about 16): the
 * matvec above for m right-hand sides at once, so a randomized check with
 * one probe vector per column panel reads A once.
 */
void or_matmul_thin_f64(int64_t M, int64_t K, const float *A, int64_t lda,
                        int64_t m, const double *X, double *Y, int absval)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
        const float *ai = A + i * lda;
        double *yi = Y + i * m;
        for (int64_t c = 0; c < m; ++c)
            yi[c] = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            double a = (double)ai[k];
            if (absval)
                a = fabs(a);
            const double *xk = X + k * m;
            for (int64_t c = 0; c < m; ++c)
                yi[c] += a * xk[c];
        }
    }
}

/* ---------------------------------------------------------------- histogram
 * 256-bin integer histogram: h[b] = #{ i : v[i] == b }.  The annotation's
 * reduce(+) mode (Sec. 2.3) makes the target the sum of all contributions,
 * starting from the identity 0, so h is overwritten.  Values outside [0, 256)
 * contribute nothing.
 */
void or_hist256_i32(int64_t n, const int32_t *v, int32_t *h)
{
    memset(h, 0, 256 * sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) {
        int32_t b = v[i];
        if (b >= 0 && b < 256)
            h[b] += 1;
    }
}

/* ------------------------------------------------------------------ k-means
 * Assignment step of k-means (Sec. 4.2 "K-Means"): each point takes the
 * label of its nearest centre in squared Euclidean distance.  The distance is
 * a float32 fused multiply-add chain over the coordinates in order, starting
 * from 0:  d = x[j] - c[j];  acc = fma(d, d, acc).  Ties go to the smallest
 * centre index (strict less-than while scanning k upward).  X is N x dim,
 * centres K x dim, both row-major.
 */
void or_kmeans_assign_f32(int64_t N, int64_t dim, int64_t K, const float *X,
                          const float *Cen, int32_t *lab)
{
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < N; ++p) {
        const float *xp = X + p * dim;
        float best = INFINITY;
        int32_t arg = 0;
        for (int64_t k = 0; k < K; ++k) {
            const float *ck = Cen + k * dim;
            float acc = 0.0f;
            for (int64_t j = 0; j < dim; ++j) {
                float d = xp[j] - ck[j];
                acc = fmaf(d, d, acc);
            }
            if (acc < best) {
                best = acc;
                arg = (int32_t)k;
            }
        }
        lab[p] = arg;
    }
}

/* Float64 squared distance of point p to centre k: the exact-arithmetic scale
 * used to decide whether two labels are a near-tie.
 */
double or_kmeans_dist_f64(int64_t dim, const float *x, const float *c)
{
    double acc = 0.0;
    for (int64_t j = 0; j < dim; ++j) {
        double d = (double)x[j] - (double)c[j];
        acc += d * d;
    }
    return acc;
}

/* -------------------------------------------------------------- reductions
 * reduce(f) (Sec. 2.3): the contributions of all threads are folded with f
 * into the target, which is overwritten by the fold; the fold starts from
 * f's identity (0 for +, 1 for *, +inf for min, -inf for max), so a target
 * element nobody contributes to ends as the identity.  Here the fold runs in
 * float64 over float32 contributions, in index order; min and max are exact
 * in any order.
 *
 * Row reduction -- the Sec. 2.3 example "global [i, j] => read A[i,j],
 * reduce(+) sum[i]":  out[i] = f over j of A[i][j] for an n x m matrix A.
 * op: 0 = +, 1 = *, 2 = min, 3 = max.  abs_out (may be NULL) receives the
 * sum over j of |A[i][j]|, the scale of the rounding bound of a float sum.
 */
void or_reduce_rows_f64(int64_t n, int64_t m, int op, const float *A, double *out, double *abs_out)
{
    for (int64_t i = 0; i < n; ++i) {
        double acc = op == 0 ? 0.0 : op == 1 ? 1.0 : op == 2 ? INFINITY : -INFINITY;
        double sa = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            const double a = (double)A[i * m + j];
            if (op == 0) acc += a;
            else if (op == 1) acc *= a;
            else if (op == 2) acc = a < acc ? a : acc;
            else acc = a > acc ? a : acc;
            sa += fabs(a);
        }
        out[i] = acc;
        if (abs_out) abs_out[i] = sa;
    }
}

/* K-means centre update (the reduction step of the K-Means benchmark,
 * Sec. 4.1, whose centre calculation runs on the GPU through reduce(+)):
 *     sums[k][j] = sum over points p with lab[p] = k of X[p][j]   (float64)
 *     counts[k]  = number of points p with lab[p] = k
 *     abss[k][j] = sum over the same p of |X[p][j]|   (rounding scale; may be NULL)
 * Points are visited in index order.  Labels outside [0, K) contribute
 * nothing.
 */
void or_kmeans_update_f64(int64_t N, int64_t dim, int64_t K, const float *X, const int32_t *lab,
                          double *sums, int64_t *counts, double *abss)
{
    for (int64_t e = 0; e < K * dim; ++e) {
        sums[e] = 0.0;
        if (abss) abss[e] = 0.0;
    }
    for (int64_t k = 0; k < K; ++k)
        counts[k] = 0;
    for (int64_t p = 0; p < N; ++p) {
        const int32_t k = lab[p];
        if (k < 0 || k >= K)
            continue;
        counts[k] += 1;
        for (int64_t j = 0; j < dim; ++j) {
            sums[k * dim + j] += (double)X[p * dim + j];
            if (abss) abss[k * dim + j] += fabs((double)X[p * dim + j]);
        }
    }
}

/* New centres from the update: cen[k][j] = sums[k][j] / counts[k], computed
 * in float64 and rounded once to float32; a cluster with no points keeps its
 * previous centre (cen is updated in place).
 */
void or_kmeans_centres_f32(int64_t K, int64_t dim, const double *sums, const int64_t *counts, float *cen)
{
    for (int64_t k = 0; k < K; ++k) {
        if (counts[k] == 0)
            continue;
        for (int64_t j = 0; j < dim; ++j)
            cen[k * dim + j] = (float)(sums[k * dim + j] / (double)counts[k]);
    }
}

/* ------------------------------------------------------------------- touch
 * Exactly-once probe: every thread index i of the grid with i < n adds one to
 * y[i].  Running it over the whole grid leaves y[i] = y0[i] + 1 for i < n.
 */
void or_touch_i32(int64_t n, int64_t grid, int32_t *y)
{
    for (int64_t i = 0; i < grid && i < n; ++i)
        y[i] += 1;
}

/* Number of OpenMP threads the parallel loops above use. */
#ifdef _OPENMP
#include <omp.h>
#endif
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
