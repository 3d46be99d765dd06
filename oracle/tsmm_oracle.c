/*
 * FP64 CPU oracle for the pre-packed tall-and-skinny matrix multiply.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no header, helper, table
 * or constant with the GPU path.
 *
 * What it computes is the plain definition of the operation (AutoTSMM,
 * Sec. I, Eq. (1); the output line of Algorithm 1):
 *
 *     C = alpha * A * B + beta * C0
 *
 * The method's packing and tiling (Alg. 1, Sec. IV-A) only reorder memory
 * traffic and the order of the summation, so the oracle is the definition
 * written out and nothing else:
 *   - every product and every sum in IEEE binary64, one rounding per
 *     operation (build with -ffp-contract=off, no fast-math);
 *   - each dot product summed from s = 0.0 with the shared index ascending;
 *   - epilogue t = alpha*s, then t = t + beta*c0 (two separately rounded
 *     operations), with the reference-BLAS conventions the paper leaves
 *     open: beta == 0 never reads C0, alpha == 0 never reads A or B,
 *     k == 0 gives beta*C0, m == 0 or n == 0 does nothing;
 *   - OpenMP splits output rows only, so a dot product is never split and
 *     the result does not depend on the thread count.
 *
 * Layouts are row-major and contiguous.  "op N": A is m x k, B is k x n.
 * "op T" (the reduction shape over a long shared dimension): A is K x m,
 * B is K x n and C = alpha * A^T * B + beta * C0.
 *
 * The bf16 split (oracle_split_bf16) is the plain bit-level definition of
 * round-to-nearest-even conversion from binary32 to bfloat16 applied to the
 * running residual; it pins the packed planes of the split-bf16 mode.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_BAD_ARG 1

static int pick_threads(int threads)
{
#ifdef _OPENMP
    return threads > 0 ? threads : omp_get_max_threads();
#else
    (void)threads;
    return 1;
#endif
}

/* C(m x n) = alpha * A(m x k) * B(k x n) + beta * C0(m x n), row-major. */
int oracle_gemm_n_f64(int64_t m, int64_t n, int64_t k, double alpha,
                      const double *A, const double *B, double beta,
                      const double *C0, double *C, int threads)
{
    int64_t i;
    if (m < 0 || n < 0 || k < 0) return ORACLE_BAD_ARG;
    if (m == 0 || n == 0) return ORACLE_OK;
    if (!C) return ORACLE_BAD_ARG;
    if (alpha != 0.0 && k > 0 && (!A || !B)) return ORACLE_BAD_ARG;
    if (beta != 0.0 && !C0) return ORACLE_BAD_ARG;
    threads = pick_threads(threads);
#pragma omp parallel for schedule(static) num_threads(threads)
    for (i = 0; i < m; ++i) {
        int64_t j, l;
        for (j = 0; j < n; ++j) {
            double t = 0.0;
            if (alpha != 0.0) {
                double s = 0.0;
                for (l = 0; l < k; ++l) s = s + A[i * k + l] * B[l * n + j];
                t = alpha * s;
            }
            if (beta != 0.0) t = t + beta * C0[i * n + j];
            C[i * n + j] = t;
        }
    }
    return ORACLE_OK;
}

/* C(m x n) = alpha * A^T * B + beta * C0, A is K x m, B is K x n, row-major.
 * Loop order i -> r -> j keeps r ascending for every output element. */
int oracle_gemm_t_f64(int64_t m, int64_t n, int64_t K, double alpha,
                      const double *A, const double *B, double beta,
                      const double *C0, double *C, int threads)
{
    int64_t i;
    if (m < 0 || n < 0 || K < 0) return ORACLE_BAD_ARG;
    if (m == 0 || n == 0) return ORACLE_OK;
    if (!C) return ORACLE_BAD_ARG;
    if (alpha != 0.0 && K > 0 && (!A || !B)) return ORACLE_BAD_ARG;
    if (beta != 0.0 && !C0) return ORACLE_BAD_ARG;
    threads = pick_threads(threads);
#pragma omp parallel for schedule(static) num_threads(threads)
    for (i = 0; i < m; ++i) {
        int64_t j, r;
        double *row = C + i * n;
        for (j = 0; j < n; ++j) row[j] = 0.0;
        if (alpha != 0.0) {
            for (r = 0; r < K; ++r) {
                const double a = A[r * m + i];
                const double *brow = B + r * n;
                for (j = 0; j < n; ++j) row[j] = row[j] + a * brow[j];
            }
            for (j = 0; j < n; ++j) row[j] = alpha * row[j];
        }
        if (beta != 0.0)
            for (j = 0; j < n; ++j) row[j] = row[j] + beta * C0[i * n + j];
    }
    return ORACLE_OK;
}

/* binary32 -> bfloat16 bits, round to nearest, ties to even.  NaN stays a
 * quiet NaN.  This is the definition of the rounding, done on the bits. */
static uint16_t f32_to_bf16_rne(float x)
{
    uint32_t u;
    memcpy(&u, &x, sizeof u);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))
        return (uint16_t)((u >> 16) | 0x0040u);
    {
        uint32_t lsb = (u >> 16) & 1u;
        u = u + 0x7fffu + lsb;
    }
    return (uint16_t)(u >> 16);
}

static float bf16_to_f32(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float x;
    memcpy(&x, &u, sizeof x);
    return x;
}

/* Split each binary32 value into `terms` bfloat16 values:
 *   p0 = bf16(x), p1 = bf16(x - p0), p2 = bf16(x - p0 - p1), ...
 * with every residual formed in binary32 (the residuals are exact).
 * planes[t * count + e] holds term t of element e. */
int oracle_split_bf16(const float *x, int64_t count, int terms, uint16_t *planes)
{
    int64_t e;
    if (count < 0 || terms < 1 || terms > 3) return ORACLE_BAD_ARG;
    if (count > 0 && (!x || !planes)) return ORACLE_BAD_ARG;
    for (e = 0; e < count; ++e) {
        float r = x[e];
        int t;
        for (t = 0; t < terms; ++t) {
            uint16_t h = f32_to_bf16_rne(r);
            planes[(int64_t)t * count + e] = h;
            r = r - bf16_to_f32(h);
        }
    }
    return ORACLE_OK;
}

/* Power-of-two exponent per column of a row-major k x n binary32 matrix:
 * e[j] is the integer with 1 <= max_i |B[i][j]| * 2^-e[j] < 2, or 0 for a
 * column that is all zero or holds a non-finite value. */
int oracle_column_scale_exp(const float *B, int64_t k, int64_t n, int32_t *e)
{
    int64_t i, j;
    if (k < 0 || n < 0) return ORACLE_BAD_ARG;
    if (n > 0 && !e) return ORACLE_BAD_ARG;
    if (k > 0 && n > 0 && !B) return ORACLE_BAD_ARG;
    for (j = 0; j < n; ++j) {
        float mx = 0.0f;
        int finite = 1;
        for (i = 0; i < k; ++i) {
            float a = fabsf(B[i * n + j]);
            if (!isfinite(a)) finite = 0;
            else if (a > mx) mx = a;
        }
        if (!finite || mx == 0.0f) {
            e[j] = 0;
        } else {
            int ex;
            (void)frexpf(mx, &ex);  /* mx = f * 2^ex, 0.5 <= f < 1 */
            e[j] = ex - 1;
        }
    }
    return ORACLE_OK;
}
