/*
 * Reference ("oracle") implementation of the single-precision GEMM problem.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow, obviously correct
 * CPU definition that the GPU library is checked against. It shares no code,
 * header or constant with the GPU library, and the GPU library never calls it.
 *
 * Problem (Section III-A, the statement of what the generated sgemm solves):
 *     C_out = alpha * op(A) * op(B) + beta * C_in
 * with op(X) = X or X^T, column-major storage with leading dimensions, and
 * arbitrary M, N, K.  Section III-C restates it for the inner micro-kernel
 * with the same alpha/beta post-processing after the K-sum.
 *
 * Evaluation: every product of two FP32 values is exact in FP64 (24+24 <= 53
 * significand bits), the K-sum runs in FP64 in ascending p, and the alpha and
 * beta terms are applied after the sum, as the paper's host post-processing
 * does.  Beside Cref the oracle returns the error denominator
 *     den(i,j) = |alpha| * sum_p |op(A)(i,p)| |op(B)(p,j)| + |beta| |C_in(i,j)|
 * that scales the acceptance bound.
 *
 * Degenerate cases (the paper gives only the formula; these follow the
 * reference BLAS): alpha == 0 or K == 0 -> A and B are not read; beta == 0 ->
 * C_in is not read, so NaN in it does not propagate.
 *
 * The bf16x3 functions restate the split-precision form: each FP32 value is
 * written as the sum of three bfloat16 values, each the round-to-nearest-even
 * of what the previous parts left over, and the six part products whose part
 * indices sum to at most 2 are kept.
 *
 * The dgemm functions state the same problem for FP64 storage (the paper's
 * double-precision variant, Section IV-B): products of two FP64 values are
 * exact in binary128 (53+53 <= 113 significand bits), the K-sum runs in
 * binary128 in ascending p, alpha and beta are applied after the sum, and
 * the result is rounded once to FP64.
 *
 * The LU functions restate the factorization behind the paper's Linpack
 * run (Section IV-C, HPL): P A = L U with partial pivoting, by the textbook
 * right-looking elimination in FP64 (column j: pick the row of largest
 * magnitude at or below the diagonal, first one on ties; swap it up; divide
 * the column below the diagonal by the pivot; subtract the outer product
 * from the trailing matrix), and the triangular solves that use it.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no -ffast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORACLE_OK 0
#define ORACLE_BAD_ARG (-1)
#define ORACLE_NO_MEMORY (-2)

/* 'N'/'n' -> 0, 'T'/'t'/'C'/'c' -> 1 (C equals T for real data, as the
 * paper's BLIS test parameters n/c and t/h coincide for real matrices). */
static int trans_flag(char t)
{
    if (t == 'N' || t == 'n') return 0;
    if (t == 'T' || t == 't' || t == 'C' || t == 'c') return 1;
    return -1;
}

/* Element (i,p) of op(X) where X is stored column-major with leading
 * dimension ld: X[i + p*ld] when not transposed, X[p + i*ld] when transposed. */
static double op_elem(const float *X, int64_t ld, int trans, int64_t i, int64_t p)
{
    return trans ? (double)X[p + i * ld] : (double)X[i + p * ld];
}

static void set_threads(int nthreads)
{
    if (nthreads > 0) omp_set_num_threads(nthreads);
}

int oracle_max_threads(void) { return omp_get_max_threads(); }

/*
 * Full oracle.  Cref and den are m*n FP64 arrays, column-major with leading
 * dimension m (Cref[i + j*m]).  C0 may be NULL when beta == 0.
 * Returns 0, ORACLE_BAD_ARG for an unknown transpose character or negative
 * size, or ORACLE_NO_MEMORY.
 */
int oracle_sgemm_f64(char transa, char transb, int64_t m, int64_t n, int64_t k,
                     float alpha, const float *A, int64_t lda,
                     const float *B, int64_t ldb,
                     float beta, const float *C0, int64_t ldc,
                     double *Cref, double *den, int nthreads)
{
    int ta = trans_flag(transa), tb = trans_flag(transb);
    if (ta < 0 || tb < 0 || m < 0 || n < 0 || k < 0) return ORACLE_BAD_ARG;
    if (m == 0 || n == 0) return ORACLE_OK;
    set_threads(nthreads);

    const int use_ab = (alpha != 0.0f && k > 0);
    double *opA = NULL, *opB = NULL, *absA = NULL;
    if (use_ab) {
        /* op(A) as an m x k FP64 column-major copy, and its absolute value. */
        opA = (double *)malloc(sizeof(double) * (size_t)m * (size_t)k);
        absA = (double *)malloc(sizeof(double) * (size_t)m * (size_t)k);
        /* op(B) as a k x n FP64 column-major copy. */
        opB = (double *)malloc(sizeof(double) * (size_t)k * (size_t)n);
        if (!opA || !absA || !opB) {
            free(opA); free(absA); free(opB);
            return ORACLE_NO_MEMORY;
        }
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < k; ++p)
            for (int64_t i = 0; i < m; ++i) {
                double v = op_elem(A, lda, ta, i, p);
                opA[i + p * m] = v;
                absA[i + p * m] = fabs(v);
            }
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < n; ++j)
            for (int64_t p = 0; p < k; ++p)
                opB[p + j * k] = op_elem(B, ldb, tb, p, j);
    }

    const double a = (double)alpha, b = (double)beta;
#pragma omp parallel
    {
        double *s = (double *)malloc(sizeof(double) * (size_t)m);
        double *sabs = (double *)malloc(sizeof(double) * (size_t)m);
#pragma omp for schedule(dynamic, 1)
        for (int64_t j = 0; j < n; ++j) {
            for (int64_t i = 0; i < m; ++i) { s[i] = 0.0; sabs[i] = 0.0; }
            if (use_ab) {
                /* s(:,j) = sum over ascending p of op(A)(:,p) * op(B)(p,j) */
                for (int64_t p = 0; p < k; ++p) {
                    const double bpj = opB[p + j * k];
                    const double abpj = fabs(bpj);
                    const double *acol = opA + p * m;
                    const double *aabs = absA + p * m;
                    for (int64_t i = 0; i < m; ++i) {
                        s[i] += acol[i] * bpj;
                        sabs[i] += aabs[i] * abpj;
                    }
                }
            }
            for (int64_t i = 0; i < m; ++i) {
                double c = a * s[i];
                double d = fabs(a) * sabs[i];
                if (beta != 0.0f) {
                    double c0 = (double)C0[i + j * ldc];
                    c += b * c0;
                    d += fabs(b) * fabs(c0);
                }
                Cref[i + j * m] = c;
                den[i + j * m] = d;
            }
        }
        free(s);
        free(sabs);
    }
    free(opA); free(absA); free(opB);
    return ORACLE_OK;
}

/*
 * Oracle for a list of single entries (rows[e], cols[e]), e < count: the
 * same definition as oracle_sgemm_f64, one dot product per entry, so that
 * outputs of full-size problems can be checked one by one.
 */
int oracle_sgemm_f64_entries(char transa, char transb, int64_t m, int64_t n, int64_t k,
                             float alpha, const float *A, int64_t lda,
                             const float *B, int64_t ldb,
                             float beta, const float *C0, int64_t ldc,
                             int64_t count, const int64_t *rows, const int64_t *cols,
                             double *cref, double *den, int nthreads)
{
    int ta = trans_flag(transa), tb = trans_flag(transb);
    if (ta < 0 || tb < 0 || m < 0 || n < 0 || k < 0 || count < 0) return ORACLE_BAD_ARG;
    for (int64_t e = 0; e < count; ++e)
        if (rows[e] < 0 || rows[e] >= m || cols[e] < 0 || cols[e] >= n) return ORACLE_BAD_ARG;
    set_threads(nthreads);
    const int use_ab = (alpha != 0.0f && k > 0);
    const double a = (double)alpha, b = (double)beta;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t e = 0; e < count; ++e) {
        const int64_t i = rows[e], j = cols[e];
        double s = 0.0, sabs = 0.0;
        if (use_ab)
            for (int64_t p = 0; p < k; ++p) {
                double x = op_elem(A, lda, ta, i, p);
                double y = op_elem(B, ldb, tb, p, j);
                s += x * y;
                sabs += fabs(x) * fabs(y);
            }
        double c = a * s, d = fabs(a) * sabs;
        if (beta != 0.0f) {
            double c0 = (double)C0[i + j * ldc];
            c += b * c0;
            d += fabs(b) * fabs(c0);
        }
        cref[e] = c;
        den[e] = d;
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------
 * bfloat16 split (the split-precision form).
 * ------------------------------------------------------------------------ */

static uint32_t f32_bits(float x) { uint32_t u; memcpy(&u, &x, 4); return u; }
static float bits_f32(uint32_t u) { float x; memcpy(&x, &u, 4); return x; }

/*
 * Round an FP32 value to bfloat16 (8 significand bits, FP32's exponent
 * range), to nearest with ties to even.  Works on the magnitude: the 16
 * dropped bits are compared with one half of the kept unit; above half, or
 * exactly half with an odd kept part, rounds the magnitude up (a carry into
 * the exponent field is the correct result, up to infinity).  NaN stays a
 * quiet NaN.
 */
uint16_t oracle_bf16_rne(float x)
{
    uint32_t u = f32_bits(x);
    uint32_t sign = u & 0x80000000u;
    uint32_t mag = u & 0x7fffffffu;
    if (mag > 0x7f800000u) return (uint16_t)((sign | 0x7fc00000u) >> 16);
    uint32_t kept = mag >> 16;
    uint32_t dropped = mag & 0xffffu;
    if (dropped > 0x8000u || (dropped == 0x8000u && (kept & 1u))) kept += 1u;
    return (uint16_t)((sign >> 16) | kept);
}

float oracle_bf16_to_f32(uint16_t h) { return bits_f32((uint32_t)h << 16); }

/*
 * Three-way split x = x0 + x1 + x2: x0 = bf16(x), x1 = bf16(x - x0),
 * x2 = bf16(x - x0 - x1).  Each residual is formed in FP32; for finite x below
 * bf16's overflow threshold and away from the bottom of the exponent range
 * every residual is exact, so the three parts sum to x exactly.
 */
void oracle_bf16x3_split(float x, uint16_t parts[3])
{
    float r = x;
    for (int t = 0; t < 3; ++t) {
        uint16_t h = oracle_bf16_rne(r);
        parts[t] = h;
        r = r - oracle_bf16_to_f32(h);
    }
}

/* Vector form over count values (parts is count*3, part-major per value). */
void oracle_bf16x3_split_array(const float *x, int64_t count, uint16_t *parts)
{
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < count; ++e) oracle_bf16x3_split(x[e], parts + 3 * e);
}

/*
 * Digest of the split over bit patterns lo <= u < hi, for comparing another
 * implementation with this one over all 2^32 patterns without moving the
 * parts: the sum, modulo 2^64, of (p0 | p1 << 16 | p2 << 32) * (2u + 1) over
 * the patterns of the split's domain (finite, 2^-110 <= |x| < 0x1.fefp127,
 * the domain of oracle_bf16x3_sweep), p0..p2 the bf16 parts of x.
 */
uint64_t oracle_bf16x3_split_digest(uint64_t lo, uint64_t hi, int nthreads)
{
    set_threads(nthreads);
    uint64_t digest = 0;
    const float lo_mag = ldexpf(1.0f, -110);
    const float hi_mag = bits_f32(0x7f7f8000u);
#pragma omp parallel for schedule(static) reduction(+:digest)
    for (int64_t w = (int64_t)lo; w < (int64_t)hi; ++w) {
        float x = bits_f32((uint32_t)w);
        float ax = fabsf(x);
        if (!(ax >= lo_mag && ax < hi_mag)) continue;
        uint16_t p[3];
        oracle_bf16x3_split(x, p);
        const uint64_t key = (uint64_t)p[0] | ((uint64_t)p[1] << 16) | ((uint64_t)p[2] << 32);
        digest += key * (2u * (uint64_t)w + 1u);
    }
    return digest;
}

/*
 * Exhaustive property sweep over all 2^32 FP32 bit patterns (parallel).
 * For every finite x with 2^-110 <= |x| < 0x1.fefp127 (below the value that
 * rounds to bf16 infinity) it checks:
 *   (a) x0 + x1 + x2 == x exactly (summed in FP64, which is exact here);
 *   (b) every part is a bf16 value (its FP32 widening has 16 zero low bits,
 *       which holds by construction of the encoding) and finite;
 *   (c) the residuals obey the round-to-nearest bounds |x - x0| <= 2^-8 |x|
 *       and |x - x0 - x1| <= 2^-16 |x| (half a unit of an 8-bit significand,
 *       applied twice).
 * counts[0] = values checked, counts[1] = failures of (a), counts[2] =
 * failures of (c), counts[3] = non-finite parts.  max_rel[0] receives the
 * largest |x1|/|x|, max_rel[1] the largest |x2|/|x|.
 * lo and hi bound the sweep (bit patterns lo <= u < hi) so tests can split it.
 */
void oracle_bf16x3_sweep(uint64_t lo, uint64_t hi, int64_t counts[4], double max_rel[2], int nthreads)
{
    set_threads(nthreads);
    int64_t n_checked = 0, n_sum = 0, n_bound = 0, n_inf = 0;
    double m1 = 0.0, m2 = 0.0;
    const float lo_mag = ldexpf(1.0f, -110);
    const float hi_mag = bits_f32(0x7f7f8000u); /* smallest value rounding to inf */
#pragma omp parallel for schedule(static) reduction(+:n_checked,n_sum,n_bound,n_inf) reduction(max:m1,m2)
    for (int64_t w = (int64_t)lo; w < (int64_t)hi; ++w) {
        float x = bits_f32((uint32_t)w);
        float ax = fabsf(x);
        if (!(ax >= lo_mag && ax < hi_mag)) continue;
        uint16_t p[3];
        oracle_bf16x3_split(x, p);
        double x0 = oracle_bf16_to_f32(p[0]);
        double x1 = oracle_bf16_to_f32(p[1]);
        double x2 = oracle_bf16_to_f32(p[2]);
        n_checked++;
        if (!isfinite(x0) || !isfinite(x1) || !isfinite(x2)) { n_inf++; continue; }
        if (x0 + x1 + x2 != (double)x) n_sum++;
        double r1 = fabs((double)x - x0), r2 = fabs((double)x - x0 - x1);
        double dx = fabs((double)x);
        if (r1 > ldexp(dx, -8) || r2 > ldexp(dx, -16)) n_bound++;
        double q1 = fabs(x1) / dx, q2 = fabs(x2) / dx;
        if (q1 > m1) m1 = q1;
        if (q2 > m2) m2 = q2;
    }
    counts[0] = n_checked; counts[1] = n_sum; counts[2] = n_bound; counts[3] = n_inf;
    max_rel[0] = m1; max_rel[1] = m2;
}

/*
 * Oracle of the split-precision method itself: C = alpha * S + beta * C0 with
 *     S(i,j) = sum_p  sum_{s+t <= 2}  a_s(i,p) * b_t(p,j)
 * where a_0 + a_1 + a_2 is the bf16 split of op(A)(i,p) and likewise for
 * op(B).  Every part product is exact in FP64; the sum runs in FP64 over
 * ascending p.  The dropped terms (s + t >= 3) are what separates this from
 * oracle_sgemm_f64.  Cref is m*n column-major with leading dimension m.
 */
int oracle_sgemm_bf16x3_f64(char transa, char transb, int64_t m, int64_t n, int64_t k,
                            float alpha, const float *A, int64_t lda,
                            const float *B, int64_t ldb,
                            float beta, const float *C0, int64_t ldc,
                            double *Cref, int nthreads)
{
    int ta = trans_flag(transa), tb = trans_flag(transb);
    if (ta < 0 || tb < 0 || m < 0 || n < 0 || k < 0) return ORACLE_BAD_ARG;
    if (m == 0 || n == 0) return ORACLE_OK;
    set_threads(nthreads);
    const int use_ab = (alpha != 0.0f && k > 0);
    double *pa = NULL, *pb = NULL;
    if (use_ab) {
        /* parts of op(A): pa[(i + p*m)*3 + s]; parts of op(B): pb[(p + j*k)*3 + t] */
        pa = (double *)malloc(sizeof(double) * 3 * (size_t)m * (size_t)k);
        pb = (double *)malloc(sizeof(double) * 3 * (size_t)k * (size_t)n);
        if (!pa || !pb) { free(pa); free(pb); return ORACLE_NO_MEMORY; }
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < k; ++p)
            for (int64_t i = 0; i < m; ++i) {
                uint16_t h[3];
                oracle_bf16x3_split(ta ? A[p + i * lda] : A[i + p * lda], h);
                for (int s = 0; s < 3; ++s) pa[(i + p * m) * 3 + s] = oracle_bf16_to_f32(h[s]);
            }
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < n; ++j)
            for (int64_t p = 0; p < k; ++p) {
                uint16_t h[3];
                oracle_bf16x3_split(tb ? B[j + p * ldb] : B[p + j * ldb], h);
                for (int t = 0; t < 3; ++t) pb[(p + j * k) * 3 + t] = oracle_bf16_to_f32(h[t]);
            }
    }
    const double a = (double)alpha, b = (double)beta;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            if (use_ab)
                for (int64_t p = 0; p < k; ++p) {
                    const double *x = pa + (i + p * m) * 3;
                    const double *y = pb + (p + j * k) * 3;
                    for (int u = 0; u < 3; ++u)
                        for (int v = 0; u + v <= 2; ++v) s += x[u] * y[v];
                }
            double c = a * s;
            if (beta != 0.0f) c += b * (double)C0[i + j * ldc];
            Cref[i + j * m] = c;
        }
    free(pa); free(pb);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------
 * Double-precision GEMM (Section IV-B), evaluated in binary128.
 * ------------------------------------------------------------------------ */
typedef __float128 quad;

static quad quad_abs(quad x) { return x < 0 ? -x : x; }

/* Element (i,p) of op(X) for FP64 storage (same indexing as op_elem). */
static double op_elem_d(const double *X, int64_t ld, int trans, int64_t i, int64_t p)
{
    return trans ? X[p + i * ld] : X[i + p * ld];
}

/* One entry: Cref(i,j) and den(i,j), both rounded once to FP64. */
static void dgemm_entry(int ta, int tb, int64_t k, double alpha, const double *A, int64_t lda,
                        const double *B, int64_t ldb, double beta, const double *C0,
                        int64_t ldc, int use_ab, int64_t i, int64_t j, double *cref,
                        double *den)
{
    quad s = 0, sabs = 0;
    if (use_ab)
        for (int64_t p = 0; p < k; ++p) {
            const quad x = (quad)op_elem_d(A, lda, ta, i, p);
            const quad y = (quad)op_elem_d(B, ldb, tb, p, j);
            s += x * y;
            sabs += quad_abs(x) * quad_abs(y);
        }
    quad c = (quad)alpha * s;
    quad d = quad_abs((quad)alpha) * sabs;
    if (beta != 0.0) {
        const quad c0 = (quad)C0[i + j * ldc];
        c += (quad)beta * c0;
        d += quad_abs((quad)beta) * quad_abs(c0);
    }
    *cref = (double)c;
    *den = (double)d;
}

/*
 * Full dgemm oracle.  Cref and den are m*n FP64 arrays, column-major with
 * leading dimension m.  C0 may be NULL when beta == 0.  Degenerate cases as
 * for oracle_sgemm_f64.
 */
int oracle_dgemm_f128(char transa, char transb, int64_t m, int64_t n, int64_t k,
                      double alpha, const double *A, int64_t lda,
                      const double *B, int64_t ldb,
                      double beta, const double *C0, int64_t ldc,
                      double *Cref, double *den, int nthreads)
{
    int ta = trans_flag(transa), tb = trans_flag(transb);
    if (ta < 0 || tb < 0 || m < 0 || n < 0 || k < 0) return ORACLE_BAD_ARG;
    if (m == 0 || n == 0) return ORACLE_OK;
    set_threads(nthreads);
    const int use_ab = (alpha != 0.0 && k > 0);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i)
            dgemm_entry(ta, tb, k, alpha, A, lda, B, ldb, beta, C0, ldc, use_ab, i, j,
                        &Cref[i + j * m], &den[i + j * m]);
    return ORACLE_OK;
}

/* The dgemm oracle at single entries (rows[e], cols[e]). */
int oracle_dgemm_f128_entries(char transa, char transb, int64_t m, int64_t n, int64_t k,
                              double alpha, const double *A, int64_t lda,
                              const double *B, int64_t ldb,
                              double beta, const double *C0, int64_t ldc,
                              int64_t count, const int64_t *rows, const int64_t *cols,
                              double *cref, double *den, int nthreads)
{
    int ta = trans_flag(transa), tb = trans_flag(transb);
    if (ta < 0 || tb < 0 || m < 0 || n < 0 || k < 0 || count < 0) return ORACLE_BAD_ARG;
    for (int64_t e = 0; e < count; ++e)
        if (rows[e] < 0 || rows[e] >= m || cols[e] < 0 || cols[e] >= n) return ORACLE_BAD_ARG;
    set_threads(nthreads);
    const int use_ab = (alpha != 0.0 && k > 0);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t e = 0; e < count; ++e)
        dgemm_entry(ta, tb, k, alpha, A, lda, B, ldb, beta, C0, ldc, use_ab, rows[e], cols[e],
                    &cref[e], &den[e]);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------
 * LU factorization with partial pivoting (Section IV-C), FP64.
 * ------------------------------------------------------------------------ */

/*
 * A (n x n FP32, leading dimension lda) is read; LU (n x n FP64, leading
 * dimension n) receives L (unit diagonal not stored) below the diagonal and
 * U on and above it; ipiv[j] is the row swapped with row j at step j
 * (0-based).  Returns 0, or 1 + the first j whose pivot is zero (the
 * elimination then continues without dividing that column), or
 * ORACLE_BAD_ARG.
 */
int oracle_getrf_f64(int64_t n, const float *A, int64_t lda, double *LU, int64_t *ipiv,
                     int nthreads)
{
    if (n < 0 || lda < (n > 0 ? n : 1)) return ORACLE_BAD_ARG;
    set_threads(nthreads);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) LU[i + j * n] = (double)A[i + j * lda];
    int info = 0;
    for (int64_t j = 0; j < n; ++j) {
        int64_t p = j;
        double best = fabs(LU[j + j * n]);
        for (int64_t i = j + 1; i < n; ++i)
            if (fabs(LU[i + j * n]) > best) { best = fabs(LU[i + j * n]); p = i; }
        ipiv[j] = p;
        if (p != j)
            for (int64_t c = 0; c < n; ++c) {
                double t = LU[j + c * n];
                LU[j + c * n] = LU[p + c * n];
                LU[p + c * n] = t;
            }
        const double piv = LU[j + j * n];
        if (piv == 0.0) {
            if (info == 0) info = (int)(j + 1);
            continue;
        }
        for (int64_t i = j + 1; i < n; ++i) LU[i + j * n] /= piv;
#pragma omp parallel for schedule(static)
        for (int64_t c = j + 1; c < n; ++c) {
            const double u = LU[j + c * n];
            for (int64_t i = j + 1; i < n; ++i) LU[i + c * n] -= LU[i + j * n] * u;
        }
    }
    return info;
}

/*
 * Solve A x = b with the factors of oracle_getrf_f64: apply the row swaps to
 * b, then L y = b (forward, unit diagonal), then U x = y (backward).  b (n
 * FP64) is overwritten with x.
 */
int oracle_getrs_f64(int64_t n, const double *LU, const int64_t *ipiv, double *b)
{
    if (n < 0) return ORACLE_BAD_ARG;
    for (int64_t j = 0; j < n; ++j) {
        const int64_t p = ipiv[j];
        if (p < 0 || p >= n) return ORACLE_BAD_ARG;
        if (p != j) { double t = b[j]; b[j] = b[p]; b[p] = t; }
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t c = 0; c < i; ++c) b[i] -= LU[i + c * n] * b[c];
    for (int64_t i = n - 1; i >= 0; --i) {
        for (int64_t c = i + 1; c < n; ++c) b[i] -= LU[i + c * n] * b[c];
        b[i] /= LU[i + i * n];
    }
    return ORACLE_OK;
}
