// LU factorization with partial pivoting and the solve that uses it: the
// Linpack (HPL) workload of the paper's Section IV-C, on the sgemm path.
//
// Recursive right-looking LU: factor the left half of the column range,
// swap its pivots into the right half, L11^{-1} A12 (recursive triangular
// solve), A22 -= A21 A12 (one sgemm -- the rank-k trailing update), factor
// A22, swap its pivots back into the left half.  Almost all flops land in
// sgemm calls of decreasing size; the leaves are 32-column panels that one
// workgroup factors column by column.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/misgemm.h"

namespace {

constexpr int LEAF = 32;       // columns of a leaf panel / rows of a leaf solve
constexpr int LEAF_THREADS = 1024;

// Factor the m x w panel P (w <= LEAF, leading dimension lda; its top-left
// element is A(row0, row0)): for each column j, the row of largest
// magnitude at or below j (first one on ties) is swapped up across the
// panel, the column below the diagonal is divided by the pivot, and the
// outer product is subtracted from the panel's remaining columns.  A zero
// pivot leaves its column as it is and records row0 + j + 1 in *info if no
// earlier zero pivot did.  ipiv receives global row indices.
__global__ __launch_bounds__(LEAF_THREADS) void lu_leaf_kernel(float *__restrict__ P,
                                                              int64_t lda, int64_t m, int w,
                                                              int64_t *__restrict__ ipiv,
                                                              int64_t row0, int *__restrict__ info)
{
    __shared__ float sbest[LEAF_THREADS];
    __shared__ int64_t sidx[LEAF_THREADS];
    __shared__ float urow[LEAF];
    const int t = threadIdx.x;
    for (int j = 0; j < w; ++j) {
        float *col = P + (int64_t)j * lda;
        float best = -1.0f;
        int64_t idx = -1;
        for (int64_t r = j + t; r < m; r += LEAF_THREADS) {
            const float v = fabsf(col[r]);
            if (v > best) { best = v; idx = r; }
        }
        sbest[t] = best;
        sidx[t] = idx;
        __syncthreads();
        for (int s = LEAF_THREADS / 2; s > 0; s >>= 1) {
            if (t < s) {
                const float b1 = sbest[t + s];
                const int64_t i1 = sidx[t + s];
                if (i1 >= 0 && (sidx[t] < 0 || b1 > sbest[t] || (b1 == sbest[t] && i1 < sidx[t]))) {
                    sbest[t] = b1;
                    sidx[t] = i1;
                }
            }
            __syncthreads();
        }
        const int64_t p = sidx[0] >= 0 ? sidx[0] : j;
        const float pivot_mag = sbest[0];
        __syncthreads();
        if (t == 0) ipiv[row0 + j] = row0 + p;
        if (p != j && t < w) {
            float *c = P + (int64_t)t * lda;
            const float x = c[j];
            c[j] = c[p];
            c[p] = x;
        }
        __syncthreads();
        const float piv = col[j];
        if (pivot_mag > 0.0f && piv != 0.0f) {
            for (int64_t r = j + 1 + t; r < m; r += LEAF_THREADS) col[r] = col[r] / piv;
            if (t > j && t < w) urow[t] = P[j + (int64_t)t * lda];
            __syncthreads();
            for (int64_t r = j + 1 + t; r < m; r += LEAF_THREADS) {
                const float l = col[r];
                for (int c = j + 1; c < w; ++c) P[r + (int64_t)c * lda] -= l * urow[c];
            }
        } else if (t == 0 && *info == 0) {
            *info = (int)(row0 + j + 1);
        }
        __syncthreads();
    }
}

// Row interchanges k0..k1-1 (ipiv global rows, applied in order) on ncols
// columns starting at C (row 0 of the matrix); one thread per column.
__global__ __launch_bounds__(256) void laswp_kernel(float *__restrict__ C, int64_t ldc,
                                                   int64_t ncols, const int64_t *__restrict__ ipiv,
                                                   int64_t k0, int64_t k1)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= ncols) return;
    float *col = C + c * ldc;
    for (int64_t k = k0; k < k1; ++k) {
        const int64_t p = ipiv[k];
        if (p != k) {
            const float x = col[k];
            col[k] = col[p];
            col[p] = x;
        }
    }
}

// B (n x ncols, n <= LEAF) := T^{-1} B for T the n x n lower unit (UPPER
// false) or upper (UPPER true) triangle at T; one thread per column of B,
// T staged in LDS.
template <bool UPPER>
__global__ __launch_bounds__(256) void trsm_leaf_kernel(const float *__restrict__ T, int64_t ldt,
                                                       float *__restrict__ B, int64_t ldb, int n,
                                                       int64_t ncols)
{
    __shared__ float sT[LEAF * LEAF];
    for (int e = threadIdx.x; e < n * n; e += 256) sT[e] = T[(e % n) + (int64_t)(e / n) * ldt];
    __syncthreads();
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= ncols) return;
    float x[LEAF];
    float *col = B + c * ldb;
#pragma unroll
    for (int i = 0; i < LEAF; ++i)
        if (i < n) x[i] = col[i];
    if (!UPPER) {
#pragma unroll
        for (int i = 0; i < LEAF; ++i)
#pragma unroll
            for (int k = 0; k < LEAF; ++k)
                if (k < i && i < n) x[i] -= sT[i + k * n] * x[k];
    } else {
#pragma unroll
        for (int ii = 0; ii < LEAF; ++ii) {
            const int i = LEAF - 1 - ii;
            if (i < n) {
#pragma unroll
                for (int k = 0; k < LEAF; ++k)
                    if (k > i && k < n) x[i] -= sT[i + k * n] * x[k];
                x[i] = x[i] / sT[i + i * n];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < LEAF; ++i)
        if (i < n) col[i] = x[i];
}

__global__ void zero_info_kernel(int *info) { *info = 0; }

struct Lu {
    float *A;
    int64_t lda, n;
    int64_t *ipiv;
    int *info;
    int mode;
    hipStream_t s;
};

int check(hipError_t e) { return e == hipSuccess ? 0 : (int)e; }

int gemm(const Lu &c, int64_t m, int64_t n, int64_t k, const float *A, int64_t lda,
         const float *B, int64_t ldb, float *C, int64_t ldc)
{
    if (m == 0 || n == 0 || k == 0) return 0;
    return misgemm_sgemm('N', 'N', m, n, k, -1.0f, A, lda, B, ldb, 1.0f, C, ldc, c.mode, c.s);
}

int laswp(const Lu &c, float *C, int64_t ldc, int64_t ncols, int64_t k0, int64_t k1)
{
    if (ncols <= 0 || k1 <= k0) return 0;
    hipLaunchKernelGGL(laswp_kernel, dim3((unsigned)((ncols + 255) / 256)), dim3(256), 0, c.s, C,
                       ldc, ncols, c.ipiv, k0, k1);
    return check(hipGetLastError());
}

// B (n x ncols) := T^{-1} B, T lower unit or upper n x n, recursively: the
// off-diagonal block goes through sgemm.
int trsm(const Lu &c, bool upper, const float *T, int64_t ldt, float *B, int64_t ldb, int64_t n,
         int64_t ncols)
{
    if (n == 0 || ncols == 0) return 0;
    if (n <= LEAF) {
        const dim3 grid((unsigned)((ncols + 255) / 256));
        if (upper)
            hipLaunchKernelGGL(trsm_leaf_kernel<true>, grid, dim3(256), 0, c.s, T, ldt, B, ldb,
                               (int)n, ncols);
        else
            hipLaunchKernelGGL(trsm_leaf_kernel<false>, grid, dim3(256), 0, c.s, T, ldt, B, ldb,
                               (int)n, ncols);
        return check(hipGetLastError());
    }
    const int64_t h = (n / 2 + LEAF - 1) / LEAF * LEAF;
    int rc;
    if (!upper) {
        if ((rc = trsm(c, false, T, ldt, B, ldb, h, ncols))) return rc;
        if ((rc = gemm(c, n - h, ncols, h, T + h, ldt, B, ldb, B + h, ldb))) return rc;
        return trsm(c, false, T + h + h * ldt, ldt, B + h, ldb, n - h, ncols);
    }
    if ((rc = trsm(c, true, T + h + h * ldt, ldt, B + h, ldb, n - h, ncols))) return rc;
    if ((rc = gemm(c, h, ncols, n - h, T + h * ldt, ldt, B + h, ldb, B, ldb))) return rc;
    return trsm(c, true, T, ldt, B, ldb, h, ncols);
}

// Factor columns j0 .. j0+w-1 over rows j0 .. n-1.
int getrf(const Lu &c, int64_t j0, int64_t w)
{
    const int64_t m = c.n - j0;
    float *P = c.A + j0 + j0 * c.lda;
    if (w <= LEAF) {
        hipLaunchKernelGGL(lu_leaf_kernel, dim3(1), dim3(LEAF_THREADS), 0, c.s, P, c.lda, m,
                           (int)w, c.ipiv, j0, c.info);
        return check(hipGetLastError());
    }
    const int64_t w1 = (w / 2 + LEAF - 1) / LEAF * LEAF, w2 = w - w1;
    int rc;
    if ((rc = getrf(c, j0, w1))) return rc;
    float *right = c.A + (j0 + w1) * c.lda;  // row 0 of the right part
    if ((rc = laswp(c, right, c.lda, w2, j0, j0 + w1))) return rc;
    if ((rc = trsm(c, false, P, c.lda, P + w1 * c.lda, c.lda, w1, w2))) return rc;
    if ((rc = gemm(c, m - w1, w2, w1, P + w1, c.lda, P + w1 * c.lda, c.lda,
                   P + w1 + w1 * c.lda, c.lda)))
        return rc;
    if ((rc = getrf(c, j0 + w1, w2))) return rc;
    return laswp(c, c.A + j0 * c.lda, c.lda, w1, j0 + w1, j0 + w);
}

bool lu_mode_ok(int mode) { return mode == MISGEMM_FP32 || mode == MISGEMM_BF16X3; }

}  // namespace

extern "C" {

int misgemm_sgetrf(int64_t n, float *A, int64_t lda, int64_t *ipiv, int *info, int mode,
                   void *stream)
{
    if (n < 0) return -1;
    if (n > 0 && A == nullptr) return -2;
    if (lda < (n > 0 ? n : 1)) return -3;
    if (n > 0 && ipiv == nullptr) return -4;
    if (info == nullptr) return -5;
    if (!lu_mode_ok(mode)) return -6;
    if (n > ((int64_t)1 << 31)) return MISGEMM_E_TOO_LARGE;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(zero_info_kernel, dim3(1), dim3(1), 0, s, info);
    int rc = check(hipGetLastError());
    if (rc != 0 || n == 0) return rc;
    const Lu c{A, lda, n, ipiv, info, mode, s};
    return getrf(c, 0, n);
}

int misgemm_sgetrs(int64_t n, int64_t nrhs, const float *A, int64_t lda, const int64_t *ipiv,
                   float *B, int64_t ldb, int mode, void *stream)
{
    if (n < 0) return -1;
    if (nrhs < 0) return -2;
    if (n > 0 && A == nullptr) return -3;
    if (lda < (n > 0 ? n : 1)) return -4;
    if (n > 0 && ipiv == nullptr) return -5;
    if (n > 0 && nrhs > 0 && B == nullptr) return -6;
    if (ldb < (n > 0 ? n : 1)) return -7;
    if (!lu_mode_ok(mode)) return -8;
    if (n == 0 || nrhs == 0) return 0;
    const Lu c{const_cast<float *>(A), lda, n, const_cast<int64_t *>(ipiv), nullptr, mode,
               (hipStream_t)stream};
    int rc = laswp(c, B, ldb, nrhs, 0, n);
    if (rc == 0) rc = trsm(c, false, A, lda, B, ldb, n, nrhs);
    if (rc == 0) rc = trsm(c, true, A, lda, B, ldb, n, nrhs);
    return rc;
}

}  // extern "C"
