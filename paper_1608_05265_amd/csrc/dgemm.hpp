// Host launchers of the double-precision GEMM (dgemm.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace misgemm {

// FP64 matrix-core GEMM over the whole problem (tile shape by size).
hipError_t launch_dgemm_fp64(int ta, int tb, int64_t m, int64_t n, int64_t k, double alpha,
                             const double *A, int64_t lda, const double *B, int64_t ldb,
                             double beta, double *C, int64_t ldc, int cus, hipStream_t s);
// y[i] = (float)x[i] for i < count.
hipError_t launch_narrow(const double *x, int64_t count, float *y, hipStream_t s);
// C = alpha * P + beta * C in FP64, P an m x n FP32 array with leading dimension m.
hipError_t launch_widen(const float *P, int64_t m, int64_t n, double alpha, double beta,
                        double *C, int64_t ldc, hipStream_t s);
// C = beta * C in FP64 (zeros when beta == 0).
hipError_t launch_dscale(double beta, double *C, int64_t m, int64_t n, int64_t ldc,
                         hipStream_t s);

}  // namespace misgemm
