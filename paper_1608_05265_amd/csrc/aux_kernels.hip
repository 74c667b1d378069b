// Small kernels beside the GEMM tiles: the beta-only update (alpha == 0 or
// K == 0) and the stand-alone bf16x3 split.
#include "registry.hpp"

namespace misgemm {

// C = beta * C over the m x n block (beta == 0 writes zeros without reading
// C, so NaN there is cleared as the reference BLAS does).  One thread per
// element, x over rows (contiguous), y over columns.
__global__ __launch_bounds__(256) void scale_kernel(float beta, float *__restrict__ C, int64_t m,
                                                   int64_t n, int64_t ldc)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y) {
        if (i < m) {
            float *p = C + i + j * ldc;
            *p = beta == 0.0f ? 0.0f : beta * *p;
        }
    }
}

hipError_t launch_scale(float beta, float *C, int64_t m, int64_t n, int64_t ldc, hipStream_t s)
{
    const int64_t gx = (m + 255) / 256;
    const int64_t gy = n < 65535 ? n : 65535;
    hipLaunchKernelGGL(scale_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, s, beta, C,
                       m, n, ldc);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void split_kernel(const float *__restrict__ x, int64_t count,
                                                   uint16_t *__restrict__ parts)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * 256) {
        __bf16 h0, h1, h2;
        split3(x[i], h0, h1, h2);
        parts[3 * i + 0] = __builtin_bit_cast(uint16_t, h0);
        parts[3 * i + 1] = __builtin_bit_cast(uint16_t, h1);
        parts[3 * i + 2] = __builtin_bit_cast(uint16_t, h2);
    }
}

hipError_t launch_split(const float *x, int64_t count, uint16_t *parts, hipStream_t s)
{
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(split_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, count, parts);
    return hipGetLastError();
}

}  // namespace misgemm
