// Measurement helper, not part of the sgemm library: the sustained rate of
// the matrix cores on this device, for the rooflines.  Every wave keeps four
// independent accumulators busy with back-to-back MFMAs on operands read
// once from `ops` (so the operand values -- random or zero -- set the
// switching activity and with it the power draw), two workgroups of four
// waves per CU (two waves per SIMD).  Built into its own library.
#include <hip/hip_runtime.h>

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// ops: 4096 floats (fp32 probe), 512 bf16x8 (bf16 probe) or 4096 doubles
// (fp64 probe); out: one float per thread of the grid; iters a multiple of 4.
__global__ __launch_bounds__(256) void probe_bf16(const bf16x8 *ops, float *out, int iters)
{
    bf16x8 a[4], b[4];
    for (int s = 0; s < 4; ++s) {
        a[s] = ops[(threadIdx.x + 64 * s) % 512];
        b[s] = ops[(threadIdx.x * 7 + 131 * s) % 512];
    }
    floatx16 acc[4] = {};
    for (int i = 0; i < iters; i += 4) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[j], b[(j + r) & 3], acc[j], 0, 0, 0);
    }
    float s = 0.0f;
    for (int j = 0; j < 4; ++j)
        for (int e = 0; e < 16; ++e) s += acc[j][e];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void probe_f32(const float *ops, float *out, int iters)
{
    float a[4], b[4];
    for (int s = 0; s < 4; ++s) {
        a[s] = ops[(threadIdx.x + 64 * s) % 4096];
        b[s] = ops[(threadIdx.x * 7 + 131 * s) % 4096];
    }
    floatx16 acc[4] = {};
    for (int i = 0; i < iters; i += 4) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[j], b[(j + r) & 3], acc[j], 0, 0, 0);
    }
    float s = 0.0f;
    for (int j = 0; j < 4; ++j)
        for (int e = 0; e < 16; ++e) s += acc[j][e];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void probe_f64(const double *ops, float *out, int iters)
{
    double a[4], b[4];
    for (int s = 0; s < 4; ++s) {
        a[s] = ops[(threadIdx.x + 64 * s) % 4096];
        b[s] = ops[(threadIdx.x * 7 + 131 * s) % 4096];
    }
    doublex4 acc[4] = {};
    for (int i = 0; i < iters; i += 4) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j], b[(j + r) & 3], acc[j], 0, 0, 0);
    }
    double s = 0.0;
    for (int j = 0; j < 4; ++j)
        for (int e = 0; e < 4; ++e) s += acc[j][e];
    out[blockIdx.x * 256 + threadIdx.x] = (float)s;
}

// Numerical behaviour of one accumulate: test case t runs exactly one MFMA in
// one wavefront on operand registers the host laid out per lane (a, b: 64
// lane vectors per case; c: the 16 (bf16, fp32 32x32) accumulator values of
// each lane), and stores the 16 results of each lane.  The host compares
// them with models of the accumulation (one rounding of the exact sum,
// rounding after every product, ...).
__global__ __launch_bounds__(64) void probe_round_bf16(const bf16x8 *a, const bf16x8 *b,
                                                       const float *c, float *out)
{
    const int64_t t = blockIdx.x, l = threadIdx.x;
    floatx16 acc;
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] = c[(t * 64 + l) * 16 + e];
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[t * 64 + l], b[t * 64 + l], acc, 0, 0, 0);
#pragma unroll
    for (int e = 0; e < 16; ++e) out[(t * 64 + l) * 16 + e] = acc[e];
}

__global__ __launch_bounds__(64) void probe_round_f32(const float *a, const float *b,
                                                      const float *c, float *out)
{
    const int64_t t = blockIdx.x, l = threadIdx.x;
    floatx16 acc;
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] = c[(t * 64 + l) * 16 + e];
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[t * 64 + l], b[t * 64 + l], acc, 0, 0, 0);
#pragma unroll
    for (int e = 0; e < 16; ++e) out[(t * 64 + l) * 16 + e] = acc[e];
}

extern "C" {

// kind 0: FP32 MFMA (32x32x2, 4096 flop each), 1: BF16 MFMA (32x32x16,
// 32768 flop each), 2: FP64 MFMA (16x16x4, 2048 flop each).  Flops of one
// launch: blocks * 4 waves * iters * 4 * flop per MFMA.  Returns a
// hipError_t.
int probe_mfma_launch(int kind, const void *ops, float *out, int iters, int blocks, void *stream)
{
    if (iters <= 0 || iters % 4 != 0 || blocks <= 0 || kind < 0 || kind > 2)
        return (int)hipErrorInvalidValue;
    if (kind == 0)
        hipLaunchKernelGGL(probe_f32, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                           (const float *)ops, out, iters);
    else if (kind == 1)
        hipLaunchKernelGGL(probe_bf16, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                           (const bf16x8 *)ops, out, iters);
    else
        hipLaunchKernelGGL(probe_f64, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                           (const double *)ops, out, iters);
    return (int)hipGetLastError();
}

// One MFMA per case, `cases` cases: kind 0 = v_mfma_f32_32x32x2_f32 (a, b:
// cases * 64 floats), kind 1 = v_mfma_f32_32x32x16_bf16 (a, b: cases * 64
// vectors of 8 bf16); c and out: cases * 64 * 16 floats (lane-major).  Every
// index stays below these sizes.  Returns a hipError_t.
int probe_mfma_round(int kind, const void *a, const void *b, const float *c, float *out,
                     int cases, void *stream)
{
    if (cases <= 0 || kind < 0 || kind > 1) return (int)hipErrorInvalidValue;
    if (kind == 0)
        hipLaunchKernelGGL(probe_round_f32, dim3(cases), dim3(64), 0, (hipStream_t)stream,
                           (const float *)a, (const float *)b, c, out);
    else
        hipLaunchKernelGGL(probe_round_bf16, dim3(cases), dim3(64), 0, (hipStream_t)stream,
                           (const bf16x8 *)a, (const bf16x8 *)b, c, out);
    return (int)hipGetLastError();
}

}  // extern "C"
