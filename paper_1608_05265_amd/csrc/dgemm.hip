// Double-precision GEMM (the paper's dgemm variants, Section IV-B).
//
//   * FP64: v_mfma_f64_16x16x4_f64 on FP64 matrix cores, FP64 accumulation,
//     the same blocked scheme as the FP32 tiles (K blocks staged into LDS in
//     one canonical layout, double-buffered, alpha/beta fused into the
//     store).
//   * FP32 compute ("false dgemm"): op(A), op(B) rounded to FP32, the product
//     on the FP32 path with FP32 accumulation, alpha and beta applied in FP64
//     to the widened result -- the paper's workaround of sending FP64 data
//     through the single-precision kernel, here as two conversion passes
//     around the sgemm path.
#include "dgemm.hpp"
#include "registry.hpp"

namespace misgemm {

typedef double doublex2 __attribute__((ext_vector_type(2)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// FP64 staging: LDS holds X as Xs[kk][r] (r contiguous, row length LD
// doubles).  A chunk is two consecutive elements along the stored
// contiguous direction (one 16-byte load).  Row length: R + 16 (even, for
// the 16-byte stores) when r is the stored contiguous direction; R + 17 when
// the slice is transposed on the way in, so that the 8-byte stores of 16
// lanes (eight k values times two rows) hit 16 distinct bank pairs.
// ---------------------------------------------------------------------------
template <int R, int BK, int NT, bool KC>
struct StageF64 {
    static constexpr int CH = R * BK / 2;            // 2-element chunks per tile
    static constexpr int S = (CH + NT - 1) / NT;
    static constexpr int LD = KC ? R + 17 : R + 16;
    static constexpr int ELEMS = BK * LD;
    doublex2 v[S];

    __device__ __forceinline__ static void chunk(int c, int &r, int &kk)
    {
        if (KC) { kk = (c % (BK / 2)) * 2; r = c / (BK / 2); }
        else    { r = (c % (R / 2)) * 2;   kk = c / (R / 2); }
    }

    // FAST: whole slice in range, 16-byte aligned.  Otherwise each element
    // is masked (zero outside the matrix).
    template <bool FAST>
    __device__ __forceinline__ void load(const double *X, int64_t ld, int64_t r0, int64_t k0,
                                         int64_t rows, int64_t kdim, int tid)
    {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int c = tid + s * NT;
            if (CH % NT != 0 && c >= CH) break;
            int r, kk;
            chunk(c, r, kk);
            const int64_t gr = r0 + r, gk = k0 + kk;
            if (FAST) {
                v[s] = *reinterpret_cast<const doublex2 *>(KC ? X + gk + gr * ld
                                                              : X + gr + gk * ld);
            } else if (KC) {
                const bool in = gr < rows;
                v[s][0] = in && gk < kdim ? X[gk + gr * ld] : 0.0;
                v[s][1] = in && gk + 1 < kdim ? X[gk + 1 + gr * ld] : 0.0;
            } else {
                const bool in = gk < kdim;
                v[s][0] = in && gr < rows ? X[gr + gk * ld] : 0.0;
                v[s][1] = in && gr + 1 < rows ? X[gr + 1 + gk * ld] : 0.0;
            }
        }
    }

    __device__ __forceinline__ void store(double *Xs, int tid) const
    {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int c = tid + s * NT;
            if (CH % NT != 0 && c >= CH) break;
            int r, kk;
            chunk(c, r, kk);
            if (KC) {
                Xs[kk * LD + r] = v[s][0];
                Xs[(kk + 1) * LD + r] = v[s][1];
            } else {
                *reinterpret_cast<doublex2 *>(Xs + kk * LD + r) = v[s];
            }
        }
    }
};

struct DArgs {
    int64_t m, n, k;
    const double *A;
    const double *B;
    double *C;
    int64_t lda, ldb, ldc;
    double alpha, beta;
    int vec_a, vec_b;  // 16-byte loads legal (aligned base, even ld)
};

// ---------------------------------------------------------------------------
// FP64 tile: BM x BN per workgroup, waves of WM x WN made of 16x16 MFMA
// blocks.  Operand layout of v_mfma_f64_16x16x4_f64 for lane l: A element
// (row l%16, k l/16), B element (k l/16, column l%16); result element e of
// lane l is row l/16 + 4e of column l%16 (measured on the device with
// one-hot operands: unlike the FP32 16x16 layout, a lane's four rows are
// spaced by four).
// ---------------------------------------------------------------------------
template <class SH, bool TA, bool TB>
struct F64Tile {
    static constexpr int RM = SH::WM / 16, RN = SH::WN / 16;
    static_assert(SH::WM % 16 == 0 && SH::WN % 16 == 0 && SH::BK % 4 == 0, "16x16x4 blocks");
    using SA = StageF64<SH::BM, SH::BK, SH::NT, TA>;   // A is K-contiguous when transposed
    using SB = StageF64<SH::BN, SH::BK, SH::NT, !TB>;  // B is K-contiguous when not transposed
    static constexpr int STAGE = SA::ELEMS + SB::ELEMS;
    static constexpr int LDS_BYTES = 2 * STAGE * 8;

    __device__ __forceinline__ static void epilogue(const DArgs &g, const doublex4 (&acc)[RM][RN],
                                                    int64_t row0, int64_t col0, int lane)
    {
        const int q = lane >> 4, c16 = lane & 15;
        const bool use_c0 = g.beta != 0.0;
#pragma unroll
        for (int j = 0; j < RN; ++j) {
            const int64_t col = col0 + j * 16 + c16;
            if (col >= g.n) continue;
            double *cc = g.C + col * g.ldc;
#pragma unroll
            for (int i = 0; i < RM; ++i) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    // lanes q = 0..3 of a column hold rows 4e + q: each store
                    // instruction writes 32 contiguous bytes per column
                    const int64_t row = row0 + i * 16 + 4 * e + q;
                    if (row < g.m) {
                        double o = g.alpha * acc[i][j][e];
                        if (use_c0) o += g.beta * cc[row];
                        cc[row] = o;
                    }
                }
            }
        }
    }

    __device__ __forceinline__ static void run(const DArgs &g, int64_t m0, int64_t n0, char *smem)
    {
        const bool fast = m0 + SH::BM <= g.m && n0 + SH::BN <= g.n && g.k % SH::BK == 0 &&
                          g.vec_a && g.vec_b;
        if (fast) run_impl<true>(g, m0, n0, smem);
        else run_impl<false>(g, m0, n0, smem);
    }

    template <bool FAST>
    __device__ __forceinline__ static void run_impl(const DArgs &g, int64_t m0, int64_t n0,
                                                    char *smem)
    {
        double *lds = reinterpret_cast<double *>(smem);
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
        const int wm = wave % SH::NWM, wn = wave / SH::NWM;
        const int kq = lane >> 4, r16 = lane & 15;

        doublex4 acc[RM][RN];
#pragma unroll
        for (int i = 0; i < RM; ++i)
#pragma unroll
            for (int j = 0; j < RN; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};

        const int64_t ktiles = (g.k + SH::BK - 1) / SH::BK;
        SA sa;
        SB sb;
        if (ktiles > 0) {
            sa.template load<FAST>(g.A, g.lda, m0, 0, g.m, g.k, tid);
            sb.template load<FAST>(g.B, g.ldb, n0, 0, g.n, g.k, tid);
            sa.store(lds, tid);
            sb.store(lds + SA::ELEMS, tid);
        }
        __syncthreads();
        for (int64_t kt = 0; kt < ktiles; ++kt) {
            const double *cur = lds + (kt & 1) * STAGE;
            double *nxt = lds + ((kt + 1) & 1) * STAGE;
            const bool more = kt + 1 < ktiles;
            if (more) {
                const int64_t k0 = (kt + 1) * SH::BK;
                sa.template load<FAST>(g.A, g.lda, m0, k0, g.m, g.k, tid);
                sb.template load<FAST>(g.B, g.ldb, n0, k0, g.n, g.k, tid);
            }
            const double *As = cur + wm * SH::WM + r16;
            const double *Bs = cur + SA::ELEMS + wn * SH::WN + r16;
#pragma unroll
            for (int ks = 0; ks < SH::BK / 4; ++ks) {
                const int kr = ks * 4 + kq;
                double a[RM], b[RN];
#pragma unroll
                for (int i = 0; i < RM; ++i) a[i] = As[kr * SA::LD + i * 16];
#pragma unroll
                for (int j = 0; j < RN; ++j) b[j] = Bs[kr * SB::LD + j * 16];
#pragma unroll
                for (int i = 0; i < RM; ++i)
#pragma unroll
                    for (int j = 0; j < RN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j],
                                                                          0, 0, 0);
            }
            if (more) {
                sa.store(nxt, tid);
                sb.store(nxt + SA::ELEMS, tid);
            }
            __syncthreads();
        }
        epilogue(g, acc, m0 + wm * SH::WM, n0 + wn * SH::WN, lane);
    }
};

template <class TILE, class SH>
__global__ __launch_bounds__(SH::NT, SH::OCC) void dgemm_kernel(DArgs g, int64_t tiles_m,
                                                                int64_t tiles_n, int group_m)
{
    __shared__ __attribute__((aligned(16))) char smem[TILE::LDS_BYTES];
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    int64_t tm, tn;
    tile_coords(t, tiles_m, tiles_n, group_m, tm, tn);
    TILE::run(g, tm * SH::BM, tn * SH::BN, smem);
}

template <class SH>
hipError_t launch_dgemm_shape(int ta, int tb, const DArgs &g, hipStream_t s)
{
    const int64_t tm = (g.m + SH::BM - 1) / SH::BM, tn = (g.n + SH::BN - 1) / SH::BN;
    const dim3 grid((unsigned)(tm * tn)), block(SH::NT);
    const int gm = GROUP_M_DEFAULT;
    if (!ta && !tb) hipLaunchKernelGGL((dgemm_kernel<F64Tile<SH, false, false>, SH>), grid, block, 0, s, g, tm, tn, gm);
    else if (!ta && tb) hipLaunchKernelGGL((dgemm_kernel<F64Tile<SH, false, true>, SH>), grid, block, 0, s, g, tm, tn, gm);
    else if (ta && !tb) hipLaunchKernelGGL((dgemm_kernel<F64Tile<SH, true, false>, SH>), grid, block, 0, s, g, tm, tn, gm);
    else hipLaunchKernelGGL((dgemm_kernel<F64Tile<SH, true, true>, SH>), grid, block, 0, s, g, tm, tn, gm);
    return hipGetLastError();
}

using DShapeL = Shape<128, 128, 16, 64, 64, 2>;
using DShapeS = Shape<64, 64, 16, 32, 32, 2>;

// Tile choice: 128x128 when that still gives every CU a tile, else 64x64.
hipError_t launch_dgemm_fp64(int ta, int tb, int64_t m, int64_t n, int64_t k, double alpha,
                             const double *A, int64_t lda, const double *B, int64_t ldb,
                             double beta, double *C, int64_t ldc, int cus, hipStream_t s)
{
    DArgs g;
    g.m = m; g.n = n; g.k = k;
    g.A = A; g.B = B; g.C = C;
    g.lda = lda; g.ldb = ldb; g.ldc = ldc;
    g.alpha = alpha; g.beta = beta;
    g.vec_a = ((uintptr_t)A & 15u) == 0 && lda % 2 == 0;
    g.vec_b = ((uintptr_t)B & 15u) == 0 && ldb % 2 == 0;
    const int64_t big = ((m + 127) / 128) * ((n + 127) / 128);
    if (big >= cus) return launch_dgemm_shape<DShapeL>(ta, tb, g, s);
    return launch_dgemm_shape<DShapeS>(ta, tb, g, s);
}

// ---------------------------------------------------------------------------
// FP32-compute path helpers.
// ---------------------------------------------------------------------------
// y[i] = (float)x[i], round to nearest even, for i < count.
__global__ __launch_bounds__(256) void narrow_kernel(const double *__restrict__ x, int64_t count,
                                                    float *__restrict__ y)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * 256)
        y[i] = (float)x[i];
}

hipError_t launch_narrow(const double *x, int64_t count, float *y, hipStream_t s)
{
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(narrow_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, count, y);
    return hipGetLastError();
}

// C[i + j*ldc] = alpha * P[i + j*m] + beta * C[i + j*ldc] in FP64 (C not
// read when beta == 0).
__global__ __launch_bounds__(256) void widen_kernel(const float *__restrict__ P, int64_t m,
                                                   int64_t n, double alpha, double beta,
                                                   double *__restrict__ C, int64_t ldc)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y) {
        double v = alpha * (double)P[i + j * m];
        if (beta != 0.0) v += beta * C[i + j * ldc];
        C[i + j * ldc] = v;
    }
}

hipError_t launch_widen(const float *P, int64_t m, int64_t n, double alpha, double beta,
                        double *C, int64_t ldc, hipStream_t s)
{
    const int64_t gx = (m + 255) / 256;
    const int64_t gy = n < 65535 ? n : 65535;
    hipLaunchKernelGGL(widen_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, s, P, m, n,
                       alpha, beta, C, ldc);
    return hipGetLastError();
}

// C = beta * C for FP64 (alpha == 0 or k == 0; beta == 0 writes zeros).
__global__ __launch_bounds__(256) void dscale_kernel(double beta, double *__restrict__ C,
                                                    int64_t m, int64_t n, int64_t ldc)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y) {
        double *p = C + i + j * ldc;
        *p = beta == 0.0 ? 0.0 : beta * *p;
    }
}

hipError_t launch_dscale(double beta, double *C, int64_t m, int64_t n, int64_t ldc,
                         hipStream_t s)
{
    const int64_t gx = (m + 255) / 256;
    const int64_t gy = n < 65535 ? n : 65535;
    hipLaunchKernelGGL(dscale_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, s, beta, C,
                       m, n, ldc);
    return hipGetLastError();
}

}  // namespace misgemm
