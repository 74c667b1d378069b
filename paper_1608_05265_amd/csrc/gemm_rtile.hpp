// Register tiles for latency-bound problems (the 256^3 single call: fewer
// tiles than compute units at any staged tile size).
//
// A workgroup of KW waves computes a BM x BN tile of 16x16 matrix-core
// blocks.  K is cut into chunks of 4 KPL k (KPL = 16 or 8: 64 or 32 k);
// wave w takes chunks w, w + KW, ... and
// loads each straight from global memory into registers, with no LDS
// staging and no barrier inside the K loop (the paper's packing step pays
// off when a panel is reused many times; here every operand element is used
// by one tile only, so the copy into LDS would be pure latency).  The next
// chunk's loads are issued before the current chunk's matrix-core work.  At
// the end the waves' accumulators are added in wave order through LDS and
// wave 0 applies alpha/beta (the post-processing of Section III-C) and
// stores.
//
// Lane layout of the 16x16 blocks: lane l owns row l % 16 of the op(A)
// block and column l % 16 of the op(B) block; lane group g = l / 16 holds
// the KPL consecutive k  c0 + KPL g .. c0 + KPL g + KPL - 1  of chunk c0,
// so an operand stored k-contiguous is read with KPL/4 16-byte loads per
// lane.
//   FP32:   v_mfma_f32_16x16x4_f32 step s (0..KPL-1) takes k = c0 + KPL g + s
//           from lane group g.
//   BF16X3: v_mfma_f32_16x16x32_bf16 step t (0 .. KPL/8 - 1) takes the eight
//           k = c0 + KPL g + 8t .. +7 from lane group g; each FP32 element is
//           split into three bf16 parts in registers and the six part
//           products of a step are added smallest first into the one FP32
//           accumulator, as in the staged split-form tiles.
// The accumulator of a block gives lane l rows 4*(l/16) .. 4*(l/16)+3 of
// column l % 16.
#pragma once

#include "gemm_tile.hpp"

namespace misgemm {

// KPL: consecutive k per lane of a chunk (16, or 8 for chunks of 32 k).
template <int BM_, int BN_, int KW_, int KPL_ = 16>
struct RShape {
    static constexpr int KPL = KPL_;
    static_assert(KPL == 16 || KPL == 8, "16 or 8 k per lane");
    static constexpr int BM = BM_, BN = BN_, BK = 4 * KPL, KW = KW_, OCC = 1;
    static constexpr int WM = BM, WN = BN, NWM = 1, NWN = 1, NW = KW, NT = 64 * KW;
    static constexpr int RM = BM / 16, RN = BN / 16;  // 16x16 blocks
    static_assert(BM % 16 == 0 && BN % 16 == 0, "the tile is made of 16x16 blocks");
};

// The N values  op(X)(row, k0 + s), s = 0..N-1 (N = 16 or 8), of one row
// of op(X) (rows x kdim).  KC: op(X)(r, k) = X[k + r*ld] (k contiguous),
// else X[r + k*ld].  FAST: row < rows and k0 + N <= kdim hold, and for KC
// the 16-byte loads are aligned (base 16-byte aligned, ld % 4 == 0; k0 is
// a multiple of N).  Otherwise entries outside op(X) read as zero and are
// not loaded.
template <bool FAST, bool KC, int N>
__device__ __forceinline__ void rload(const float *__restrict__ X, int64_t ld, int64_t row,
                                      int64_t k0, int64_t rows, int64_t kdim, float (&v)[N])
{
    if constexpr (KC) {
        const float *p = X + row * ld + k0;
        if constexpr (FAST) {
#pragma unroll
            for (int q = 0; q < N / 4; ++q) {
                const floatx4 t = *reinterpret_cast<const floatx4 *>(p + 4 * q);
#pragma unroll
                for (int e = 0; e < 4; ++e) v[4 * q + e] = t[e];
            }
        } else {
            const bool rok = row < rows;
#pragma unroll
            for (int s = 0; s < N; ++s) v[s] = (rok && k0 + s < kdim) ? p[s] : 0.0f;
        }
    } else {
        const float *p = X + row + k0 * ld;
        if constexpr (FAST) {
#pragma unroll
            for (int s = 0; s < N; ++s) v[s] = p[s * ld];
        } else {
            const bool rok = row < rows;
#pragma unroll
            for (int s = 0; s < N; ++s) v[s] = (rok && k0 + s < kdim) ? p[s * ld] : 0.0f;
        }
    }
}

// Waves 1..KW-1 post their accumulators to LDS (lane-contiguous), wave 0
// adds them in wave order.  LDS: (KW-1) * RM*RN*4 * 64 floats.
template <int KW, int RM, int RN>
__device__ __forceinline__ void rwave_sum(floatx4 (&acc)[RM][RN], float *lds, int wave, int lane)
{
    constexpr int PER = RM * RN * 4;
    if (wave > 0) {
        float *dst = lds + (wave - 1) * PER * 64;
#pragma unroll
        for (int i = 0; i < RM; ++i)
#pragma unroll
            for (int j = 0; j < RN; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) dst[((i * RN + j) * 4 + e) * 64 + lane] = acc[i][j][e];
    }
    __syncthreads();
    if (wave == 0) {
        for (int w = 1; w < KW; ++w) {
            const float *src = lds + (w - 1) * PER * 64;
#pragma unroll
            for (int i = 0; i < RM; ++i)
#pragma unroll
                for (int j = 0; j < RN; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc[i][j][e] += src[((i * RN + j) * 4 + e) * 64 + lane];
        }
    }
}

// C = alpha * acc + beta * C0 for the 16x16 blocks of one wave (beta == 0:
// C0 is not read).
template <int RM, int RN>
__device__ __forceinline__ void repilogue(const GemmArgs &g, const floatx4 (&acc)[RM][RN],
                                          int64_t m0, int64_t n0, int lane)
{
    const int r = lane & 15, grp = lane >> 4;
    const bool use_c0 = g.beta != 0.0f;
#pragma unroll
    for (int j = 0; j < RN; ++j) {
        const int64_t col = n0 + j * 16 + r;
        if (col >= g.n) continue;
        float *cc = g.C + col * g.ldc;
#pragma unroll
        for (int i = 0; i < RM; ++i) {
            const int64_t row = m0 + i * 16 + grp * 4;
            if (row >= g.m) continue;
            float *p = cc + row;
            floatx4 out;
#pragma unroll
            for (int e = 0; e < 4; ++e) out[e] = g.alpha * acc[i][j][e];
            if (g.vec_c && row + 4 <= g.m) {
                if (use_c0) {
                    const floatx4 c0 = *reinterpret_cast<const floatx4 *>(p);
#pragma unroll
                    for (int e = 0; e < 4; ++e) out[e] += g.beta * c0[e];
                }
                *reinterpret_cast<floatx4 *>(p) = out;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (row + e < g.m) {
                        float o = out[e];
                        if (use_c0) o += g.beta * p[e];
                        p[e] = o;
                    }
                }
            }
        }
    }
}

// Shared skeleton of the two register tiles; MATH::step(a, b, acc) runs the
// matrix-core work of one chunk.
template <class SH, bool TA, bool TB, class MATH>
struct RTileBase {
    static constexpr int KW = SH::KW, RM = SH::RM, RN = SH::RN, NT = SH::NT, KPL = SH::KPL;
    static constexpr int LDS_BYTES = (KW > 1 ? (KW - 1) : 1) * RM * RN * 4 * 64 * 4;

    template <bool SPLIT = false>
    __device__ __forceinline__ static void run(const GemmArgs &g, int64_t m0, int64_t n0,
                                               char *smem)
    {
        static_assert(!SPLIT, "no split-K variant");
        // op(A) is k-contiguous when transposed, op(B) when not
        const bool fast = m0 + SH::BM <= g.m && n0 + SH::BN <= g.n && g.k % SH::BK == 0 &&
                          (!TA || g.vec_a) && (TB || g.vec_b);
        if (fast) run_impl<true>(g, m0, n0, smem);
        else run_impl<false>(g, m0, n0, smem);
    }

    template <bool FAST>
    __device__ __forceinline__ static void load(const GemmArgs &g, int64_t m0, int64_t n0,
                                                int64_t k0, int r, float (&a)[RM][KPL],
                                                float (&b)[RN][KPL])
    {
#pragma unroll
        for (int i = 0; i < RM; ++i)
            rload<FAST, TA, KPL>(g.A, g.lda, m0 + i * 16 + r, k0, g.m, g.k, a[i]);
#pragma unroll
        for (int j = 0; j < RN; ++j)
            rload<FAST, !TB, KPL>(g.B, g.ldb, n0 + j * 16 + r, k0, g.n, g.k, b[j]);
    }

    template <bool FAST>
    __device__ __forceinline__ static void run_impl(const GemmArgs &g, int64_t m0, int64_t n0,
                                                    char *smem)
    {
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
        const int r = lane & 15, grp = lane >> 4;
        floatx4 acc[RM][RN];
#pragma unroll
        for (int i = 0; i < RM; ++i)
#pragma unroll
            for (int j = 0; j < RN; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[i][j][e] = 0.0f;
        const int64_t chunks = (g.k + SH::BK - 1) / SH::BK;
        float a[RM][KPL], b[RN][KPL];
        int64_t c = wave;
        if (c < chunks) load<FAST>(g, m0, n0, c * SH::BK + KPL * grp, r, a, b);
        while (c < chunks) {
            const int64_t cn = c + KW;
            float a2[RM][KPL], b2[RN][KPL];
            if (cn < chunks) load<FAST>(g, m0, n0, cn * SH::BK + KPL * grp, r, a2, b2);
            MATH::template step<RM, RN, KPL>(a, b, acc);
            if (cn < chunks) {
#pragma unroll
                for (int i = 0; i < RM; ++i)
#pragma unroll
                    for (int s = 0; s < KPL; ++s) a[i][s] = a2[i][s];
#pragma unroll
                for (int j = 0; j < RN; ++j)
#pragma unroll
                    for (int s = 0; s < KPL; ++s) b[j][s] = b2[j][s];
            }
            c = cn;
        }
        rwave_sum<KW, RM, RN>(acc, reinterpret_cast<float *>(smem), wave, lane);
        if (wave == 0) repilogue<RM, RN>(g, acc, m0, n0, lane);
    }
};

struct RMathF32 {
    template <int RM, int RN, int KPL>
    __device__ __forceinline__ static void step(const float (&a)[RM][KPL],
                                                const float (&b)[RN][KPL], floatx4 (&acc)[RM][RN])
    {
#pragma unroll
        for (int s = 0; s < KPL; ++s)
#pragma unroll
            for (int i = 0; i < RM; ++i)
#pragma unroll
                for (int j = 0; j < RN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][s], b[j][s], acc[i][j],
                                                                     0, 0, 0);
    }
};

struct RMathX3 {
    template <int RM, int RN, int KPL>
    __device__ __forceinline__ static void step(const float (&a)[RM][KPL],
                                                const float (&b)[RN][KPL], floatx4 (&acc)[RM][RN])
    {
#pragma unroll
        for (int t = 0; t < KPL / 8; ++t) {
            bf16x8 ap[RM][3], bp[RN][3];
#pragma unroll
            for (int i = 0; i < RM; ++i)
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    __bf16 h0, h1, h2;
                    split3(a[i][8 * t + e], h0, h1, h2);
                    ap[i][0][e] = h0;
                    ap[i][1][e] = h1;
                    ap[i][2][e] = h2;
                }
#pragma unroll
            for (int j = 0; j < RN; ++j)
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    __bf16 h0, h1, h2;
                    split3(b[j][8 * t + e], h0, h1, h2);
                    bp[j][0][e] = h0;
                    bp[j][1][e] = h1;
                    bp[j][2][e] = h2;
                }
#pragma unroll
            for (int i = 0; i < RM; ++i)
#pragma unroll
                for (int j = 0; j < RN; ++j) {
                    floatx4 &c = acc[i][j];
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[i][0], bp[j][2], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[i][1], bp[j][1], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[i][2], bp[j][0], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[i][0], bp[j][1], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[i][1], bp[j][0], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[i][0], bp[j][0], c, 0, 0, 0);
                }
        }
    }
};

template <class SH, bool TA, bool TB>
using F32RTile = RTileBase<SH, TA, TB, RMathF32>;
template <class SH, bool TA, bool TB>
using X3RTile = RTileBase<SH, TA, TB, RMathX3>;

}  // namespace misgemm
