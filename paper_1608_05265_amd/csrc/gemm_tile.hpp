// Device code of the sgemm path for gfx950 (CDNA4).
//
// One workgroup computes one BM x BN tile of C over the whole K range, the
// GPU form of the paper's blocked scheme (Section III-C): K is consumed in
// BK-wide blocks, each block of op(A) and op(B) is staged ("packed") from
// HBM into LDS in one canonical layout that no longer depends on the
// transposes or leading dimensions, the partial products are accumulated in
// registers for all of K (the "accumulator" variant of Section III-C), the
// next block is fetched while the current one is multiplied (the paper's
// double-buffered input transfer), and alpha/beta are applied once at the
// end (the post-processing of Section III-C), fused into the store.
//
// Two arithmetic forms share the staging/epilogue skeleton:
//   * F32:    v_mfma_f32_32x32x2_f32, FP32 in, FP32 accumulate.
//   * BF16X3: every FP32 element is split while it is staged into three
//             bf16 parts x = x0 + x1 + x2 (round to nearest even), and the six
//             part products with index sum <= 2 run on
//             v_mfma_f32_32x32x16_bf16 with FP32 accumulation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace misgemm {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// Arguments of one GEMM, as seen by a workgroup.
struct GemmArgs {
    int64_t m, n, k;
    const float *A;
    const float *B;
    float *C;
    int64_t lda, ldb, ldc;
    float alpha, beta;
    int vec_a, vec_b, vec_c;  // 16-byte vector access legal (aligned base, ld % 4 == 0)
    // Split-K (read only by the split kernels): this workgroup computes the
    // K range of split `split` of `splits` for tile `tile`; its partial sums
    // go to `part`.
    float *part;
    int64_t tile;
    int split, splits;
};

// ---------------------------------------------------------------------------
// Tile shape: BM x BN per workgroup, BK per K block, WM x WN per wave.
// ---------------------------------------------------------------------------
// OCC_: waves per SIMD the register allocation must leave room for
// (a launch bound; 8-wave tiles get two per SIMD by construction).
template <int BM_, int BN_, int BK_, int WM_, int WN_, int OCC_ = 1>
struct Shape {
    static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_, OCC = OCC_;
    static constexpr int NWM = BM / WM, NWN = BN / WN, NW = NWM * NWN, NT = 64 * NW;
    static constexpr int RM = WM / 32, RN = WN / 32;  // 32x32 MFMA blocks per wave
    static_assert(BM % WM == 0 && BN % WN == 0, "wave tiles must divide the tile");
    static_assert(WM % 32 == 0 && WN % 32 == 0, "wave tile is made of 32x32 blocks");
};

// Element (r, kk) of an op(X) tile lives at X[kk + r*ld] when the stored
// matrix is contiguous along K (KC = true: A transposed, B not transposed)
// and at X[r + kk*ld] otherwise.

__device__ __forceinline__ floatx4 load4(const float *p, bool vec, bool in_r, int64_t lim_k,
                                         int64_t step)
{
    // Four consecutive elements p[0], p[step], ... masked: element e is read
    // only when in_r and e < lim_k.  step is 1 for the contiguous direction.
    floatx4 v;
    if (vec && in_r && lim_k >= 4) {
        v = *reinterpret_cast<const floatx4 *>(p);
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (in_r && e < lim_k) ? p[e * step] : 0.0f;
    }
    return v;
}

// ---------------------------------------------------------------------------
// F32 staging: LDS holds X as Xs[kk][r] (r contiguous, row length LD).
// ---------------------------------------------------------------------------
template <int R, int BK, int NT, bool KC>
struct StageF32 {
    static constexpr int CH = R * BK / 4;            // float4 chunks per tile
    static constexpr int S = (CH + NT - 1) / NT;     // chunks per thread
    static constexpr int LD = R + (KC ? 2 : 4);      // LDS row length (floats)
    static constexpr int FLOATS = BK * LD;
    floatx4 v[S];

    __device__ __forceinline__ void chunk(int c, int &r, int &kk) const
    {
        if (KC) { kk = (c % (BK / 4)) * 4; r = c / (BK / 4); }
        else    { r = (c % (R / 4)) * 4;   kk = c / (R / 4); }
    }

    static constexpr bool NEEDS_VEC = true;  // the fast path uses 16-byte loads

    // FAST: the caller guarantees the whole R x BK slice is in range and
    // 16-byte aligned (an interior tile): unmasked loads, no branches, so the
    // wait counters see straight-line code.  Otherwise every element is
    // masked (zero fill outside the matrix).
    template <bool FAST>
    __device__ __forceinline__ void load(const float *X, int64_t ld, int64_t r0, int64_t k0,
                                         int64_t rows, int64_t kdim, bool vec, int tid)
    {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int c = tid + s * NT;
            if (CH % NT != 0 && c >= CH) break;
            int r, kk;
            chunk(c, r, kk);
            const int64_t gr = r0 + r, gk = k0 + kk;
            if (FAST) {
                v[s] = *reinterpret_cast<const floatx4 *>(KC ? X + gk + gr * ld : X + gr + gk * ld);
            } else if (KC) {
                v[s] = load4(X + gk + gr * ld, vec, gr < rows, kdim - gk, 1);
            } else {
                // four consecutive rows at one k: rows are the contiguous direction
                v[s] = load4(X + gr + gk * ld, vec, gk < kdim, rows - gr, 1);
            }
        }
    }

    __device__ __forceinline__ void store(float *Xs, int tid) const
    {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int c = tid + s * NT;
            if (CH % NT != 0 && c >= CH) break;
            int r, kk;
            chunk(c, r, kk);
            if (KC) {
#pragma unroll
                for (int e = 0; e < 4; ++e) Xs[(kk + e) * LD + r] = v[s][e];
            } else {
                *reinterpret_cast<floatx4 *>(Xs + kk * LD + r) = v[s];
            }
        }
    }
};

// ---------------------------------------------------------------------------
// BF16X3 staging: LDS holds, per part t, Xs[t][r][kk] (kk contiguous, row
// length LD bf16), so one 16-byte LDS read gives a lane the eight K values
// a 32x32x16 bf16 MFMA operand needs.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void split3(float x, __bf16 &h0, __bf16 &h1, __bf16 &h2)
{
    h0 = (__bf16)x;            // round to nearest even
    float r = x - (float)h0;   // exact
    h1 = (__bf16)r;
    r = r - (float)h1;         // exact
    h2 = (__bf16)r;
}

template <int R, int BK, int NT, bool KC>
struct StageX3 {
    // Row stride of 16*(BK/8 + 1) bytes: the 16-byte reads and writes of 32
    // consecutive rows fall in distinct LDS banks.
    static constexpr int LD = BK + 8;                  // bf16 per LDS row
    static constexpr int PART = R * LD;                // bf16 per part
    static constexpr int HALVES = 3 * PART;            // bf16 per operand tile
    // A chunk is eight consecutive k of one row; consecutive threads take
    // consecutive rows.
    static constexpr int KS = 8;
    static constexpr int CH = R * BK / KS;
    static constexpr int S = (CH + NT - 1) / NT;
    static constexpr bool UNITS_FULL = CH % NT == 0;
    static constexpr int UNITS = S;
    float v[S][KS];

    __device__ __forceinline__ static void chunk(int c, int &r, int &kk)
    {
        r = c % R;
        kk = (c / R) * KS;
    }

    static constexpr bool NEEDS_VEC = KC;  // only the K-contiguous side uses 16-byte loads

    // FAST: the caller guarantees an interior, aligned slice (unmasked loads,
    // straight-line code); otherwise every element is masked.
    template <bool FAST>
    __device__ __forceinline__ void load(const float *X, int64_t ld, int64_t r0, int64_t k0,
                                         int64_t rows, int64_t kdim, bool vec, int tid)
    {
        (void)vec;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int c = tid + s * NT;
            if (!UNITS_FULL && c >= CH) break;
            int r, kk;
            chunk(c, r, kk);
            const int64_t gr = r0 + r, gk = k0 + kk;
            if (FAST) {
                if (KC) {
                    const float *p = X + gk + gr * ld;
                    const floatx4 x0 = *reinterpret_cast<const floatx4 *>(p);
                    const floatx4 x1 = *reinterpret_cast<const floatx4 *>(p + 4);
#pragma unroll
                    for (int e = 0; e < 4; ++e) { v[s][e] = x0[e]; v[s][4 + e] = x1[e]; }
                } else {
                    const float *p = X + gr + gk * ld;
#pragma unroll
                    for (int e = 0; e < KS; ++e) v[s][e] = p[e * ld];
                }
            } else {
                const bool in_r = gr < rows;
                if (KC) {
                    const float *p = X + gk + gr * ld;
#pragma unroll
                    for (int e = 0; e < KS; ++e) v[s][e] = (in_r && gk + e < kdim) ? p[e] : 0.0f;
                } else {
                    const float *p = X + gr + gk * ld;
#pragma unroll
                    for (int e = 0; e < KS; ++e)
                        v[s][e] = (in_r && gk + e < kdim) ? p[e * ld] : 0.0f;
                }
            }
        }
    }

    __device__ __forceinline__ float unit_val(int u, int e) const { return v[u][e]; }

    __device__ __forceinline__ static int unit_offset(int u, int tid)
    {
        int r, kk;
        chunk(tid + u * NT, r, kk);
        return r * LD + kk;
    }

    // Split the eight values of unit u and write the three parts.
    __device__ __forceinline__ void store_unit(__bf16 *Xs, int u, int tid) const
    {
        bf16x8 p0, p1, p2;
#pragma unroll
        for (int e = 0; e < KS; ++e) {
            __bf16 h0, h1, h2;
            split3(v[u][e], h0, h1, h2);
            p0[e] = h0;
            p1[e] = h1;
            p2[e] = h2;
        }
        __bf16 *base = Xs + unit_offset(u, tid);
        *reinterpret_cast<bf16x8 *>(base) = p0;
        *reinterpret_cast<bf16x8 *>(base + PART) = p1;
        *reinterpret_cast<bf16x8 *>(base + 2 * PART) = p2;
    }

    __device__ __forceinline__ void store(__bf16 *Xs, int tid) const
    {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (!UNITS_FULL && tid + s * NT >= CH) break;
            store_unit(Xs, s, tid);
        }
    }
};

// ---------------------------------------------------------------------------
// Epilogue: C = alpha * acc + beta * C0 for one wave's 32x32 blocks.
// MFMA 32x32 output layout: lane l, register 4g + e holds row
// 8g + 4*(l/32) + e, column l % 32, so each lane owns four consecutive rows
// of one column (one 16-byte store in column-major C).
// ---------------------------------------------------------------------------
// beta == 0: C0 is not read.  C0 and C are one array, so as far as the
// compiler knows a store may alias any later load, and no load moves above
// an earlier store: loaded one 16-byte group at a time, every group would
// cost the wave a full memory round trip.  The C0 loads of EPI_GROUP groups
// are therefore issued together ahead of their stores (one round trip per
// EPI_GROUP groups, 4 * EPI_GROUP more VGPRs; 4 keeps the 128x128 tiles at
// three waves per SIMD, 8 does not).
constexpr int EPI_GROUP = 4;

template <int RM, int RN>
__device__ __forceinline__ void epilogue(const GemmArgs &g, const floatx16 (&acc)[RM][RN],
                                         int64_t row0, int64_t col0, int lane)
{
    const int half = lane >> 5, l32 = lane & 31;
    const bool vec = g.vec_c;
    const bool use_c0 = g.beta != 0.0f;
    constexpr int NG = RN * RM * 4;                       // 16-byte groups per lane
    constexpr int GG = EPI_GROUP < NG ? EPI_GROUP : NG;
    static_assert(NG % GG == 0, "whole load groups");
#pragma unroll
    for (int g0 = 0; g0 < NG; g0 += GG) {
        floatx4 c0[GG];
#pragma unroll
        for (int q = 0; q < GG; ++q) {
            const int idx = g0 + q, rn = idx / (RM * 4), rm = (idx / 4) % RM, gi = idx % 4;
            const int64_t col = col0 + rn * 32 + l32;
            const int64_t row = row0 + rm * 32 + gi * 8 + half * 4;
#pragma unroll
            for (int e = 0; e < 4; ++e) c0[q][e] = 0.0f;
            if (use_c0 && vec && col < g.n && row + 4 <= g.m)
                c0[q] = *reinterpret_cast<const floatx4 *>(g.C + col * g.ldc + row);
        }
#pragma unroll
        for (int q = 0; q < GG; ++q) {
            const int idx = g0 + q, rn = idx / (RM * 4), rm = (idx / 4) % RM, gi = idx % 4;
            const int64_t col = col0 + rn * 32 + l32;
            const int64_t row = row0 + rm * 32 + gi * 8 + half * 4;
            if (col >= g.n || row >= g.m) continue;
            float *p = g.C + col * g.ldc + row;
            floatx4 out;
#pragma unroll
            for (int e = 0; e < 4; ++e) out[e] = g.alpha * acc[rm][rn][gi * 4 + e];
            if (vec && row + 4 <= g.m) {
                if (use_c0) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) out[e] += g.beta * c0[q][e];
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

// ---------------------------------------------------------------------------
// End of a tile.  A whole-K tile applies alpha/beta and stores.  A split-K
// tile (SPLIT) stores its raw partial accumulator instead; a second kernel
// (splitk_reduce) adds the partials of all splits in split order and runs
// the epilogue, so the result does not depend on the order in which the
// splits ran.  Partial layout: for split s of tile t, float4 group q of
// thread x is at part[((t * splits + s) * Q + q) * NT + x] (Q = RM*RN*4
// groups per thread), so each store instruction of a wave writes 1 KB
// contiguously.
// ---------------------------------------------------------------------------
template <int RM, int RN>
__device__ __forceinline__ int64_t partial_index(int64_t tile, int splits, int split, int q,
                                                 int tid, int nt)
{
    return ((tile * splits + split) * (int64_t)(RM * RN * 4) + q) * nt + tid;
}

template <bool SPLIT, int RM, int RN>
__device__ __forceinline__ void finish(const GemmArgs &g, const floatx16 (&acc)[RM][RN],
                                       int64_t row0, int64_t col0, int tid, int nt)
{
    if constexpr (SPLIT) {
        floatx4 *const part = reinterpret_cast<floatx4 *>(g.part);
#pragma unroll
        for (int i = 0; i < RM; ++i)
#pragma unroll
            for (int j = 0; j < RN; ++j)
#pragma unroll
                for (int q4 = 0; q4 < 4; ++q4) {
                    floatx4 v;
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = acc[i][j][q4 * 4 + e];
                    part[partial_index<RM, RN>(g.tile, g.splits, g.split, (i * RN + j) * 4 + q4,
                                               tid, nt)] = v;
                }
    } else {
        epilogue<RM, RN>(g, acc, row0, col0, tid & 63);
    }
}

// ---------------------------------------------------------------------------
// The tile body: stage -> multiply -> epilogue for tile (m0, n0).
// ---------------------------------------------------------------------------
template <class SH, bool TA, bool TB, bool PF2 = false>
struct F32Tile {
    using SA = StageF32<SH::BM, SH::BK, SH::NT, TA>;   // A is K-contiguous when transposed
    using SB = StageF32<SH::BN, SH::BK, SH::NT, !TB>;  // B is K-contiguous when not transposed
    static constexpr int STAGE_FLOATS = SA::FLOATS + SB::FLOATS;
    static constexpr int LDS_BYTES = 2 * STAGE_FLOATS * 4;
    static constexpr int NT = SH::NT;

    // Interior tiles whose K range is a whole number of blocks take the
    // unmasked load path; every other tile masks its loads.
    template <bool SPLIT = false>
    __device__ __forceinline__ static void run(const GemmArgs &g, int64_t m0, int64_t n0,
                                               char *smem)
    {
        const bool fast = m0 + SH::BM <= g.m && n0 + SH::BN <= g.n && g.k % SH::BK == 0 &&
                          (g.vec_a || !SA::NEEDS_VEC) && (g.vec_b || !SB::NEEDS_VEC);
        if (fast) run_impl<true, SPLIT>(g, m0, n0, smem);
        else run_impl<false, SPLIT>(g, m0, n0, smem);
    }

    template <bool FAST, bool SPLIT>
    __device__ __forceinline__ static void run_impl(const GemmArgs &g, int64_t m0, int64_t n0,
                                                    char *smem)
    {
        float *lds = reinterpret_cast<float *>(smem);
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
        const int wm = wave % SH::NWM, wn = wave / SH::NWM;
        const int half = lane >> 5, l32 = lane & 31;

        floatx16 acc[SH::RM][SH::RN];
#pragma unroll
        for (int i = 0; i < SH::RM; ++i)
#pragma unroll
            for (int j = 0; j < SH::RN; ++j)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;

        const int64_t ktiles = (g.k + SH::BK - 1) / SH::BK;
        SA sa;
        SB sb;
        // PF2: a second register set takes the global loads of block kt+2
        // at the top of block kt and moves into the first set at its end, so
        // a load has two blocks of MFMA time to arrive instead of one
        SA sa2;
        SB sb2;
        if (ktiles > 0) {
            sa.template load<FAST>(g.A, g.lda, m0, 0, g.m, g.k, g.vec_a, tid);
            sb.template load<FAST>(g.B, g.ldb, n0, 0, g.n, g.k, g.vec_b, tid);
            sa.store(lds, tid);
            sb.store(lds + SA::FLOATS, tid);
        }
        if (PF2 && ktiles > 1) {
            sa.template load<FAST>(g.A, g.lda, m0, SH::BK, g.m, g.k, g.vec_a, tid);
            sb.template load<FAST>(g.B, g.ldb, n0, SH::BK, g.n, g.k, g.vec_b, tid);
        }
        __syncthreads();
        for (int64_t kt = 0; kt < ktiles; ++kt) {
            float *cur = lds + (kt & 1) * STAGE_FLOATS;
            float *nxt = lds + ((kt + 1) & 1) * STAGE_FLOATS;
            const bool more = kt + 1 < ktiles;
            if (PF2) {
                if (kt + 2 < ktiles) {
                    const int64_t k0 = (kt + 2) * SH::BK;
                    sa2.template load<FAST>(g.A, g.lda, m0, k0, g.m, g.k, g.vec_a, tid);
                    sb2.template load<FAST>(g.B, g.ldb, n0, k0, g.n, g.k, g.vec_b, tid);
                }
            } else if (more) {
                const int64_t k0 = (kt + 1) * SH::BK;
                sa.template load<FAST>(g.A, g.lda, m0, k0, g.m, g.k, g.vec_a, tid);
                sb.template load<FAST>(g.B, g.ldb, n0, k0, g.n, g.k, g.vec_b, tid);
            }
            const float *As = cur + wm * SH::WM + l32;
            const float *Bs = cur + SA::FLOATS + wn * SH::WN + l32;
#pragma unroll
            for (int ks = 0; ks < SH::BK / 2; ++ks) {
                const int kr = 2 * ks + half;  // lanes 0-31: even k, 32-63: odd k
                float a[SH::RM], b[SH::RN];
#pragma unroll
                for (int i = 0; i < SH::RM; ++i) a[i] = As[kr * SA::LD + i * 32];
#pragma unroll
                for (int j = 0; j < SH::RN; ++j) b[j] = Bs[kr * SB::LD + j * 32];
#pragma unroll
                for (int i = 0; i < SH::RM; ++i)
#pragma unroll
                    for (int j = 0; j < SH::RN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j],
                                                                          0, 0, 0);
            }
            if (more) {
                sa.store(nxt, tid);
                sb.store(nxt + SA::FLOATS, tid);
            }
            if (PF2 && kt + 2 < ktiles) {
                sa = sa2;
                sb = sb2;
            }
            __syncthreads();
        }
        finish<SPLIT, SH::RM, SH::RN>(g, acc, m0 + wm * SH::WM, n0 + wn * SH::WN, tid, NT);
    }
};

// ---------------------------------------------------------------------------
// Software-pipelined FP32 tile.  The operand fragments of K step s+1 are read
// from LDS before the MFMAs of step s are issued (so a LDS round trip never
// stalls the matrix core), and the LDS store of the next K block, whose
// global loads were issued at the top of the block, sits between the MFMAs
// of step STORE_STEP instead of after the last one.  The order is pinned
// with sched_barrier.
// ---------------------------------------------------------------------------
template <class SH, bool TA, bool TB>
struct F32PTile {
    using SA = StageF32<SH::BM, SH::BK, SH::NT, TA>;
    using SB = StageF32<SH::BN, SH::BK, SH::NT, !TB>;
    static constexpr int STAGE_FLOATS = SA::FLOATS + SB::FLOATS;
    static constexpr int LDS_BYTES = 2 * STAGE_FLOATS * 4;
    static constexpr int NT = SH::NT;
    static constexpr int RM = SH::RM, RN = SH::RN;
    static constexpr int NKS = SH::BK / 2;           // MFMA K steps per block
    static constexpr int STORE_STEP = NKS * 3 / 4;   // step that carries the store

    __device__ __forceinline__ static void read_frag(const float *As, const float *Bs, int ks,
                                                     int half, float (&a)[RM], float (&b)[RN])
    {
        const int kr = 2 * ks + half;  // lanes 0-31: even k, 32-63: odd k
#pragma unroll
        for (int i = 0; i < RM; ++i) a[i] = As[kr * SA::LD + i * 32];
#pragma unroll
        for (int j = 0; j < RN; ++j) b[j] = Bs[kr * SB::LD + j * 32];
    }

    __device__ __forceinline__ static void body(floatx16 (&acc)[RM][RN], const float *cur,
                                                float *nxt, const SA &sa, const SB &sb, int tid,
                                                int wm, int wn, int half, int l32)
    {
        const float *As = cur + wm * SH::WM + l32;
        const float *Bs = cur + SA::FLOATS + wn * SH::WN + l32;
        float a[2][RM], b[2][RN];
        read_frag(As, Bs, 0, half, a[0], b[0]);
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
            if (ks + 1 < NKS) {
                read_frag(As, Bs, ks + 1, half, a[(ks + 1) & 1], b[(ks + 1) & 1]);
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int i = 0; i < RM; ++i)
#pragma unroll
                for (int j = 0; j < RN; ++j) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[ks & 1][i], b[ks & 1][j],
                                                                      acc[i][j], 0, 0, 0);
                    if (ks == STORE_STEP && i == 0 && j == 0) {
                        __builtin_amdgcn_sched_barrier(0);
                        sa.store(nxt, tid);
                        sb.store(nxt + SA::FLOATS, tid);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
        }
    }

    // Interior tiles whose K range is a whole number of blocks take the
    // unmasked load path; every other tile masks its loads.
    template <bool SPLIT = false>
    __device__ __forceinline__ static void run(const GemmArgs &g, int64_t m0, int64_t n0,
                                               char *smem)
    {
        const bool fast = m0 + SH::BM <= g.m && n0 + SH::BN <= g.n && g.k % SH::BK == 0 &&
                          (g.vec_a || !SA::NEEDS_VEC) && (g.vec_b || !SB::NEEDS_VEC);
        if (fast) run_impl<true, SPLIT>(g, m0, n0, smem);
        else run_impl<false, SPLIT>(g, m0, n0, smem);
    }

    template <bool FAST, bool SPLIT>
    __device__ __forceinline__ static void run_impl(const GemmArgs &g, int64_t m0, int64_t n0,
                                                    char *smem)
    {
        float *lds = reinterpret_cast<float *>(smem);
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
        const int wm = wave % SH::NWM, wn = wave / SH::NWM;
        const int half = lane >> 5, l32 = lane & 31;

        floatx16 acc[RM][RN];
#pragma unroll
        for (int i = 0; i < RM; ++i)
#pragma unroll
            for (int j = 0; j < RN; ++j)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;

        const int64_t ktiles = (g.k + SH::BK - 1) / SH::BK;
        SA sa;
        SB sb;
        if (ktiles > 0) {
            sa.template load<FAST>(g.A, g.lda, m0, 0, g.m, g.k, g.vec_a, tid);
            sb.template load<FAST>(g.B, g.ldb, n0, 0, g.n, g.k, g.vec_b, tid);
            sa.store(lds, tid);
            sb.store(lds + SA::FLOATS, tid);
        }
        __syncthreads();
        for (int64_t kt = 0; kt < ktiles; ++kt) {
            const float *cur = lds + (kt & 1) * STAGE_FLOATS;
            float *nxt = lds + ((kt + 1) & 1) * STAGE_FLOATS;
            if (kt + 1 < ktiles) {
                const int64_t k0 = (kt + 1) * SH::BK;
                sa.template load<FAST>(g.A, g.lda, m0, k0, g.m, g.k, g.vec_a, tid);
                sb.template load<FAST>(g.B, g.ldb, n0, k0, g.n, g.k, g.vec_b, tid);
            }
            // On the last block the store rewrites the idle buffer with data
            // already consumed; nothing reads it afterwards.
            body(acc, cur, nxt, sa, sb, tid, wm, wn, half, l32);
            __syncthreads();
        }
        finish<SPLIT, RM, RN>(g, acc, m0 + wm * SH::WM, n0 + wn * SH::WN, tid, NT);
    }
};

template <class SH, bool TA, bool TB, bool ACC2>
struct X3Tile {
    using SA = StageX3<SH::BM, SH::BK, SH::NT, TA>;
    using SB = StageX3<SH::BN, SH::BK, SH::NT, !TB>;
    static_assert(SH::BK % 16 == 0, "bf16 MFMA consumes K in steps of 16");
    static constexpr int STAGE_HALVES = SA::HALVES + SB::HALVES;
    static constexpr int LDS_BYTES = 2 * STAGE_HALVES * 2;
    static constexpr int NT = SH::NT;

    // Interior tiles whose K range is a whole number of blocks take the
    // unmasked load path; every other tile masks its loads.
    template <bool SPLIT = false>
    __device__ __forceinline__ static void run(const GemmArgs &g, int64_t m0, int64_t n0,
                                               char *smem)
    {
        const bool fast = m0 + SH::BM <= g.m && n0 + SH::BN <= g.n && g.k % SH::BK == 0 &&
                          (g.vec_a || !SA::NEEDS_VEC) && (g.vec_b || !SB::NEEDS_VEC);
        if (fast) run_impl<true, SPLIT>(g, m0, n0, smem);
        else run_impl<false, SPLIT>(g, m0, n0, smem);
    }

    template <bool FAST, bool SPLIT>
    __device__ __forceinline__ static void run_impl(const GemmArgs &g, int64_t m0, int64_t n0,
                                                    char *smem)
    {
        __bf16 *lds = reinterpret_cast<__bf16 *>(smem);
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
        const int wm = wave % SH::NWM, wn = wave / SH::NWM;
        const int half = lane >> 5, l32 = lane & 31;

        floatx16 acc[SH::RM][SH::RN];
        floatx16 lo[ACC2 ? SH::RM : 1][ACC2 ? SH::RN : 1];
#pragma unroll
        for (int i = 0; i < SH::RM; ++i)
#pragma unroll
            for (int j = 0; j < SH::RN; ++j)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;
        if (ACC2) {
#pragma unroll
            for (int i = 0; i < (ACC2 ? SH::RM : 1); ++i)
#pragma unroll
                for (int j = 0; j < (ACC2 ? SH::RN : 1); ++j)
#pragma unroll
                    for (int e = 0; e < 16; ++e) lo[i][j][e] = 0.0f;
        }

        const int64_t ktiles = (g.k + SH::BK - 1) / SH::BK;
        SA sa;
        SB sb;
        if (ktiles > 0) {
            sa.template load<FAST>(g.A, g.lda, m0, 0, g.m, g.k, g.vec_a, tid);
            sb.template load<FAST>(g.B, g.ldb, n0, 0, g.n, g.k, g.vec_b, tid);
            sa.store(lds, tid);
            sb.store(lds + SA::HALVES, tid);
        }
        __syncthreads();
        for (int64_t kt = 0; kt < ktiles; ++kt) {
            __bf16 *cur = lds + (kt & 1) * STAGE_HALVES;
            __bf16 *nxt = lds + ((kt + 1) & 1) * STAGE_HALVES;
            const bool more = kt + 1 < ktiles;
            if (more) {
                const int64_t k0 = (kt + 1) * SH::BK;
                sa.template load<FAST>(g.A, g.lda, m0, k0, g.m, g.k, g.vec_a, tid);
                sb.template load<FAST>(g.B, g.ldb, n0, k0, g.n, g.k, g.vec_b, tid);
            }
            const __bf16 *As = cur + (wm * SH::WM + l32) * SA::LD + half * 8;
            const __bf16 *Bs = cur + SA::HALVES + (wn * SH::WN + l32) * SB::LD + half * 8;
#pragma unroll
            for (int ks = 0; ks < SH::BK / 16; ++ks) {
                bf16x8 a[SH::RM][3], b[SH::RN][3];
#pragma unroll
                for (int i = 0; i < SH::RM; ++i)
#pragma unroll
                    for (int t = 0; t < 3; ++t)
                        a[i][t] = *reinterpret_cast<const bf16x8 *>(
                            As + t * SA::PART + i * 32 * SA::LD + ks * 16);
#pragma unroll
                for (int j = 0; j < SH::RN; ++j)
#pragma unroll
                    for (int t = 0; t < 3; ++t)
                        b[j][t] = *reinterpret_cast<const bf16x8 *>(
                            Bs + t * SB::PART + j * 32 * SB::LD + ks * 16);
#pragma unroll
                for (int i = 0; i < SH::RM; ++i)
#pragma unroll
                    for (int j = 0; j < SH::RN; ++j) {
                        // smallest terms first; (0,0) is the leading product
                        floatx16 &small = ACC2 ? lo[ACC2 ? i : 0][ACC2 ? j : 0] : acc[i][j];
                        small = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][0], b[j][2], small, 0, 0, 0);
                        small = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][1], b[j][1], small, 0, 0, 0);
                        small = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][2], b[j][0], small, 0, 0, 0);
                        small = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][0], b[j][1], small, 0, 0, 0);
                        small = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][1], b[j][0], small, 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][0], b[j][0], acc[i][j], 0, 0, 0);
                    }
            }
            if (more) {
                sa.store(nxt, tid);
                sb.store(nxt + SA::HALVES, tid);
            }
            __syncthreads();
        }
        if (ACC2) {
#pragma unroll
            for (int i = 0; i < SH::RM; ++i)
#pragma unroll
                for (int j = 0; j < SH::RN; ++j)
                    acc[i][j] += lo[ACC2 ? i : 0][ACC2 ? j : 0];
        }
        finish<SPLIT, SH::RM, SH::RN>(g, acc, m0 + wm * SH::WM, n0 + wn * SH::WN, tid, NT);
    }
};

// ---------------------------------------------------------------------------
// Software-pipelined split-precision tile.  While the matrix cores work on K
// block kt from LDS, the global loads of block kt+1 are in flight, and once a
// fraction Q0_NUM/Q0_DEN of the block's MFMA instructions are issued the
// split and LDS store of block kt+1 are interleaved between the remaining
// ones.  One workgroup barrier per K block.
// ---------------------------------------------------------------------------
template <class SH, bool TA, bool TB, int Q0_NUM = 1, int Q0_DEN = 3, bool FENCED = false,
          bool PF2 = false>
struct X3PTile {
    using SA = StageX3<SH::BM, SH::BK, SH::NT, TA>;
    using SB = StageX3<SH::BN, SH::BK, SH::NT, !TB>;
    static_assert(SH::BK == 16, "one bf16 MFMA K step per K block");
    static_assert(SA::UNITS_FULL && SB::UNITS_FULL, "every thread stages whole units");
    static constexpr int STAGE_HALVES = SA::HALVES + SB::HALVES;
    static constexpr int LDS_BYTES = 2 * STAGE_HALVES * 2;
    static constexpr int NT = SH::NT;
    static constexpr int RM = SH::RM, RN = SH::RN;
    static constexpr int NMFMA = RM * RN * 6;
    static constexpr int NELEM = SA::KS * (SA::UNITS + SB::UNITS);
    // first MFMA slot that carries split/store work for the next block
    static constexpr int Q0 = NMFMA * Q0_NUM / Q0_DEN;

    // Split element e (A units first, then B units) of the staged block into
    // the pending part vectors; after the last element of a unit, write the
    // unit's three parts to LDS.
    __device__ __forceinline__ static void split_elem(int e, const SA &sa, const SB &sb,
                                                      __bf16 *dst, int tid, bf16x8 &p0,
                                                      bf16x8 &p1, bf16x8 &p2)
    {
        constexpr int KS = SA::KS;
        const int u = e / KS, q = e % KS;
        __bf16 h0, h1, h2;
        if (u < SA::UNITS) split3(sa.unit_val(u, q), h0, h1, h2);
        else split3(sb.unit_val(u - SA::UNITS, q), h0, h1, h2);
        p0[q] = h0;
        p1[q] = h1;
        p2[q] = h2;
        if (q == KS - 1) {
            __bf16 *base;
            int part;
            if (u < SA::UNITS) { base = dst + SA::unit_offset(u, tid); part = SA::PART; }
            else { base = dst + SA::HALVES + SB::unit_offset(u - SA::UNITS, tid); part = SB::PART; }
            *reinterpret_cast<bf16x8 *>(base) = p0;
            *reinterpret_cast<bf16x8 *>(base + part) = p1;
            *reinterpret_cast<bf16x8 *>(base + 2 * part) = p2;
        }
    }

    template <bool STORE>
    __device__ __forceinline__ static void body(floatx16 (&acc)[RM][RN], const __bf16 *cur,
                                                __bf16 *nxt, const SA &sa, const SB &sb,
                                                int tid, int wm, int wn, int half, int l32)
    {
        const __bf16 *As = cur + (wm * SH::WM + l32) * SA::LD + half * 8;
        const __bf16 *Bs = cur + SA::HALVES + (wn * SH::WN + l32) * SB::LD + half * 8;
        bf16x8 a[RM][3], b[2][3];
#pragma unroll
        for (int i = 0; i < RM; ++i)
#pragma unroll
            for (int t = 0; t < 3; ++t)
                a[i][t] = *reinterpret_cast<const bf16x8 *>(As + t * SA::PART + i * 32 * SA::LD);
#pragma unroll
        for (int t = 0; t < 3; ++t)
            b[0][t] = *reinterpret_cast<const bf16x8 *>(Bs + t * SB::PART);
        if constexpr (FENCED) {
            // Explicit order: after slot Q0 every MFMA is followed by the
            // split of a few elements (and the unit's LDS write when its last
            // element is done); sched_barrier keeps the compiler from moving
            // anything across.
            bf16x8 p0, p1, p2;
            int q = 0;
#pragma unroll
            for (int j = 0; j < RN; ++j) {
#pragma unroll
                for (int pr = 0; pr < 6; ++pr) {
#pragma unroll
                    for (int i = 0; i < RM; ++i) {
                        const int sa_i = pr == 0 ? 0 : pr == 1 ? 1 : pr == 2 ? 2 : pr == 3 ? 0 : pr == 4 ? 1 : 0;
                        const int sb_j = pr == 0 ? 2 : pr == 1 ? 1 : pr == 2 ? 0 : pr == 3 ? 1 : pr == 4 ? 0 : 0;
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            a[i][sa_i], b[j & 1][sb_j], acc[i][j], 0, 0, 0);
                        __builtin_amdgcn_sched_barrier(0);
                        if (i == 0 && pr == 0 && j + 1 < RN) {
#pragma unroll
                            for (int t = 0; t < 3; ++t)
                                b[(j + 1) & 1][t] = *reinterpret_cast<const bf16x8 *>(
                                    Bs + t * SB::PART + (j + 1) * 32 * SB::LD);
                            __builtin_amdgcn_sched_barrier(0);
                        }
                        if (STORE && q >= Q0) {
                            const int e0 = (q - Q0) * NELEM / (NMFMA - Q0);
                            const int e1 = (q + 1 - Q0) * NELEM / (NMFMA - Q0);
#pragma unroll
                            for (int e = e0; e < e1; ++e) split_elem(e, sa, sb, nxt, tid, p0, p1, p2);
                            if (e1 > e0) __builtin_amdgcn_sched_barrier(0);
                        }
                        ++q;
                    }
                }
            }
            return;
        }
#pragma unroll
        for (int j = 0; j < RN; ++j) {
            // products, smallest first: (0,2) (1,1) (2,0) (0,1) (1,0) (0,0);
            // consecutive MFMAs go to different accumulators (i varies fastest)
#pragma unroll
            for (int pr = 0; pr < 6; ++pr) {
#pragma unroll
                for (int i = 0; i < RM; ++i) {
                    const int sa_i = pr == 0 ? 0 : pr == 1 ? 1 : pr == 2 ? 2 : pr == 3 ? 0 : pr == 4 ? 1 : 0;
                    const int sb_j = pr == 0 ? 2 : pr == 1 ? 1 : pr == 2 ? 0 : pr == 3 ? 1 : pr == 4 ? 0 : 0;
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][sa_i], b[j & 1][sb_j],
                                                                         acc[i][j], 0, 0, 0);
                    if (i == 0 && pr == 0 && j + 1 < RN) {
#pragma unroll
                        for (int t = 0; t < 3; ++t)
                            b[(j + 1) & 1][t] = *reinterpret_cast<const bf16x8 *>(
                                Bs + t * SB::PART + (j + 1) * 32 * SB::LD);
                    }
                }
            }
        }
        if (STORE) {
#pragma unroll
            for (int u = 0; u < SA::UNITS; ++u) sa.store_unit(nxt, u, tid);
#pragma unroll
            for (int u = 0; u < SB::UNITS; ++u) sb.store_unit(nxt + SA::HALVES, u, tid);
        }
        // Issue order: the fragment reads first, then one MFMA at a time;
        // from MFMA slot Q0 on, each slot also carries a share of the split
        // (independent VALU work from several elements, so the in-order issue
        // does not wait on one element's dependency chain) and, every few
        // slots, one 16-byte LDS write.  B fragments of the next column are
        // read right after the first MFMA of the current column.
        constexpr int NWRITE = 3 * (SA::UNITS + SB::UNITS);
        constexpr int NVALU = 8 * NELEM;  // split work plus address arithmetic
        constexpr int SLOTS = NMFMA - Q0;
        constexpr int VPER = (NVALU + SLOTS - 1) / SLOTS;
        __builtin_amdgcn_sched_group_barrier(0x100, 3 * RM + 3, 0);
#pragma unroll
        for (int qq = 0; qq < NMFMA; ++qq) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            if (qq % (6 * RM) == 0 && qq / (6 * RM) + 1 < RN)
                __builtin_amdgcn_sched_group_barrier(0x100, 3, 0);
            if (STORE && qq >= Q0) {
                __builtin_amdgcn_sched_group_barrier(0x002, VPER, 0);
                if ((qq - Q0) * NWRITE / SLOTS != (qq + 1 - Q0) * NWRITE / SLOTS)
                    __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
            }
        }
    }

    // Interior tiles whose K range is a whole number of blocks take the
    // unmasked load path; every other tile masks its loads.
    template <bool SPLIT = false>
    __device__ __forceinline__ static void run(const GemmArgs &g, int64_t m0, int64_t n0,
                                               char *smem)
    {
        const bool fast = m0 + SH::BM <= g.m && n0 + SH::BN <= g.n && g.k % SH::BK == 0 &&
                          (g.vec_a || !SA::NEEDS_VEC) && (g.vec_b || !SB::NEEDS_VEC);
        if (fast) run_impl<true, SPLIT>(g, m0, n0, smem);
        else run_impl<false, SPLIT>(g, m0, n0, smem);
    }

    template <bool FAST, bool SPLIT>
    __device__ __forceinline__ static void run_impl(const GemmArgs &g, int64_t m0, int64_t n0,
                                                    char *smem)
    {
        __bf16 *lds = reinterpret_cast<__bf16 *>(smem);
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
        const int wm = wave % SH::NWM, wn = wave / SH::NWM;
        const int half = lane >> 5, l32 = lane & 31;

        floatx16 acc[RM][RN];
#pragma unroll
        for (int i = 0; i < RM; ++i)
#pragma unroll
            for (int j = 0; j < RN; ++j)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;

        const int64_t ktiles = (g.k + SH::BK - 1) / SH::BK;
        if constexpr (PF2) {
            // Two register sets: the global loads of block kt+2 go to the
            // second set at the top of block kt, while the first set (block
            // kt+1, loaded a whole block earlier) is split and stored between
            // the MFMAs; at the end of the block the second set moves into
            // the first.  A load thus has a block and a third of MFMA time to
            // arrive instead of a third, and the one body keeps the
            // accumulators in place.
            SA sa, sa2;
            SB sb, sb2;
            if (ktiles > 0) {
                sa.template load<FAST>(g.A, g.lda, m0, 0, g.m, g.k, g.vec_a, tid);
                sb.template load<FAST>(g.B, g.ldb, n0, 0, g.n, g.k, g.vec_b, tid);
                sa.store(lds, tid);
                sb.store(lds + SA::HALVES, tid);
            }
            if (ktiles > 1) {
                sa.template load<FAST>(g.A, g.lda, m0, SH::BK, g.m, g.k, g.vec_a, tid);
                sb.template load<FAST>(g.B, g.ldb, n0, SH::BK, g.n, g.k, g.vec_b, tid);
            }
            __syncthreads();
            for (int64_t kt = 0; kt < ktiles; ++kt) {
                const __bf16 *cur = lds + (kt & 1) * STAGE_HALVES;
                __bf16 *nxt = lds + ((kt + 1) & 1) * STAGE_HALVES;
                if (kt + 2 < ktiles) {
                    const int64_t k0 = (kt + 2) * SH::BK;
                    sa2.template load<FAST>(g.A, g.lda, m0, k0, g.m, g.k, g.vec_a, tid);
                    sb2.template load<FAST>(g.B, g.ldb, n0, k0, g.n, g.k, g.vec_b, tid);
                }
                // a store whose block does not exist rewrites an idle stage
                // that nothing reads again
                body<true>(acc, cur, nxt, sa, sb, tid, wm, wn, half, l32);
                if (kt + 2 < ktiles) {
                    sa = sa2;
                    sb = sb2;
                }
                __syncthreads();
            }
            finish<SPLIT, RM, RN>(g, acc, m0 + wm * SH::WM, n0 + wn * SH::WN, tid, NT);
            return;
        }
        SA sa;
        SB sb;
        if (ktiles > 0) {
            sa.template load<FAST>(g.A, g.lda, m0, 0, g.m, g.k, g.vec_a, tid);
            sb.template load<FAST>(g.B, g.ldb, n0, 0, g.n, g.k, g.vec_b, tid);
            sa.store(lds, tid);
            sb.store(lds + SA::HALVES, tid);
        }
        __syncthreads();
        for (int64_t kt = 0; kt < ktiles; ++kt) {
            const __bf16 *cur = lds + (kt & 1) * STAGE_HALVES;
            __bf16 *nxt = lds + ((kt + 1) & 1) * STAGE_HALVES;
            if (kt + 1 < ktiles) {
                const int64_t k0 = (kt + 1) * SH::BK;
                sa.template load<FAST>(g.A, g.lda, m0, k0, g.m, g.k, g.vec_a, tid);
                sb.template load<FAST>(g.B, g.ldb, n0, k0, g.n, g.k, g.vec_b, tid);
            }
            // On the last block the store rewrites the idle buffer with the
            // block already consumed; nothing reads it afterwards.  One body
            // for every iteration keeps the accumulators in place.
            body<true>(acc, cur, nxt, sa, sb, tid, wm, wn, half, l32);
            __syncthreads();
        }
        finish<SPLIT, RM, RN>(g, acc, m0 + wm * SH::WM, n0 + wn * SH::WN, tid, NT);
    }
};

// ---------------------------------------------------------------------------
// Small tiles for grids that leave CUs idle (a 256^3 problem has 16 tiles of
// 64x64): every one of KW waves holds the whole BM x BN tile and takes every
// KW-th K step of each staged block, so a tile's MFMA chain is KW times
// shorter; at the end the waves' accumulators are added in wave order
// through LDS and wave 0 stores.  The partial sums of one element therefore
// run over the k steps s = w (mod KW) of wave w, and the result is the same
// bits for every launch.
// ---------------------------------------------------------------------------
template <int BM_, int BN_, int BK_, int KW_>
struct WShape {
    static constexpr int BM = BM_, BN = BN_, BK = BK_, KW = KW_, OCC = 1;
    static constexpr int WM = BM, WN = BN, NWM = 1, NWN = 1, NW = KW, NT = 64 * KW;
    static constexpr int RM = BM / 32, RN = BN / 32;
    static_assert(BM % 32 == 0 && BN % 32 == 0, "the tile is made of 32x32 blocks");
};

// Waves 1..KW-1 post their accumulators to LDS (lane-contiguous, so every
// store and load of a wave is conflict-free), wave 0 adds them in wave
// order.  The caller's K loop ended with a barrier, so the staging buffers
// are free.
template <int KW, int RM, int RN>
__device__ __forceinline__ void wave_sum(floatx16 (&acc)[RM][RN], float *lds, int wave,
                                         int lane)
{
    constexpr int PER = RM * RN * 16 * 64;
    if (wave > 0) {
        float *dst = lds + (wave - 1) * PER;
#pragma unroll
        for (int i = 0; i < RM; ++i)
#pragma unroll
            for (int j = 0; j < RN; ++j)
#pragma unroll
                for (int e = 0; e < 16; ++e) dst[((i * RN + j) * 16 + e) * 64 + lane] = acc[i][j][e];
    }
    __syncthreads();
    if (wave == 0) {
        for (int w = 1; w < KW; ++w) {
            const float *src = lds + (w - 1) * PER;
#pragma unroll
            for (int i = 0; i < RM; ++i)
#pragma unroll
                for (int j = 0; j < RN; ++j)
#pragma unroll
                    for (int e = 0; e < 16; ++e)
                        acc[i][j][e] += src[((i * RN + j) * 16 + e) * 64 + lane];
        }
    }
}

template <class SH, bool TA, bool TB>
struct F32WTile {
    using SA = StageF32<SH::BM, SH::BK, SH::NT, TA>;
    using SB = StageF32<SH::BN, SH::BK, SH::NT, !TB>;
    static constexpr int KW = SH::KW, RM = SH::RM, RN = SH::RN, NT = SH::NT;
    static constexpr int STEPS = SH::BK / 2;  // two k per v_mfma_f32_32x32x2_f32
    static_assert(STEPS % KW == 0, "every wave takes the same number of k steps");
    static constexpr int STAGE_FLOATS = SA::FLOATS + SB::FLOATS;
    static constexpr int RED_FLOATS = (KW - 1) * RM * RN * 16 * 64;
    static constexpr int LDS_BYTES =
        (2 * STAGE_FLOATS > RED_FLOATS ? 2 * STAGE_FLOATS : RED_FLOATS) * 4;

    template <bool SPLIT = false>
    __device__ __forceinline__ static void run(const GemmArgs &g, int64_t m0, int64_t n0,
                                               char *smem)
    {
        static_assert(!SPLIT, "no split-K variant");
        const bool fast = m0 + SH::BM <= g.m && n0 + SH::BN <= g.n && g.k % SH::BK == 0 &&
                          (g.vec_a || !SA::NEEDS_VEC) && (g.vec_b || !SB::NEEDS_VEC);
        if (fast) run_impl<true>(g, m0, n0, smem);
        else run_impl<false>(g, m0, n0, smem);
    }

    template <bool FAST>
    __device__ __forceinline__ static void run_impl(const GemmArgs &g, int64_t m0, int64_t n0,
                                                    char *smem)
    {
        float *lds = reinterpret_cast<float *>(smem);
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
        const int half = lane >> 5, l32 = lane & 31;
        floatx16 acc[RM][RN];
#pragma unroll
        for (int i = 0; i < RM; ++i)
#pragma unroll
            for (int j = 0; j < RN; ++j)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;
        const int64_t ktiles = (g.k + SH::BK - 1) / SH::BK;
        SA sa;
        SB sb;
        if (ktiles > 0) {
            sa.template load<FAST>(g.A, g.lda, m0, 0, g.m, g.k, g.vec_a, tid);
            sb.template load<FAST>(g.B, g.ldb, n0, 0, g.n, g.k, g.vec_b, tid);
            sa.store(lds, tid);
            sb.store(lds + SA::FLOATS, tid);
        }
        __syncthreads();
        for (int64_t kt = 0; kt < ktiles; ++kt) {
            float *cur = lds + (kt & 1) * STAGE_FLOATS;
            float *nxt = lds + ((kt + 1) & 1) * STAGE_FLOATS;
            const bool more = kt + 1 < ktiles;
            if (more) {
                const int64_t k0 = (kt + 1) * SH::BK;
                sa.template load<FAST>(g.A, g.lda, m0, k0, g.m, g.k, g.vec_a, tid);
                sb.template load<FAST>(g.B, g.ldb, n0, k0, g.n, g.k, g.vec_b, tid);
            }
            const float *As = cur + l32;
            const float *Bs = cur + SA::FLOATS + l32;
#pragma unroll
            for (int s = 0; s < STEPS / KW; ++s) {
                const int kr = 2 * (s * KW + wave) + half;  // lanes 0-31: even k, 32-63: odd k
                float a[RM], b[RN];
#pragma unroll
                for (int i = 0; i < RM; ++i) a[i] = As[kr * SA::LD + i * 32];
#pragma unroll
                for (int j = 0; j < RN; ++j) b[j] = Bs[kr * SB::LD + j * 32];
#pragma unroll
                for (int i = 0; i < RM; ++i)
#pragma unroll
                    for (int j = 0; j < RN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j],
                                                                          0, 0, 0);
            }
            if (more) {
                sa.store(nxt, tid);
                sb.store(nxt + SA::FLOATS, tid);
            }
            __syncthreads();
        }
        wave_sum<KW, RM, RN>(acc, lds, wave, lane);
        if (wave == 0) epilogue<RM, RN>(g, acc, m0, n0, lane);
    }
};

// The split form of the small tile: each K block holds KW steps of 16 k,
// one per wave, split while staged; a wave adds its six part products
// smallest first into one accumulator, as the large split-form tiles do.
template <class SH, bool TA, bool TB>
struct X3WTile {
    using SA = StageX3<SH::BM, SH::BK, SH::NT, TA>;
    using SB = StageX3<SH::BN, SH::BK, SH::NT, !TB>;
    static constexpr int KW = SH::KW, RM = SH::RM, RN = SH::RN, NT = SH::NT;
    static constexpr int STEPS = SH::BK / 16;  // 16 k per v_mfma_f32_32x32x16_bf16
    static_assert(STEPS % KW == 0, "every wave takes the same number of k steps");
    static constexpr int STAGE_HALVES = SA::HALVES + SB::HALVES;
    static constexpr int RED_FLOATS = (KW - 1) * RM * RN * 16 * 64;
    static constexpr int LDS_BYTES =
        (2 * STAGE_HALVES * 2 > RED_FLOATS * 4 ? 2 * STAGE_HALVES * 2 : RED_FLOATS * 4);

    template <bool SPLIT = false>
    __device__ __forceinline__ static void run(const GemmArgs &g, int64_t m0, int64_t n0,
                                               char *smem)
    {
        static_assert(!SPLIT, "no split-K variant");
        const bool fast = m0 + SH::BM <= g.m && n0 + SH::BN <= g.n && g.k % SH::BK == 0 &&
                          (g.vec_a || !SA::NEEDS_VEC) && (g.vec_b || !SB::NEEDS_VEC);
        if (fast) run_impl<true>(g, m0, n0, smem);
        else run_impl<false>(g, m0, n0, smem);
    }

    template <bool FAST>
    __device__ __forceinline__ static void run_impl(const GemmArgs &g, int64_t m0, int64_t n0,
                                                    char *smem)
    {
        __bf16 *lds = reinterpret_cast<__bf16 *>(smem);
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
        const int half = lane >> 5, l32 = lane & 31;
        floatx16 acc[RM][RN];
#pragma unroll
        for (int i = 0; i < RM; ++i)
#pragma unroll
            for (int j = 0; j < RN; ++j)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;
        const int64_t ktiles = (g.k + SH::BK - 1) / SH::BK;
        SA sa;
        SB sb;
        if (ktiles > 0) {
            sa.template load<FAST>(g.A, g.lda, m0, 0, g.m, g.k, g.vec_a, tid);
            sb.template load<FAST>(g.B, g.ldb, n0, 0, g.n, g.k, g.vec_b, tid);
            sa.store(lds, tid);
            sb.store(lds + SA::HALVES, tid);
        }
        __syncthreads();
        for (int64_t kt = 0; kt < ktiles; ++kt) {
            __bf16 *cur = lds + (kt & 1) * STAGE_HALVES;
            __bf16 *nxt = lds + ((kt + 1) & 1) * STAGE_HALVES;
            const bool more = kt + 1 < ktiles;
            if (more) {
                const int64_t k0 = (kt + 1) * SH::BK;
                sa.template load<FAST>(g.A, g.lda, m0, k0, g.m, g.k, g.vec_a, tid);
                sb.template load<FAST>(g.B, g.ldb, n0, k0, g.n, g.k, g.vec_b, tid);
            }
            const __bf16 *As = cur + l32 * SA::LD + half * 8;
            const __bf16 *Bs = cur + SA::HALVES + l32 * SB::LD + half * 8;
#pragma unroll
            for (int s = 0; s < STEPS / KW; ++s) {
                const int ks = s * KW + wave;
                bf16x8 a[RM][3], b[RN][3];
#pragma unroll
                for (int i = 0; i < RM; ++i)
#pragma unroll
                    for (int t = 0; t < 3; ++t)
                        a[i][t] = *reinterpret_cast<const bf16x8 *>(
                            As + t * SA::PART + i * 32 * SA::LD + ks * 16);
#pragma unroll
                for (int j = 0; j < RN; ++j)
#pragma unroll
                    for (int t = 0; t < 3; ++t)
                        b[j][t] = *reinterpret_cast<const bf16x8 *>(
                            Bs + t * SB::PART + j * 32 * SB::LD + ks * 16);
#pragma unroll
                for (int i = 0; i < RM; ++i)
#pragma unroll
                    for (int j = 0; j < RN; ++j) {
                        floatx16 &c = acc[i][j];
                        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][0], b[j][2], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][1], b[j][1], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][2], b[j][0], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][0], b[j][1], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][1], b[j][0], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][0], b[j][0], c, 0, 0, 0);
                    }
            }
            if (more) {
                sa.store(nxt, tid);
                sb.store(nxt + SA::HALVES, tid);
            }
            __syncthreads();
        }
        wave_sum<KW, RM, RN>(acc, reinterpret_cast<float *>(smem), wave, lane);
        if (wave == 0) epilogue<RM, RN>(g, acc, m0, n0, lane);
    }
};

// ---------------------------------------------------------------------------
// Tile order: blocks are dispatched round-robin over the 8 XCDs (block b goes
// to XCD b % 8).  Renumber so that each XCD receives a contiguous range of
// tile ids, then walk tiles in groups of GROUP_M tile-rows so that the tiles
// resident on one XCD share A row-panels and B column-panels in its L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nb)
{
    const int64_t q = nb / 8, r = nb % 8;
    const int64_t x = bid % 8, idx = bid / 8;
    const int64_t base = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    return base + idx;
}

__device__ __forceinline__ void tile_coords(int64_t t, int64_t tiles_m, int64_t tiles_n,
                                            int group_m, int64_t &tm, int64_t &tn)
{
    const int64_t per_group = (int64_t)group_m * tiles_n;
    const int64_t grp = t / per_group;
    const int64_t first_m = grp * group_m;
    const int64_t gsize = tiles_m - first_m < group_m ? tiles_m - first_m : group_m;
    const int64_t in_grp = t - grp * per_group;
    tm = first_m + in_grp % gsize;
    tn = in_grp / gsize;
}

}  // namespace misgemm
