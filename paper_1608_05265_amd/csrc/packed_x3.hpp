// Packed split-precision path: the BLIS packing step made explicit.
//
// pack_x3 turns op(A) (and op(B)) into "packed panels": for every block of
// 16 consecutive k, for every part t of the bf16 split, for each half h of
// the block (k 0-7, k 8-15), for every row r (rows padded to a multiple of
// PACK_ROWS, k padded to a multiple of 16, both with zeros) the 8 bf16 values
// of that row, 16 contiguous bytes:
//     P[(((kb * 3 + t) * 2 + h) * rows_pad + r) * 8 + (k % 8)]
// The layout no longer depends on transposes or leading dimensions (as
// BLIS's packed micro-panels, Section III-A of the paper), so one tile
// kernel serves all four transpose pairs, with no masking in its main loop
// and no split work between its MFMAs: a K block of a tile is six
// contiguous runs of rows*16 bytes per operand, copied to LDS unchanged, and
// 32 rows x 16 k of one part is exactly one 32x32x16 MFMA operand, which a
// wave reads as two contiguous runs of 512 bytes (lanes 0-31 the low half of
// k, lanes 32-63 the high half), free of LDS bank conflicts.
#pragma once

#include "gemm_tile.hpp"

namespace misgemm {

constexpr int PACK_ROWS = 256;  // row padding of packed panels (largest tile)
constexpr int PACK_K = 16;      // k per packed block

__host__ __device__ inline int64_t pack_rows_pad(int64_t rows)
{
    return (rows + PACK_ROWS - 1) / PACK_ROWS * PACK_ROWS;
}

__host__ __device__ inline int64_t pack_kblocks(int64_t k) { return (k + PACK_K - 1) / PACK_K; }

// bf16 elements of one packed operand.
__host__ __device__ inline int64_t pack_halves(int64_t rows, int64_t k)
{
    return pack_kblocks(k) * 3 * pack_rows_pad(rows) * PACK_K;
}

// One thread per (row, 16-k block): row r, k block kb of op(X), split and
// written to the three part runs of its panel.  KC: op(X)(r, k) = X[k + r*ld]
// (k contiguous); otherwise X[r + k*ld] (rows contiguous, so a wave's loads
// of one k are coalesced).  Rows in [rows, rows_pad) and k past kdim are
// written as zeros.
template <bool KC>
__device__ __forceinline__ void pack_unit(const float *__restrict__ X, int64_t ld, int64_t rows,
                                          int64_t kdim, int64_t rows_pad, int vec,
                                          __bf16 *__restrict__ out, int64_t r, int64_t kb)
{
    const int64_t k0 = kb * PACK_K;
    float v[PACK_K];
    const bool in_r = r < rows;
    if (KC) {
        const float *p = X + k0 + r * ld;
        if (vec && in_r && k0 + PACK_K <= kdim) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const floatx4 x = *reinterpret_cast<const floatx4 *>(p + 4 * q);
#pragma unroll
                for (int e = 0; e < 4; ++e) v[4 * q + e] = x[e];
            }
        } else {
#pragma unroll
            for (int e = 0; e < PACK_K; ++e) v[e] = (in_r && k0 + e < kdim) ? p[e] : 0.0f;
        }
    } else {
        const float *p = X + r + k0 * ld;
#pragma unroll
        for (int e = 0; e < PACK_K; ++e) v[e] = (in_r && k0 + e < kdim) ? p[e * ld] : 0.0f;
    }
    bf16x8 lo[3], hi[3];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        __bf16 a0, a1, a2, b0, b1, b2;
        split3(v[e], a0, a1, a2);
        split3(v[8 + e], b0, b1, b2);
        lo[0][e] = a0; lo[1][e] = a1; lo[2][e] = a2;
        hi[0][e] = b0; hi[1][e] = b1; hi[2][e] = b2;
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        __bf16 *dst = out + ((kb * 3 + t) * 2 * rows_pad + r) * 8;
        *reinterpret_cast<bf16x8 *>(dst) = lo[t];
        *reinterpret_cast<bf16x8 *>(dst + rows_pad * 8) = hi[t];
    }
}

template <bool KC>
__global__ __launch_bounds__(256) void pack_x3_kernel(const float *__restrict__ X, int64_t ld,
                                                      int64_t rows, int64_t kdim,
                                                      int64_t rows_pad, int vec,
                                                      __bf16 *__restrict__ out)
{
    pack_unit<KC>(X, ld, rows, kdim, rows_pad, vec, out, (int64_t)blockIdx.x * 256 + threadIdx.x,
                  blockIdx.y);
}

// One operand of one problem of a packed batch: its blocks of 256 rows x 16
// k are blocks [first_block, first_block + row_blocks * kblocks) of the
// batch's pack launch (row block fastest).
struct PackJob {
    const float *X;
    __bf16 *out;
    int64_t ld, rows, kdim, rows_pad;
    int64_t first_block, row_blocks;
    int32_t kc, vec;
};

// Arguments of the packed tile kernel.
struct PackedArgs {
    GemmArgs g;           // m, n, C, ldc, alpha, beta, vec_c (A, B, k unused)
    const __bf16 *Ap;     // packed op(A): rows m
    const __bf16 *Bp;     // packed op(B): rows n
    int64_t mp, np;       // padded row counts
    int64_t kblocks;      // number of 16-k blocks
};

// ---------------------------------------------------------------------------
// Tile kernel on packed panels.  Two LDS stages; the 16-byte pieces of K
// block kb+1 are fetched at the top of block kb and written to the idle
// stage after STORE_AT of the block's MFMAs, one barrier per block.
// ---------------------------------------------------------------------------
template <class SH>
struct X3KTile {
    static constexpr int BM = SH::BM, BN = SH::BN;
    static constexpr int RM = SH::RM, RN = SH::RN, NT = SH::NT;
    static constexpr int A_HALVES = 3 * BM * PACK_K, B_HALVES = 3 * BN * PACK_K;
    static constexpr int STAGE_HALVES = A_HALVES + B_HALVES;
    static constexpr int LDS_BYTES = 2 * STAGE_HALVES * 2;
    static constexpr int PIECES = STAGE_HALVES / 8;     // 16-byte pieces per stage
    static constexpr int A_PIECES = A_HALVES / 8;
    static constexpr int PPT = PIECES / NT;             // pieces per thread
    static_assert(PIECES % NT == 0, "whole pieces per thread");
    static_assert(BM <= PACK_ROWS && PACK_ROWS % BM == 0 && PACK_ROWS % BN == 0,
                  "tiles divide the packed row padding");
    static constexpr int NMFMA = RM * RN * 6;
    static constexpr int STORE_AT = NMFMA * 2 / 3;

    struct Stage {
        bf16x8 v[PPT];
    };

    // Source of 16-byte piece q of K block kb: A pieces first, in the order
    // part t, half h, row r (the order of the stage in LDS), then B.
    __device__ __forceinline__ static const __bf16 *piece(const PackedArgs &p, int64_t m0,
                                                         int64_t n0, int64_t kb, int q)
    {
        if (q < A_PIECES) {
            const int t = q / (BM * 2), h = (q / BM) % 2, r = q % BM;
            return p.Ap + (((kb * 3 + t) * 2 + h) * p.mp + m0 + r) * 8;
        }
        const int qb = q - A_PIECES;
        const int t = qb / (BN * 2), h = (qb / BN) % 2, r = qb % BN;
        return p.Bp + (((kb * 3 + t) * 2 + h) * p.np + n0 + r) * 8;
    }

    __device__ __forceinline__ static void load(Stage &st, const PackedArgs &p, int64_t m0,
                                                int64_t n0, int64_t kb, int tid)
    {
#pragma unroll
        for (int s = 0; s < PPT; ++s) {
            const int q = tid + s * NT;
            st.v[s] = *reinterpret_cast<const bf16x8 *>(piece(p, m0, n0, kb, q));
        }
    }

    // LDS stage layout: A part t, half h, row r at ((t*2 + h)*BM + r)*8, then B
    // likewise; piece q lands at q*8 halves.
    __device__ __forceinline__ static void store(const Stage &st, __bf16 *dst, int tid)
    {
#pragma unroll
        for (int s = 0; s < PPT; ++s)
            *reinterpret_cast<bf16x8 *>(dst + (tid + s * NT) * 8) = st.v[s];
    }

    __device__ __forceinline__ static void body(floatx16 (&acc)[RM][RN], const __bf16 *cur,
                                                __bf16 *nxt, const Stage &st, int tid, int wm,
                                                int wn, int half, int l32)
    {
        const __bf16 *As = cur + (half * BM + wm * SH::WM + l32) * 8;
        const __bf16 *Bs = cur + A_HALVES + (half * BN + wn * SH::WN + l32) * 8;
        bf16x8 a[RM][3], b[2][3];
#pragma unroll
        for (int i = 0; i < RM; ++i)
#pragma unroll
            for (int t = 0; t < 3; ++t)
                a[i][t] = *reinterpret_cast<const bf16x8 *>(As + (t * 2 * BM + i * 32) * 8);
#pragma unroll
        for (int t = 0; t < 3; ++t)
            b[0][t] = *reinterpret_cast<const bf16x8 *>(Bs + t * 2 * BN * 8);
        int q = 0;
#pragma unroll
        for (int j = 0; j < RN; ++j) {
            // products smallest first; i fastest so consecutive MFMAs use
            // different accumulators
#pragma unroll
            for (int pr = 0; pr < 6; ++pr) {
#pragma unroll
                for (int i = 0; i < RM; ++i) {
                    const int sa = pr == 0 ? 0 : pr == 1 ? 1 : pr == 2 ? 2 : pr == 3 ? 0 : pr == 4 ? 1 : 0;
                    const int sb = pr == 0 ? 2 : pr == 1 ? 1 : pr == 2 ? 0 : pr == 3 ? 1 : pr == 4 ? 0 : 0;
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][sa], b[j & 1][sb],
                                                                         acc[i][j], 0, 0, 0);
                    __builtin_amdgcn_sched_barrier(0);
                    if (i == 0 && pr == 0 && j + 1 < RN) {
#pragma unroll
                        for (int t = 0; t < 3; ++t)
                            b[(j + 1) & 1][t] = *reinterpret_cast<const bf16x8 *>(
                                Bs + (t * 2 * BN + (j + 1) * 32) * 8);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    if (q == STORE_AT) {
                        store(st, nxt, tid);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    ++q;
                }
            }
        }
    }

    // The MFMA part of body() alone (operands already in LDS, nothing to store).
    __device__ __forceinline__ static void body_nostore(floatx16 (&acc)[RM][RN],
                                                        const __bf16 *cur, int tid, int wm,
                                                        int wn, int half, int l32)
    {
        const __bf16 *As = cur + (half * BM + wm * SH::WM + l32) * 8;
        const __bf16 *Bs = cur + A_HALVES + (half * BN + wn * SH::WN + l32) * 8;
        bf16x8 a[RM][3], b[2][3];
#pragma unroll
        for (int i = 0; i < RM; ++i)
#pragma unroll
            for (int t = 0; t < 3; ++t)
                a[i][t] = *reinterpret_cast<const bf16x8 *>(As + (t * 2 * BM + i * 32) * 8);
#pragma unroll
        for (int t = 0; t < 3; ++t)
            b[0][t] = *reinterpret_cast<const bf16x8 *>(Bs + t * 2 * BN * 8);
        (void)tid;
#pragma unroll
        for (int j = 0; j < RN; ++j) {
            // products smallest first; i fastest so consecutive MFMAs use
            // different accumulators
#pragma unroll
            for (int pr = 0; pr < 6; ++pr) {
#pragma unroll
                for (int i = 0; i < RM; ++i) {
                    const int sa = pr == 0 ? 0 : pr == 1 ? 1 : pr == 2 ? 2 : pr == 3 ? 0 : pr == 4 ? 1 : 0;
                    const int sb = pr == 0 ? 2 : pr == 1 ? 1 : pr == 2 ? 0 : pr == 3 ? 1 : pr == 4 ? 0 : 0;
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][sa], b[j & 1][sb],
                                                                         acc[i][j], 0, 0, 0);
                    __builtin_amdgcn_sched_barrier(0);
                    if (i == 0 && pr == 0 && j + 1 < RN) {
#pragma unroll
                        for (int t = 0; t < 3; ++t)
                            b[(j + 1) & 1][t] = *reinterpret_cast<const bf16x8 *>(
                                Bs + (t * 2 * BN + (j + 1) * 32) * 8);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
            }
        }
    }

    __device__ __forceinline__ static void run(const PackedArgs &p, int64_t m0, int64_t n0,
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
        Stage st;
        if (p.kblocks > 0) {
            load(st, p, m0, n0, 0, tid);
            store(st, lds, tid);
        }
        __syncthreads();
        for (int64_t kb = 0; kb < p.kblocks; ++kb) {
            const __bf16 *cur = lds + (kb & 1) * STAGE_HALVES;
            __bf16 *nxt = lds + ((kb + 1) & 1) * STAGE_HALVES;
            if (kb + 1 < p.kblocks) load(st, p, m0, n0, kb + 1, tid);
            // the last block's store rewrites the idle stage; nothing reads it
            body(acc, cur, nxt, st, tid, wm, wn, half, l32);
            __syncthreads();
        }
        epilogue<RM, RN>(p.g, acc, m0 + wm * SH::WM, n0 + wn * SH::WN, lane);
    }
};

}  // namespace misgemm

namespace misgemm {

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void global_void_t;

// ---------------------------------------------------------------------------
// Tile kernel on packed panels with direct global->LDS loads
// (global_load_lds_dwordx4: each lane's 16 bytes land at the wave's LDS base
// + 16 * lane, so a wave copies 1 KB of a panel without touching VGPRs) and
// three LDS stages: the copy of K block kb+2 is in flight while block kb is
// multiplied.  The loop is unrolled by three so that every stage is a
// distinct LDS array and the wait before reading a stage covers only the
// copies into that stage.
// ---------------------------------------------------------------------------
template <class SH>
struct X3DTile {
    using K = X3KTile<SH>;
    static constexpr int RM = SH::RM, RN = SH::RN, NT = SH::NT;
    static constexpr int STAGE_BYTES = K::STAGE_HALVES * 2;
    static constexpr int PPT = K::PPT;

    // Issue the copies of K block kb into `stage`.
    __device__ __forceinline__ static void issue(const PackedArgs &p, int64_t m0, int64_t n0,
                                                 int64_t kb, __bf16 *stage, int tid)
    {
        const int wave = tid >> 6;
#pragma unroll
        for (int s = 0; s < PPT; ++s) {
            const int q = tid + s * NT;
            const __bf16 *src = K::piece(p, m0, n0, kb, q);
            __bf16 *dst = stage + (s * NT + wave * 64) * 8;  // wave-uniform base
            __builtin_amdgcn_global_load_lds((global_void_t *)src, (lds_void_t *)dst, 16, 0, 0);
        }
    }

    // One K block from `stage`: wait for this thread's copies into it (the
    // copies of the following block may stay in flight), make every wave's
    // copies visible, start the copies of block kb+2 into the stage freed by
    // block kb-1, and multiply.
    __device__ __forceinline__ static void step(floatx16 (&acc)[RM][RN], const PackedArgs &p,
                                                int64_t m0, int64_t n0, int64_t kb,
                                                __bf16 *stage, __bf16 *next2, int tid, int wm,
                                                int wn, int half, int l32)
    {
        if (kb + 1 < p.kblocks) __builtin_amdgcn_s_waitcnt(0x0f70 | (PPT & 15) | ((PPT >> 4) << 14));
        else __builtin_amdgcn_s_waitcnt(0x0f70);
        // A bare barrier: the wait above already completed this thread's
        // copies into the stage; a release fence here would also wait for
        // the copies of the next block, which must stay in flight.  The empty
        // asm keeps the compiler from moving LDS accesses across it.
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        if (kb + 2 < p.kblocks) issue(p, m0, n0, kb + 2, next2, tid);
        K::body_nostore(acc, stage, tid, wm, wn, half, l32);
    }

    __device__ __forceinline__ static void run(const PackedArgs &p, int64_t m0, int64_t n0,
                                               __bf16 *s0, __bf16 *s1, __bf16 *s2)
    {
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
        if (p.kblocks > 0) issue(p, m0, n0, 0, s0, tid);
        if (p.kblocks > 1) issue(p, m0, n0, 1, s1, tid);
        for (int64_t kb = 0; kb < p.kblocks; kb += 3) {
            step(acc, p, m0, n0, kb, s0, s2, tid, wm, wn, half, l32);
            if (kb + 1 < p.kblocks) step(acc, p, m0, n0, kb + 1, s1, s0, tid, wm, wn, half, l32);
            if (kb + 2 < p.kblocks) step(acc, p, m0, n0, kb + 2, s2, s1, tid, wm, wn, half, l32);
        }
        epilogue<RM, RN>(p.g, acc, m0 + wm * SH::WM, n0 + wn * SH::WN, lane);
    }
};

}  // namespace misgemm
