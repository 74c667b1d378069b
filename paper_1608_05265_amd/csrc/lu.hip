// LU factorization with partial pivoting and the solve that uses it: the
// Linpack (HPL) workload of the paper's Section IV-C, on the sgemm path.
//
// Recursive right-looking LU: factor the left half of the column range,
// L11^{-1} A12 (recursive triangular solve), A22 -= A21 A12 (one sgemm --
// the rank-k trailing update), factor A22.  Almost all flops land in sgemm
// calls of decreasing size.  The leaves are narrow panels (8 columns, 4
// when the panel is taller than 8192 rows) that one workgroup factors with
// the panel held in registers (panels taller than 16384 rows are factored
// in memory, 8 columns at a time); where both halves of a node are leaves,
// the right one also applies the node's solve and update.  Each leaf's row
// interchanges are applied to every other column of the matrix right after
// it, which gives the same result as swapping at each level of the
// recursion (a column receives the interchanges in pivot order either way,
// and the columns right of a range are not touched before its left half is
// done); for a node whose halves are both leaves, the right leaf (or, for
// leaves too tall to take the node's update, the node's triangular-solve
// leaf) first applies the left one's interchanges to the right half's
// columns, and one launch after the pair applies both leaves' to every
// other column.  The solve applies the interchanges to the right-hand
// sides and then the two triangular solves; with few right-hand sides the
// interchanges run in LDS and the triangular recursion stops at 1024-row
// diagonal blocks that one workgroup solves.
#include <hip/hip_runtime.h>
#include <float.h>
#include <stdint.h>

#include "../../include/misgemm.h"

namespace {

constexpr int LEAF = 64;            // rows of a leaf triangular solve (one per lane)
constexpr int PANEL_LEAF = 8;       // columns of a leaf panel
constexpr int LEAF_THREADS = 1024;  // threads of the leaf-panel workgroup
constexpr int LEAF_WAVES = LEAF_THREADS / 64;
constexpr int LEAF_REGS = 64;       // panel values one thread holds
constexpr int LEAF_UPD_RPT = 16;    // tallest leaf (rows per thread) that fuses its sibling's update
constexpr int SWAP_BLOCK = 32;      // interchanges composed into one permutation
constexpr int SWAP_THREADS = 256;   // laswp workgroup: four wavefronts
constexpr int SWAP_COLS_PER_WAVE = 16;
// One-workgroup triangular solve for a few right-hand sides (the solve
// after the factorization): up to TRSV_ROWS rows per launch, used when the
// right-hand sides number at most TRSV_MAX_RHS.
constexpr int TRSV_ROWS = 1024;
constexpr int64_t TRSV_MAX_RHS = 16;
// Rows of a column whose interchanges are applied in LDS (the column and
// the pivot list: 8 bytes per row).
constexpr int LASWP_LDS_ROWS = 16384;

// Pivot search key: the magnitude's bits above the complemented row index.
// Magnitudes are non-negative, so their bit patterns order as the values
// do, and the largest key is the largest magnitude at the lowest row -- the
// first row of largest magnitude, as a sequential scan finds it.  0 means
// "no candidate" (a row whose magnitude is NaN is never one).
__device__ inline uint64_t pivot_key(float mag, int row)
{
    return ((uint64_t)__float_as_uint(mag) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)row);
}

// v from another lane of the same 16-lane row (DPP control CTRL).
template <int CTRL>
__device__ inline uint32_t dpp32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, true);
}

__device__ inline uint32_t readlane32(uint32_t v, int lane)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

__device__ inline uint64_t readlane64(uint64_t v, int lane)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// Maximum (MIN false) or minimum (MIN true) over the wavefront (all lanes
// active), uniform: within each 16-lane row exchange with the neighbour
// (quad_perm 1,0,3,2), the other pair (quad_perm 2,3,0,1), the mirrored
// quad in the half row and the mirrored half row; then the four rows
// through scalar readlanes.
template <bool MIN>
__device__ inline uint32_t wave_reduce_u32(uint32_t v)
{
    const auto op = [](uint32_t a, uint32_t b) { return MIN ? (a < b ? a : b) : (a > b ? a : b); };
    v = op(v, dpp32<0xB1>(v));
    v = op(v, dpp32<0x4E>(v));
    v = op(v, dpp32<0x141>(v));
    v = op(v, dpp32<0x140>(v));
    return op(op(readlane32(v, 0), readlane32(v, 16)), op(readlane32(v, 32), readlane32(v, 48)));
}

// The wavefront's largest pivot key (uniform; 0 when no lane has a
// candidate): from each lane's best magnitude (negative: none) and its row,
// the largest magnitude first, then the smallest row among the lanes that
// hold it -- the same key as the maximum of the lanes' pivot keys, in two
// 32-bit reductions instead of one over 64-bit keys.
__device__ inline uint64_t wave_pivot_key(float best, int row)
{
    const uint32_t u = best >= 0.0f ? __float_as_uint(best) + 1u : 0u;
    const uint32_t umax = wave_reduce_u32<false>(u);
    if (umax == 0) return 0;
    const uint32_t rmin = wave_reduce_u32<true>(u == umax ? (uint32_t)row : 0xFFFFFFFFu);
    return pivot_key(__uint_as_float(umax - 1u), (int)rmin);
}

__device__ inline void laswp_wave(float *__restrict__ C, int64_t ldc, int64_t nrows, int64_t ncols,
                                  int64_t gap0, int64_t gapw, const int64_t *__restrict__ ipiv,
                                  int64_t k0, int64_t k1, int64_t cbase, int t);

// The multipliers of a pivot column: the entries below the pivot times the
// pivot's reciprocal when the pivot is at least the smallest normal number
// (so that the reciprocal is finite), as LAPACK's sgetf2 and HPL scale the
// column, else divided by the pivot.
__device__ inline bool scale_by_reciprocal(float piv) { return fabsf(piv) >= FLT_MIN; }

typedef float leaf_f4 __attribute__((ext_vector_type(4)));

// Panel row of register slot i of thread t.  Interleaved (VEC false): rows
// t, t + LEAF_THREADS, ...; grouped (VEC true, RPT a multiple of 4): slots
// 4s .. 4s+3 hold the four consecutive rows 4 LEAF_THREADS s + 4t .. + 3, so
// a wavefront moves 1 KB of a column with one 16-byte access per lane
// instead of 256 bytes with one 4-byte access.
template <bool VEC>
__device__ __forceinline__ int leaf_row(int t, int i)
{
    return VEC ? (i >> 2) * (4 * LEAF_THREADS) + 4 * t + (i & 3) : t + i * LEAF_THREADS;
}
template <bool VEC>
__device__ __forceinline__ int leaf_owner(int r)  // the thread that holds panel row r
{
    return VEC ? (r % (4 * LEAF_THREADS)) >> 2 : r % LEAF_THREADS;
}
template <bool VEC>
__device__ __forceinline__ int leaf_slot(int r)  // its register slot
{
    return VEC ? (r / (4 * LEAF_THREADS)) * 4 + (r & 3) : r / LEAF_THREADS;
}
// Slots whose row can lie at or above a panel column j < 8 (every other
// slot's row is LEAF_THREADS or more rows down).
template <bool VEC>
__host__ __device__ constexpr bool leaf_near_top(int i)
{
    return VEC ? i < 4 : i == 0;
}

// Factor the m x w panel P (w <= W, m <= RPT * LEAF_THREADS, leading
// dimension lda; its top-left element is A(row0, row0)).  Thread t holds
// its rows of the panel (leaf_row) in registers; the rows past m hold NaN,
// so that they are never a pivot candidate and need no mask (they are not
// stored).  VEC needs P 16-byte aligned and lda a multiple of 4.  For each column j: the row of largest magnitude at or
// below j (first one on ties) is exchanged with row j across the panel,
// the entries below the diagonal become multipliers, and the outer product
// is subtracted from the remaining columns.  A zero pivot leaves its column
// as it is and records row0 + j + 1 in *info if no earlier zero pivot did.
// ipiv receives global row indices.  With UPD and wl > 0 the panel is the
// right half of a node whose left half (the wl columns left of it) is the
// leaf just factored: wavefront 0 first applies that leaf's interchanges
// (rows row0 - wl .. row0 - 1 with their pivot rows) to the panel's columns
// over the whole matrix height, then the node's solve and update run on the
// panel (below).  One barrier per column: before it,
// every wave posts its own candidate row (its largest key) and folds the
// key into an LDS maximum, and thread j posts row j; after it, every thread
// reads the winning key and takes the pivot row from the wave that owns it.
// The row buffers alternate between even and odd columns and the maximum
// cycles over three slots (one is cleared two columns ahead of its use), so
// a wave that runs ahead never overwrites what a slower one still reads.
template <int RPT, int W, bool UPD, bool VEC>
__global__ __launch_bounds__(LEAF_THREADS) void lu_leaf_kernel(float *__restrict__ P,
                                                              int64_t lda, int m, int w, int wl,
                                                              int64_t *__restrict__ ipiv,
                                                              int64_t row0, int *__restrict__ info)
{
    static_assert(RPT * W <= LEAF_REGS, "panel does not fit the register budget");
    static_assert(LEAF_THREADS % 64 == 0, "waves own whole 64-row groups of a thread row");
    static_assert(!VEC || RPT % 4 == 0, "grouped rows come four at a time");
    static_assert(W <= 8, "rows at or above a panel column lie in the near-top slots");
    __shared__ float wrow[2][LEAF_WAVES][W];   // each wave's candidate row
    __shared__ float jrow[2][W];               // row j before its exchange
    __shared__ unsigned long long gkey[3];     // largest pivot key of the column
    __shared__ float su[W][W];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const float qnan = __int_as_float(0x7fc00000);
    if (t < 3) gkey[t] = 0;
    if (UPD && wl > 0) {
        // the left sibling's interchanges on this panel's columns (global row
        // 0 of the panel's first column is P - row0)
        if (wave == 0) laswp_wave(P - row0, lda, row0 + m, w, w, 0, ipiv, row0 - wl, row0, 0, lane);
        __syncthreads();
    }
    float v[RPT][W];
#pragma unroll
    for (int c = 0; c < W; ++c) {
        const float *pc = P + (int64_t)c * lda;  // uniform column base, 32-bit row offsets
        if (VEC) {
#pragma unroll
            for (int s4 = 0; s4 < RPT / 4; ++s4) {
                const int rb = leaf_row<VEC>(t, 4 * s4);
                leaf_f4 x;
                if (c < w && rb + 4 <= m) {
                    x = *reinterpret_cast<const leaf_f4 *>(pc + rb);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        x[e] = rb + e < m ? (c < w ? pc[rb + e] : 0.0f) : qnan;
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) v[4 * s4 + e][c] = x[e];
            }
        } else {
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const uint32_t r = (uint32_t)leaf_row<VEC>(t, i);
                v[i][c] = r < (uint32_t)m ? (c < w ? pc[r] : 0.0f) : qnan;
            }
        }
    }
    __syncthreads();  // gkey cleared
    if (UPD && wl > 0) {
        // The parent node's update from the left sibling leaf (the wl <= W
        // columns left of the panel, already factored and swapped): U12 = L11^{-1}
        // A12 on the wl rows above the panel (thread c solves column c, terms
        // in the order k = 0, 1, ..., as the triangular leaves take them),
        // then A22 -= A21 U12 on the panel in registers, one column of A21
        // (one rank-1 term) at a time.
        if (t < w) {
            float x[W];
#pragma unroll
            for (int q = 0; q < W; ++q)
                x[q] = q < wl ? P[(int64_t)t * lda + (q - wl)] : 0.0f;
#pragma unroll
            for (int q = 1; q < W; ++q)
                if (q < wl) {
#pragma unroll
                    for (int k = 0; k < q; ++k)
                        x[q] -= P[(int64_t)(k - wl) * lda + (q - wl)] * x[k];
                }
#pragma unroll
            for (int q = 0; q < W; ++q)
                if (q < wl) {
                    P[(int64_t)t * lda + (q - wl)] = x[q];
                    su[q][t] = x[q];
                }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < W; ++q) {
            if (q < wl) {  // uniform
                const float *lq = P + (int64_t)(q - wl) * lda;  // column q of A21
                float a[RPT];
                if (VEC) {
#pragma unroll
                    for (int s4 = 0; s4 < RPT / 4; ++s4) {
                        const int rb = leaf_row<VEC>(t, 4 * s4);
                        leaf_f4 x;
                        if (rb + 4 <= m) {
                            x = *reinterpret_cast<const leaf_f4 *>(lq + rb);
                        } else {
#pragma unroll
                            for (int e = 0; e < 4; ++e) x[e] = rb + e < m ? lq[rb + e] : 0.0f;
                        }
#pragma unroll
                        for (int e = 0; e < 4; ++e) a[4 * s4 + e] = x[e];
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < RPT; ++i) {
                        const uint32_t r = (uint32_t)leaf_row<VEC>(t, i);
                        a[i] = r < (uint32_t)m ? lq[r] : 0.0f;
                    }
                }
#pragma unroll
                for (int i = 0; i < RPT; ++i)
#pragma unroll
                    for (int c = 0; c < W; ++c) v[i][c] -= a[i] * su[q][c];
            }
        }
    }
#pragma unroll
    for (int j = 0; j < W; ++j) {
        if (j >= w) break;
        const int b2 = j & 1, b3 = j % 3;
        // this thread's candidate: its first row at or below j of largest
        // magnitude (NaN never compares greater, rows above j take -1)
        float best = -1.0f;
        int bi = 0;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const float a = (leaf_near_top<VEC>(i) && leaf_row<VEC>(t, i) < j) ? -1.0f
                                                                             : fabsf(v[i][j]);
            if (a > best) {
                best = a;
                bi = i;
            }
        }
        const uint64_t key = wave_pivot_key(best, leaf_row<VEC>(t, bi));
        if (key != 0) {  // uniform
            const int r = (int)(0xFFFFFFFFu - (uint32_t)key);
            if (lane == (leaf_owner<VEC>(r) & 63)) {
                const int ri = leaf_slot<VEC>(r);
#pragma unroll
                for (int i = 0; i < RPT; ++i)
                    if (i == ri) {
#pragma unroll
                        for (int c = 0; c < W; ++c) wrow[b2][wave][c] = v[i][c];
                    }
                atomicMax(&gkey[b3], (unsigned long long)key);
            }
        }
        if (t == leaf_owner<VEC>(j)) {
#pragma unroll
            for (int c = 0; c < W; ++c) jrow[b2][c] = v[leaf_slot<VEC>(j)][c];
        }
        __syncthreads();
        const uint64_t g0 = gkey[b3];
        const uint32_t ghi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(g0 >> 32));
        const uint32_t glo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)g0);
        const uint64_t g = ((uint64_t)ghi << 32) | glo;
        if (t == 0) gkey[(j + 2) % 3] = 0;  // last read before this column's barrier
        const int idx = g == 0 ? -1 : (int)(0xFFFFFFFFu - (uint32_t)g);
        const float pivot_mag = g == 0 ? -1.0f : __uint_as_float((uint32_t)(g >> 32));
        const int p = idx >= 0 ? idx : j;
        const int pt = leaf_owner<VEC>(p), pi = leaf_slot<VEC>(p);
        if (t == 0) ipiv[row0 + j] = row0 + p;
        // the pivot row, the new row j (row j itself when nothing qualifies)
        float u[W];
#pragma unroll
        for (int c = 0; c < W; ++c) u[c] = g != 0 ? wrow[b2][pt >> 6][c] : jrow[b2][c];
        if (p != j) {
            if (t == leaf_owner<VEC>(j)) {
#pragma unroll
                for (int c = 0; c < W; ++c) v[leaf_slot<VEC>(j)][c] = u[c];
            }
            if (t == pt) {
#pragma unroll
                for (int i = 0; i < RPT; ++i)
                    if (i == pi) {
#pragma unroll
                        for (int c = 0; c < W; ++c) v[i][c] = jrow[b2][c];
                    }
            }
        }
        const float piv = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(u[j])));
        if (pivot_mag > 0.0f && piv != 0.0f) {
            float l[RPT];
            if (scale_by_reciprocal(piv)) {
                const float rinv = 1.0f / piv;
#pragma unroll
                for (int i = 0; i < RPT; ++i) l[i] = v[i][j] * rinv;
            } else {
#pragma unroll
                for (int i = 0; i < RPT; ++i) l[i] = v[i][j] / piv;
            }
            // only the near-top slots can hold a row at or above row j
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                if (leaf_near_top<VEC>(i)) {
                    const bool below = leaf_row<VEC>(t, i) > j;
                    v[i][j] = below ? l[i] : v[i][j];
#pragma unroll
                    for (int c = j + 1; c < W; ++c)
                        v[i][c] = below ? v[i][c] - l[i] * u[c] : v[i][c];
                } else {
                    v[i][j] = l[i];
#pragma unroll
                    for (int c = j + 1; c < W; ++c) v[i][c] -= l[i] * u[c];
                }
            }
        } else if (t == 0 && *info == 0) {
            *info = (int)(row0 + j + 1);
        }
    }
#pragma unroll
    for (int c = 0; c < W; ++c) {
        float *pc = P + (int64_t)c * lda;
        if (VEC) {
#pragma unroll
            for (int s4 = 0; s4 < RPT / 4; ++s4) {
                const int rb = leaf_row<VEC>(t, 4 * s4);
                if (c < w && rb + 4 <= m) {
                    leaf_f4 x;
#pragma unroll
                    for (int e = 0; e < 4; ++e) x[e] = v[4 * s4 + e][c];
                    *reinterpret_cast<leaf_f4 *>(pc + rb) = x;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (c < w && rb + e < m) pc[rb + e] = v[4 * s4 + e][c];
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const uint32_t r = (uint32_t)leaf_row<VEC>(t, i);
                if (r < (uint32_t)m && c < w) pc[r] = v[i][c];
            }
        }
    }
}

// The same factorization for panels taller than the register-resident
// kernel takes: the panel stays in memory and every column pass walks it.
__global__ __launch_bounds__(LEAF_THREADS) void lu_leaf_tall_kernel(float *__restrict__ P,
                                                                   int64_t lda, int64_t m, int w,
                                                                   int64_t *__restrict__ ipiv,
                                                                   int64_t row0,
                                                                   int *__restrict__ info)
{
    __shared__ float sbest[LEAF_THREADS];
    __shared__ int64_t sidx[LEAF_THREADS];
    __shared__ float urow[PANEL_LEAF];
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
            if (scale_by_reciprocal(piv)) {
                const float rinv = 1.0f / piv;
                for (int64_t r = j + 1 + t; r < m; r += LEAF_THREADS) col[r] = col[r] * rinv;
            } else {
                for (int64_t r = j + 1 + t; r < m; r += LEAF_THREADS) col[r] = col[r] / piv;
            }
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

// Row interchanges k0..k1-1, in order (row k with row ipiv[k]; an entry
// outside [0, nrows) is skipped), on ncols columns of C (row 0 of the
// matrix, leading dimension ldc).  Column index c is matrix column c below
// gap0 and c + gapw from there on, so that a band of gapw columns is left
// alone.  The interchanges are taken SWAP_BLOCK at a time and each block is
// composed into one permutation of at most 2 * SWAP_BLOCK rows ("slots":
// slot i < nb is row k + i, a row outside the block takes slot nb + i for
// the first i that names it).  Each wavefront composes the permutation with
// lane s tracking slot s, then moves SWAP_COLS_PER_WAVE columns: S lanes
// per column (S = the power of two >= 2 nb), lane s loading the row of
// slot s, receiving the value its slot ends up with from the lane that
// loaded it, and storing it -- one load and one store per moved element,
// no chain of dependent swaps.
template <int S>
__device__ inline void laswp_move(float *__restrict__ C, int64_t ldc, int64_t ncols, int64_t gap0,
                                  int64_t gapw, int64_t cbase, int lane, int64_t row, int content)
{
    constexpr int CPP = 64 / S;                       // columns per pass
    constexpr int PASSES = SWAP_COLS_PER_WAVE / CPP;
    const int s = lane & (S - 1), g = lane / S;
    const int64_t rs = __shfl(row, s);
    const int fs = __shfl(content, s);
    const bool moved = rs >= 0 && fs != s;
    float val[PASSES];
    float *colp[PASSES];
#pragma unroll
    for (int q = 0; q < PASSES; ++q) {
        int64_t c = cbase + q * CPP + g;
        const bool act = moved && c < ncols;
        if (c >= gap0) c += gapw;
        colp[q] = act ? C + c * ldc : nullptr;
        val[q] = act ? colp[q][rs] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < PASSES; ++q) {
        const float nv = __shfl(val[q], g * S + fs);
        if (colp[q]) colp[q][rs] = nv;
    }
}

// One wavefront's share of the interchanges: columns cbase ..
// cbase + SWAP_COLS_PER_WAVE - 1 (those below ncols) of C, lane t.
__device__ inline void laswp_wave(float *__restrict__ C, int64_t ldc, int64_t nrows, int64_t ncols,
                                  int64_t gap0, int64_t gapw, const int64_t *__restrict__ ipiv,
                                  int64_t k0, int64_t k1, int64_t cbase, int t)
{
    for (int64_t kb = k0; kb < k1; kb += SWAP_BLOCK) {
        const int nb = (int)(k1 - kb < SWAP_BLOCK ? k1 - kb : SWAP_BLOCK);
        int64_t p = -1;
        if (t < nb) {
            p = ipiv[kb + t];
            if (p < 0 || p >= nrows) p = kb + t;
        }
        // the composition reads uniform lanes: scalar readlanes, not the
        // LDS-routed lane shuffles (it is the dependent chain of a launch)
        int first = t;
        for (int i = 0; i < nb; ++i) {
            const int64_t q = (int64_t)readlane64((uint64_t)p, i);
            if (i < t && q == p && first == t) first = i;
        }
        int pslot = -1;
        if (t < nb) pslot = (p >= kb && p < kb + nb) ? (int)(p - kb) : nb + first;
        // row of slot t
        const int src = t >= nb ? t - nb : 0;
        const int64_t q = __shfl(p, src);
        const int qs = __shfl(pslot, src);
        int64_t row = -1;
        if (t < nb) row = kb + t;
        else if (t < 2 * nb && qs == t) row = q;
        // compose: content = slot whose original value ends in slot t
        int content = t;
        for (int i = 0; i < nb; ++i) {
            const int b = __builtin_amdgcn_readlane(pslot, i);
            const int ca = __builtin_amdgcn_readlane(content, i);
            const int cb = __builtin_amdgcn_readlane(content, b);
            if (t == i) content = cb;
            else if (t == b) content = ca;
        }
        if (nb <= 8)
            laswp_move<16>(C, ldc, ncols, gap0, gapw, cbase, t, row, content);
        else if (nb <= 16)
            laswp_move<32>(C, ldc, ncols, gap0, gapw, cbase, t, row, content);
        else
            laswp_move<64>(C, ldc, ncols, gap0, gapw, cbase, t, row, content);
    }
}

// The interchanges on the columns of the first main_blocks workgroups
// (laswp_wave's arguments); the workgroups after them take the band of
// bandw columns at band0, with the interchanges bk0 .. k1-1 only.
__global__ __launch_bounds__(SWAP_THREADS) void laswp_kernel(
    float *__restrict__ C, int64_t ldc, int64_t nrows, int64_t ncols, int64_t gap0, int64_t gapw,
    const int64_t *__restrict__ ipiv, int64_t k0, int64_t k1, int64_t main_blocks, int64_t band0,
    int64_t bandw, int64_t bk0)
{
    const int t = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if ((int64_t)blockIdx.x < main_blocks) {
        const int64_t cbase =
            ((int64_t)blockIdx.x * (SWAP_THREADS / 64) + wave) * SWAP_COLS_PER_WAVE;
        if (cbase >= ncols) return;  // whole wavefront past the last column
        laswp_wave(C, ldc, nrows, ncols, gap0, gapw, ipiv, k0, k1, cbase, t);
    } else {
        const int64_t cbase =
            (((int64_t)blockIdx.x - main_blocks) * (SWAP_THREADS / 64) + wave) * SWAP_COLS_PER_WAVE;
        if (cbase >= bandw) return;
        laswp_wave(C + band0 * ldc, ldc, nrows, bandw, bandw, 0, ipiv, bk0, k1, cbase, t);
    }
}

// The interchanges k0 .. k1-1 on column blockIdx.x of C (nrows <=
// LASWP_LDS_ROWS rows, k1 - k0 <= nrows), for the solve's few right-hand
// sides: the column and the pivot list are staged in LDS, one lane applies
// the interchanges one by one in order (each an LDS round trip, with the
// pivot reads independent of the column), and the column is written back.
// Entries outside [0, nrows) are skipped.
__global__ __launch_bounds__(SWAP_THREADS) void laswp_lds_kernel(float *__restrict__ C,
                                                                int64_t ldc, int nrows,
                                                                const int64_t *__restrict__ ipiv,
                                                                int64_t k0, int64_t k1)
{
    __shared__ float col[LASWP_LDS_ROWS];
    __shared__ int piv[LASWP_LDS_ROWS];
    float *c = C + (int64_t)blockIdx.x * ldc;
    for (int i = threadIdx.x; i < nrows; i += SWAP_THREADS) col[i] = c[i];
    for (int64_t k = k0 + threadIdx.x; k < k1; k += SWAP_THREADS) {
        const int64_t p = ipiv[k];
        piv[k - k0] = (int)((p < 0 || p >= nrows) ? k : p);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int n = (int)(k1 - k0), base = (int)k0;
        for (int i = 0; i < n; ++i) {
            const int r = base + i, p = piv[i];
            const float a = col[r], b = col[p];
            col[r] = b;
            col[p] = a;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nrows; i += SWAP_THREADS) c[i] = col[i];
}

// x of lane q (a constant after unrolling) in every lane, through a scalar
// register.
__device__ inline float lane_value(float x, int q)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), q));
}

// B (n x ncols, n <= N) := T^{-1} B for T the n x n lower unit (UPPER
// false) or upper (UPPER true) triangle at T.  N lanes per column (lane i
// holds row i of T and x_i), 64 / N columns per wavefront; x_k reaches the
// other rows once it is final, by a lane shuffle (a scalar broadcast when
// the wavefront holds one column).  The lower solve takes
// the terms of x_i in the order k = 0, 1, ..., i-1; the upper one in the
// order k = n-1, ..., i+1, then divides by the diagonal.
// With SWAP the workgroup first applies the interchanges k0..k1-1 to its
// columns of B over the whole matrix height (B's row 0 is matrix row row0;
// nrows rows in all), one wavefront per SWAP_COLS_PER_WAVE columns, then
// solves: the left sibling leaf's interchanges on the right half's columns,
// where the node's halves are leaves too tall to fuse its update.
template <bool UPPER, int N, bool SWAP>
__global__ __launch_bounds__(256) void trsm_leaf_kernel(const float *__restrict__ T, int64_t ldt,
                                                       float *__restrict__ B, int64_t ldb, int n,
                                                       int64_t ncols,
                                                       const int64_t *__restrict__ ipiv,
                                                       int64_t nrows, int64_t row0, int64_t k0,
                                                       int64_t k1)
{
    constexpr int CPW = 64 / N;
    if (SWAP) {
        constexpr int CPB = 4 * CPW;  // columns of a workgroup
        const int64_t c0 = (int64_t)blockIdx.x * CPB;
        const int64_t bc = ncols - c0 < CPB ? ncols - c0 : CPB;
        const int64_t cb = (int64_t)(threadIdx.x >> 6) * SWAP_COLS_PER_WAVE;
        if (cb < bc)  // wavefront-uniform
            laswp_wave(B - row0 + c0 * ldb, ldb, nrows, bc, bc, 0, ipiv, k0, k1, cb,
                       threadIdx.x & 63);
        __syncthreads();
    }
    const int lane = threadIdx.x & 63, i = lane % N, g = lane / N;
    const int64_t c = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * CPW + g;
    const bool act = c < ncols && i < n;
    float trow[N];
#pragma unroll
    for (int k = 0; k < N; ++k) trow[k] = (i < n && k < n) ? T[i + (int64_t)k * ldt] : 0.0f;
    float x = act ? B[c * ldb + i] : 0.0f;
    if (!UPPER) {
#pragma unroll
        for (int k = 0; k < N - 1; ++k) {
            const float xk = N == 64 ? lane_value(x, k) : __shfl(x, g * N + k);
            if (i > k) x -= trow[k] * xk;
        }
    } else {
#pragma unroll
        for (int k = N - 1; k >= 0; --k) {
            if (i == k && k < n) x = x / trow[k];
            const float xk = N == 64 ? lane_value(x, k) : __shfl(x, g * N + k);
            if (i < k) x -= trow[k] * xk;
        }
    }
    if (act) B[c * ldb + i] = x;
}

// B (n x 1, n <= TRSV_ROWS, column blockIdx.x of B) := T^{-1} B for T the
// lower unit (UPPER false) or upper (UPPER true) triangle, one workgroup per
// right-hand side: wave w holds rows 64w .. 64w+63 (lane = row) in a
// register, and the 64-row blocks are taken in the solve's order (lower:
// first to last, upper: last to first).  The wave that owns block k
// finishes its rows, each final value broadcast from its lane through a
// scalar register (the terms in the triangular leaves' order), and posts
// them to LDS; after one barrier every wave whose rows
// still depend on block k subtracts its contribution, with the entries of T
// it needs loaded before the barrier.  No row reads another row's value
// before that row is final, so the sums are those of substitution by
// blocks.
template <bool UPPER>
__global__ __launch_bounds__(TRSV_ROWS) void trsv_block_kernel(const float *__restrict__ T,
                                                              int64_t ldt, float *__restrict__ B,
                                                              int64_t ldb, int n)
{
    __shared__ float xs[TRSV_ROWS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = wave * 64 + lane;
    const bool live = r < n;
    float *b = B + (int64_t)blockIdx.x * ldb;
    float x = live ? b[r] : 0.0f;
    const int nb = (n + 63) / 64;
    for (int step = 0; step < nb; ++step) {
        const int k = UPPER ? nb - 1 - step : step;
        const bool needs = UPPER ? wave <= k : wave >= k;  // rows that depend on block k
        float tv[64];
        const float *tc = T + (int64_t)k * 64 * ldt;      // column 64k of T
#pragma unroll
        for (int q = 0; q < 64; ++q)
            tv[q] = (needs && live && k * 64 + q < n) ? tc[(int64_t)q * ldt + r] : 0.0f;
        if (wave == k) {
            if (!UPPER) {
#pragma unroll
                for (int q = 0; q < 63; ++q) {
                    const float xq = lane_value(x, q);
                    if (lane > q) x -= tv[q] * xq;
                }
            } else {
                // Each row's quotient by its diagonal entry: where every
                // diagonal entry of the block is a normal number, through
                // its reciprocal (computed before the dependent chain) and
                // one correction step, q0 = x d', x = q0 + (x - q0 d) d'
                // with both updates fused (correctly rounded for a correctly
                // rounded d', so exact wherever the quotient is
                // representable); otherwise by division, so that a zero or
                // non-finite diagonal gives what x / d gives.
                float dg = 1.0f;
#pragma unroll
                for (int q = 0; q < 64; ++q) dg = q == lane ? tv[q] : dg;
                const bool normal = !live || (fabsf(dg) >= FLT_MIN && fabsf(dg) <= FLT_MAX);
                if (__all(normal)) {
                    const float rdg = 1.0f / dg;
#pragma unroll
                    for (int q = 63; q >= 0; --q) {
                        if (lane == q && live) {
                            const float q0 = x * rdg;
                            x = fmaf(fmaf(-q0, dg, x), rdg, q0);
                        }
                        const float xq = lane_value(x, q);
                        if (lane < q) x -= tv[q] * xq;
                    }
                } else {
#pragma unroll
                    for (int q = 63; q >= 0; --q) {
                        if (lane == q && live) x = x / tv[q];
                        const float xq = lane_value(x, q);
                        if (lane < q) x -= tv[q] * xq;
                    }
                }
            }
            xs[r] = x;
        }
        __syncthreads();
        if (needs && wave != k) {
            if (!UPPER) {
#pragma unroll
                for (int q = 0; q < 64; ++q) x -= tv[q] * xs[k * 64 + q];
            } else {
#pragma unroll
                for (int q = 63; q >= 0; --q) x -= tv[q] * xs[k * 64 + q];
            }
        }
    }
    if (live) b[r] = x;
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

// Interchanges k0..k1-1 on ncols columns of C (all rows of the matrix),
// skipping the band of gapw columns at gap0; with bandw > 0 the same launch
// also applies the interchanges bk0..k1-1 to the bandw columns at band0.
int laswp(const Lu &c, float *C, int64_t ldc, int64_t ncols, int64_t gap0, int64_t gapw,
          int64_t k0, int64_t k1, int64_t band0 = 0, int64_t bandw = 0, int64_t bk0 = 0)
{
    constexpr int cols_per_block = SWAP_THREADS / 64 * SWAP_COLS_PER_WAVE;
    const int64_t main_blocks = k1 > k0 ? (ncols + cols_per_block - 1) / cols_per_block : 0;
    const int64_t band_blocks = k1 > bk0 ? (bandw + cols_per_block - 1) / cols_per_block : 0;
    if (main_blocks + band_blocks <= 0) return 0;
    hipLaunchKernelGGL(laswp_kernel, dim3((unsigned)(main_blocks + band_blocks)),
                       dim3(SWAP_THREADS), 0, c.s, C, ldc, c.n, ncols, gap0, gapw, c.ipiv, k0,
                       k1, main_blocks, band0, bandw, bk0);
    return check(hipGetLastError());
}

// k1 > k0: the interchanges k0..k1-1 go to B's columns first (B's row 0 is
// matrix row row0).
template <bool UPPER, int N>
void launch_trsm_leaf_n(const Lu &c, const float *T, int64_t ldt, float *B, int64_t ldb, int n,
                        int64_t ncols, int64_t row0, int64_t k0, int64_t k1)
{
    constexpr int cols_per_block = 4 * (64 / N);
    const dim3 grid((unsigned)((ncols + cols_per_block - 1) / cols_per_block)), block(256);
    if (k1 > k0)
        hipLaunchKernelGGL((trsm_leaf_kernel<UPPER, N, true>), grid, block, 0, c.s, T, ldt, B,
                           ldb, n, ncols, c.ipiv, c.n, row0, k0, k1);
    else
        hipLaunchKernelGGL((trsm_leaf_kernel<UPPER, N, false>), grid, block, 0, c.s, T, ldt, B,
                           ldb, n, ncols, c.ipiv, c.n, row0, k0, k1);
}

template <bool UPPER>
void launch_trsm_leaf(const Lu &c, const float *T, int64_t ldt, float *B, int64_t ldb, int n,
                      int64_t ncols, int64_t row0 = 0, int64_t k0 = 0, int64_t k1 = 0)
{
    if (n <= 8)
        launch_trsm_leaf_n<UPPER, 8>(c, T, ldt, B, ldb, n, ncols, row0, k0, k1);
    else if (n <= 16)
        launch_trsm_leaf_n<UPPER, 16>(c, T, ldt, B, ldb, n, ncols, row0, k0, k1);
    else if (n <= 32)
        launch_trsm_leaf_n<UPPER, 32>(c, T, ldt, B, ldb, n, ncols, row0, k0, k1);
    else
        launch_trsm_leaf_n<UPPER, LEAF>(c, T, ldt, B, ldb, n, ncols, row0, k0, k1);
}

template <bool UPPER>
void launch_trsv_block(const Lu &c, const float *T, int64_t ldt, float *B, int64_t ldb, int n,
                       int64_t ncols)
{
    hipLaunchKernelGGL((trsv_block_kernel<UPPER>), dim3((unsigned)ncols), dim3(TRSV_ROWS), 0,
                       c.s, T, ldt, B, ldb, n);
}

// B (n x ncols) := T^{-1} B, T lower unit or upper n x n, recursively: the
// off-diagonal block goes through sgemm.  few_rhs (ncols <= TRSV_MAX_RHS)
// ends the recursion at TRSV_ROWS rows with the one-workgroup solve.
int trsm(const Lu &c, bool upper, const float *T, int64_t ldt, float *B, int64_t ldb, int64_t n,
         int64_t ncols, bool few_rhs = false)
{
    if (n == 0 || ncols == 0) return 0;
    if (few_rhs && n <= TRSV_ROWS && ncols <= TRSV_MAX_RHS) {
        if (upper)
            launch_trsv_block<true>(c, T, ldt, B, ldb, (int)n, ncols);
        else
            launch_trsv_block<false>(c, T, ldt, B, ldb, (int)n, ncols);
        return check(hipGetLastError());
    }
    if (n <= LEAF) {
        if (upper)
            launch_trsm_leaf<true>(c, T, ldt, B, ldb, (int)n, ncols);
        else
            launch_trsm_leaf<false>(c, T, ldt, B, ldb, (int)n, ncols);
        return check(hipGetLastError());
    }
    const int64_t h = (n / 2 + LEAF - 1) / LEAF * LEAF;
    int rc;
    if (!upper) {
        if ((rc = trsm(c, false, T, ldt, B, ldb, h, ncols, few_rhs))) return rc;
        if ((rc = gemm(c, n - h, ncols, h, T + h, ldt, B, ldb, B + h, ldb))) return rc;
        return trsm(c, false, T + h + h * ldt, ldt, B + h, ldb, n - h, ncols, few_rhs);
    }
    if ((rc = trsm(c, true, T + h + h * ldt, ldt, B + h, ldb, n - h, ncols, few_rhs))) return rc;
    if ((rc = gemm(c, h, ncols, n - h, T + h * ldt, ldt, B + h, ldb, B, ldb))) return rc;
    return trsm(c, true, T, ldt, B, ldb, h, ncols, few_rhs);
}

// Rows per thread of the register-resident leaf for an m-row panel (a
// power of two), or 0 when the panel is taller than it takes.
int leaf_rpt(int64_t m)
{
    for (int rpt = 1; rpt <= 16; rpt *= 2)
        if (m <= (int64_t)rpt * LEAF_THREADS) return rpt;
    return 0;
}

// Widest leaf panel whose m x w values fit LEAF_REGS registers per thread.
int64_t leaf_width(int64_t m)
{
    const int rpt = leaf_rpt(m);
    if (rpt == 0) return PANEL_LEAF;
    return LEAF_REGS / rpt < PANEL_LEAF ? LEAF_REGS / rpt : PANEL_LEAF;
}

// Factor the leaf panel at P (m x w, top-left element A(j0, j0)); wl > 0
// (at most the leaf width) first applies the parent node's solve and update
// from the wl columns left of it (register kernels of up to LEAF_UPD_RPT
// rows per thread, whose registers leave room for it).
int leaf(const Lu &c, float *P, int64_t m, int w, int64_t j0, int wl)
{
    const dim3 grid(1), block(LEAF_THREADS);
#define MISGEMM_LEAF(R, W, U, V)                                                           \
    hipLaunchKernelGGL((lu_leaf_kernel<R, W, U, V>), grid, block, 0, c.s, P, c.lda, (int)m, w, \
                       wl, c.ipiv, j0, c.info)
    const int rpt = leaf_rpt(m);
    if (wl > 0 && (rpt == 0 || rpt > LEAF_UPD_RPT)) return MISGEMM_E_BAD_CONFIG;
    // four consecutive rows per 16-byte access where the panel's columns
    // are 16-byte aligned and a thread holds 8 or more rows (at 4 rows per
    // thread the grouped leaf measured slower)
    const bool vec = c.lda % 4 == 0 && (reinterpret_cast<uintptr_t>(P) & 15) == 0;
    switch (rpt) {
    case 1: if (wl > 0) MISGEMM_LEAF(1, PANEL_LEAF, true, false); else MISGEMM_LEAF(1, PANEL_LEAF, false, false); break;
    case 2: if (wl > 0) MISGEMM_LEAF(2, PANEL_LEAF, true, false); else MISGEMM_LEAF(2, PANEL_LEAF, false, false); break;
    case 4: if (wl > 0) MISGEMM_LEAF(4, PANEL_LEAF, true, false); else MISGEMM_LEAF(4, PANEL_LEAF, false, false); break;
    case 8:
        if (vec) { if (wl > 0) MISGEMM_LEAF(8, PANEL_LEAF, true, true); else MISGEMM_LEAF(8, PANEL_LEAF, false, true); }
        else { if (wl > 0) MISGEMM_LEAF(8, PANEL_LEAF, true, false); else MISGEMM_LEAF(8, PANEL_LEAF, false, false); }
        break;
    case 16:
        if (vec) { if (wl > 0) MISGEMM_LEAF(16, LEAF_REGS / 16, true, true); else MISGEMM_LEAF(16, LEAF_REGS / 16, false, true); }
        else { if (wl > 0) MISGEMM_LEAF(16, LEAF_REGS / 16, true, false); else MISGEMM_LEAF(16, LEAF_REGS / 16, false, false); }
        break;
    default:
        hipLaunchKernelGGL(lu_leaf_tall_kernel, grid, block, 0, c.s, P, c.lda, m, w, c.ipiv, j0,
                           c.info);
        break;
    }
#undef MISGEMM_LEAF
    return check(hipGetLastError());
}

// Factor columns j0 .. j0+w-1 over rows j0 .. n-1.
int getrf(const Lu &c, int64_t j0, int64_t w)
{
    const int64_t m = c.n - j0;
    float *P = c.A + j0 + j0 * c.lda;
    const int64_t lw = leaf_width(m);
    int rc;
    if (w <= lw) {
        if ((rc = leaf(c, P, m, (int)w, j0, 0))) return rc;
        // this leaf's interchanges on every other column
        return laswp(c, c.A, c.lda, c.n - w, j0, w, j0, j0 + w);
    }
    const int64_t w1 = (w / 2 + lw - 1) / lw * lw, w2 = w - w1, m2 = m - w1;
    const int rpt2 = leaf_rpt(m2);
    if (w <= 2 * lw && rpt2 > 0 && rpt2 <= LEAF_UPD_RPT && w1 <= leaf_width(m2) &&
        w2 <= leaf_width(m2)) {
        // both halves are leaves: the right one applies the left one's
        // interchanges to its own columns and this node's solve and update
        // itself (no separate interchange, triangular-solve and sgemm
        // launches); then one launch takes the node's interchanges to every
        // column outside it and the right half's to the left half
        if ((rc = leaf(c, P, m, (int)w1, j0, 0))) return rc;
        if ((rc = leaf(c, P + w1 + w1 * c.lda, m2, (int)w2, j0 + w1, (int)w1))) return rc;
        return laswp(c, c.A, c.lda, c.n - w, j0, w, j0, j0 + w, j0, w1, j0 + w1);
    }
    if (w1 <= lw && w2 <= leaf_width(m2) && w1 <= LEAF) {
        // both halves are leaves, too tall for the right one to take the
        // node's update (over LEAF_UPD_RPT * LEAF_THREADS rows, where the
        // in-memory leaf factors them): the triangular solve applies the left leaf's
        // interchanges to the right half's columns before solving, and one
        // launch after the pair takes the node's interchanges to every
        // other column and the right leaf's to the left one (as above)
        if ((rc = leaf(c, P, m, (int)w1, j0, 0))) return rc;
        launch_trsm_leaf<false>(c, P, c.lda, P + w1 * c.lda, c.lda, (int)w1, w2, j0, j0,
                                j0 + w1);
        if ((rc = check(hipGetLastError()))) return rc;
        if ((rc = gemm(c, m - w1, w2, w1, P + w1, c.lda, P + w1 * c.lda, c.lda,
                       P + w1 + w1 * c.lda, c.lda)))
            return rc;
        if ((rc = leaf(c, P + w1 + w1 * c.lda, m2, (int)w2, j0 + w1, 0))) return rc;
        return laswp(c, c.A, c.lda, c.n - w, j0, w, j0, j0 + w, j0, w1, j0 + w1);
    }
    if ((rc = getrf(c, j0, w1))) return rc;
    if ((rc = trsm(c, false, P, c.lda, P + w1 * c.lda, c.lda, w1, w2))) return rc;
    if ((rc = gemm(c, m - w1, w2, w1, P + w1, c.lda, P + w1 * c.lda, c.lda,
                   P + w1 + w1 * c.lda, c.lda)))
        return rc;
    return getrf(c, j0 + w1, w2);
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
    const bool few = nrhs <= TRSV_MAX_RHS;
    int rc = 0;
    if (few && n <= LASWP_LDS_ROWS) {
        hipLaunchKernelGGL(laswp_lds_kernel, dim3((unsigned)nrhs), dim3(SWAP_THREADS), 0, c.s, B,
                           ldb, (int)n, ipiv, (int64_t)0, n);
        rc = check(hipGetLastError());
    } else {
        rc = laswp(c, B, ldb, nrhs, nrhs, 0, 0, n);
    }
    if (rc == 0) rc = trsm(c, false, A, lda, B, ldb, n, nrhs, few);
    if (rc == 0) rc = trsm(c, true, A, lda, B, ldb, n, nrhs, few);
    return rc;
}

}  // extern "C"
