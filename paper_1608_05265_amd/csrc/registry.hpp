// Kernel entry points and the table of compiled tile configurations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/misgemm.h"
#include "gemm_rtile.hpp"
#include "gemm_tile.hpp"
#include "packed_x3.hpp"

namespace misgemm {

// One problem of a batch as the persistent kernel reads it.
struct ProbDev {
    GemmArgs g;
    int32_t ta, tb;
    int64_t tiles_m, tiles_n;
};

// One tile of a batch: problem index and tile coordinates.
struct TileDev {
    int32_t prob;
    int32_t tm;
    int32_t tn;
    int32_t pad;
};

// Partition of a batch's tile list over the XCDs: the workgroups of XCD x
// (blockIdx % nx == x, the hardware hands workgroups to the XCDs in turn)
// run tiles[off[x] .. off[x+1]).  nx is 1 (one shared list) or MAX_XCD.
constexpr int MAX_XCD = 8;
struct BatchSplit {
    int64_t off[MAX_XCD + 1];
    int32_t nx;
    int32_t pad;
};

typedef hipError_t (*launch_fn)(const GemmArgs &g, int group_m, hipStream_t s);
typedef hipError_t (*batch_launch_fn)(const ProbDev *probs, const TileDev *tiles,
                                      const BatchSplit &split, int grid, hipStream_t s);
typedef int (*occupancy_fn)();
typedef hipError_t (*packed_launch_fn)(const PackedArgs &p, int group_m, hipStream_t s);
// Persistent kernel over the tiles of a batch whose operands were packed
// (one PackedArgs per problem).
typedef hipError_t (*packed_batch_fn)(const PackedArgs *probs, const TileDev *tiles,
                                      const BatchSplit &split, int grid, hipStream_t s);

struct ConfigEntry {
    misgemm_config_desc desc;
    launch_fn launch[2][2];    // [transa][transb]; NULL for packed configs
    launch_fn splitk[2][2];    // split-K variant (g.splits > 1 set); NULL when not compiled
    batch_launch_fn batch;     // NULL when no persistent variant is compiled
    occupancy_fn batch_occupancy;
    packed_launch_fn packed;   // tile kernel on packed panels (packed configs only)
    packed_batch_fn packed_batch;  // persistent variant of it (NULL when not compiled)
};

// A batched (persistent) variant of either kind is compiled.
inline bool has_batch(const ConfigEntry &e) { return e.batch != nullptr || e.packed_batch != nullptr; }

// Default number of tile-rows walked together (see tile_coords).
constexpr int GROUP_M_DEFAULT = 8;

template <class TILE, class SH>
__global__ __launch_bounds__(SH::NT, SH::OCC) void sgemm_kernel(GemmArgs g, int64_t tiles_m,
                                                          int64_t tiles_n, int group_m)
{
    __shared__ __attribute__((aligned(16))) char smem[TILE::LDS_BYTES];
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    int64_t tm, tn;
    tile_coords(t, tiles_m, tiles_n, group_m, tm, tn);
    TILE::run(g, tm * SH::BM, tn * SH::BN, smem);
}

template <class TILE, class SH>
hipError_t launch_tile_kernel(const GemmArgs &g, int group_m, hipStream_t s)
{
    const int64_t tm = (g.m + SH::BM - 1) / SH::BM, tn = (g.n + SH::BN - 1) / SH::BN;
    hipLaunchKernelGGL((sgemm_kernel<TILE, SH>), dim3((unsigned)(tm * tn)), dim3(SH::NT), 0, s,
                       g, tm, tn, group_m);
    return hipGetLastError();
}

// Split-K, first kernel: workgroup b (after the XCD remap) computes split
// b % splits of tile b / splits over the K range [s*kblk, min(k, (s+1)*kblk)),
// kblk a whole number of BK blocks, and stores its raw partial tile.
__host__ __device__ inline int64_t splitk_kblk(int64_t k, int bk, int splits)
{
    const int64_t kt = (k + bk - 1) / bk;
    return (kt + splits - 1) / splits * bk;
}

template <class TILE, class SH, bool TA, bool TB>
__global__ __launch_bounds__(SH::NT, SH::OCC) void splitk_kernel(GemmArgs g, int64_t tiles_m,
                                                                 int64_t tiles_n, int group_m)
{
    __shared__ __attribute__((aligned(16))) char smem[TILE::LDS_BYTES];
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t tile = t / g.splits;
    const int s = (int)(t % g.splits);
    int64_t tm, tn;
    tile_coords(tile, tiles_m, tiles_n, group_m, tm, tn);
    const int64_t kblk = splitk_kblk(g.k, SH::BK, g.splits);
    const int64_t k0 = s * kblk;
    GemmArgs gs = g;
    gs.k = g.k - k0 < kblk ? g.k - k0 : kblk;
    gs.A = TA ? g.A + k0 : g.A + k0 * g.lda;   // op(A)(i, k0 + p)
    gs.B = TB ? g.B + k0 * g.ldb : g.B + k0;   // op(B)(k0 + p, j)
    gs.tile = tile;
    gs.split = s;
    TILE::template run<true>(gs, tm * SH::BM, tn * SH::BN, smem);
}

// Split-K, second kernel: one workgroup per tile, threads laid out as in the
// tile kernel (so each thread owns the same accumulator entries), adds the
// partials of splits 0, 1, ... in that order and applies alpha/beta.
template <class SH>
__global__ __launch_bounds__(SH::NT) void splitk_reduce_kernel(GemmArgs g, int64_t tiles_m,
                                                               int64_t tiles_n, int group_m)
{
    constexpr int RM = SH::RM, RN = SH::RN;
    const int64_t tile = blockIdx.x;
    int64_t tm, tn;
    tile_coords(tile, tiles_m, tiles_n, group_m, tm, tn);
    const int tid = threadIdx.x, wave = tid >> 6;
    const int wm = wave % SH::NWM, wn = wave / SH::NWM;
    const floatx4 *part = reinterpret_cast<const floatx4 *>(g.part);
    floatx16 acc[RM][RN];
#pragma unroll
    for (int i = 0; i < RM; ++i)
#pragma unroll
        for (int j = 0; j < RN; ++j)
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4) {
                const int q = (i * RN + j) * 4 + q4;
                floatx4 sum = part[partial_index<RM, RN>(tile, g.splits, 0, q, tid, SH::NT)];
                for (int s = 1; s < g.splits; ++s) {
                    const floatx4 v = part[partial_index<RM, RN>(tile, g.splits, s, q, tid, SH::NT)];
#pragma unroll
                    for (int e = 0; e < 4; ++e) sum[e] += v[e];
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[i][j][q4 * 4 + e] = sum[e];
            }
    epilogue<RM, RN>(g, acc, tm * SH::BM + wm * SH::WM, tn * SH::BN + wn * SH::WN, tid & 63);
}

// g.splits >= 2 with every split's K range non-empty (the host sets splits =
// ceil(ktiles / ceil(ktiles / requested))), g.part sized for splits * tiles
// partial tiles.  Two launches on stream s.
template <class TILE, class SH, bool TA, bool TB>
hipError_t launch_splitk_kernel(const GemmArgs &g, int group_m, hipStream_t s)
{
    const int64_t tm = (g.m + SH::BM - 1) / SH::BM, tn = (g.n + SH::BN - 1) / SH::BN;
    hipLaunchKernelGGL((splitk_kernel<TILE, SH, TA, TB>), dim3((unsigned)(tm * tn * g.splits)),
                       dim3(SH::NT), 0, s, g, tm, tn, group_m);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((splitk_reduce_kernel<SH>), dim3((unsigned)(tm * tn)), dim3(SH::NT), 0, s,
                       g, tm, tn, group_m);
    return hipGetLastError();
}

template <int A, int B>
struct MaxI { static constexpr int value = A > B ? A : B; };

// Persistent kernel over a list of tiles of many problems.  Workgroup w
// takes tiles w, w + grid, w + 2*grid, ... of a list sorted by decreasing
// work, so the longest tiles start first.
template <template <class, bool, bool> class TILE, class SH>
__global__ __launch_bounds__(SH::NT, SH::OCC) void batch_kernel(const ProbDev *__restrict__ probs,
                                                          const TileDev *__restrict__ tiles,
                                                          BatchSplit split)
{
    constexpr int L0 = TILE<SH, false, false>::LDS_BYTES, L1 = TILE<SH, false, true>::LDS_BYTES;
    constexpr int L2 = TILE<SH, true, false>::LDS_BYTES, L3 = TILE<SH, true, true>::LDS_BYTES;
    __shared__ __attribute__((aligned(16)))
    char smem[MaxI<MaxI<L0, L1>::value, MaxI<L2, L3>::value>::value];
    // The grid is a multiple of nx: every XCD has gridDim.x / nx slots, and
    // slot s of XCD x runs tiles off[x] + s, off[x] + s + slots, ...
    const int x = (int)(blockIdx.x % (unsigned)split.nx);
    const int64_t slot = blockIdx.x / (unsigned)split.nx, slots = gridDim.x / (unsigned)split.nx;
    const int64_t end = split.off[x + 1];
    for (int64_t t = split.off[x] + slot; t < end; t += slots) {
        const TileDev td = tiles[t];
        const ProbDev &p = probs[td.prob];
        const GemmArgs g = p.g;
        const int64_t m0 = (int64_t)td.tm * SH::BM, n0 = (int64_t)td.tn * SH::BN;
        const int sel = p.ta * 2 + p.tb;
        if (sel == 0) TILE<SH, false, false>::run(g, m0, n0, smem);
        else if (sel == 1) TILE<SH, false, true>::run(g, m0, n0, smem);
        else if (sel == 2) TILE<SH, true, false>::run(g, m0, n0, smem);
        else TILE<SH, true, true>::run(g, m0, n0, smem);
        __syncthreads();
    }
}

template <template <class, bool, bool> class TILE, class SH>
hipError_t launch_batch_kernel(const ProbDev *probs, const TileDev *tiles, const BatchSplit &split,
                               int grid, hipStream_t s)
{
    hipLaunchKernelGGL((batch_kernel<TILE, SH>), dim3(grid), dim3(SH::NT), 0, s, probs, tiles,
                       split);
    return hipGetLastError();
}

template <template <class, bool, bool> class TILE, class SH>
int batch_occupancy()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_kernel<TILE, SH>, SH::NT, 0) !=
        hipSuccess)
        return 1;
    return blocks > 0 ? blocks : 1;
}

// Registration hooks, one per translation unit.
void register_f32(std::vector<ConfigEntry> &out);
void register_x3(std::vector<ConfigEntry> &out);
void register_x3k(std::vector<ConfigEntry> &out);

// Pack op(X) (rows x k, KC: k contiguous) into split panels (packed_x3.hpp).
hipError_t launch_pack(const float *X, int64_t ld, bool kc, int64_t rows, int64_t k, int vec,
                       __bf16 *out, hipStream_t s);
// Pack every operand of a batch in one launch: jobs sorted by first_block,
// `blocks` = the blocks of all jobs.
hipError_t launch_pack_batch(const PackJob *jobs, int njobs, int64_t blocks, hipStream_t s);

// Host helpers shared by the entry points.
hipError_t launch_scale(float beta, float *C, int64_t m, int64_t n, int64_t ldc, hipStream_t s);
hipError_t launch_split(const float *x, int64_t count, uint16_t *parts, hipStream_t s);

}  // namespace misgemm
