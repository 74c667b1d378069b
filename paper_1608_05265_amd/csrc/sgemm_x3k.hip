// Packed split-precision configurations: operands split once into panels
// (pack_x3_kernel), then one tile kernel for every transpose pair.
#include <string.h>

#include "registry.hpp"

namespace misgemm {

template <class SH>
__global__ __launch_bounds__(SH::NT, SH::OCC) void packed_kernel(PackedArgs p, int64_t tiles_m,
                                                           int64_t tiles_n, int group_m)
{
    __shared__ __attribute__((aligned(16))) char smem[X3KTile<SH>::LDS_BYTES];
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    int64_t tm, tn;
    tile_coords(t, tiles_m, tiles_n, group_m, tm, tn);
    X3KTile<SH>::run(p, tm * SH::BM, tn * SH::BN, smem);
}

template <class SH>
hipError_t launch_packed(const PackedArgs &p, int group_m, hipStream_t s)
{
    const int64_t tm = (p.g.m + SH::BM - 1) / SH::BM, tn = (p.g.n + SH::BN - 1) / SH::BN;
    hipLaunchKernelGGL((packed_kernel<SH>), dim3((unsigned)(tm * tn)), dim3(SH::NT), 0, s, p, tm,
                       tn, group_m);
    return hipGetLastError();
}

template <class SH>
__global__ __launch_bounds__(SH::NT, SH::OCC) void packed_direct_kernel(PackedArgs p, int64_t tiles_m,
                                                                  int64_t tiles_n, int group_m)
{
    constexpr int SB = X3DTile<SH>::STAGE_BYTES;
    __shared__ __attribute__((aligned(16))) __bf16 s0[SB / 2];
    __shared__ __attribute__((aligned(16))) __bf16 s1[SB / 2];
    __shared__ __attribute__((aligned(16))) __bf16 s2[SB / 2];
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    int64_t tm, tn;
    tile_coords(t, tiles_m, tiles_n, group_m, tm, tn);
    X3DTile<SH>::run(p, tm * SH::BM, tn * SH::BN, s0, s1, s2);
}

template <class SH>
hipError_t launch_packed_direct(const PackedArgs &p, int group_m, hipStream_t s)
{
    const int64_t tm = (p.g.m + SH::BM - 1) / SH::BM, tn = (p.g.n + SH::BN - 1) / SH::BN;
    hipLaunchKernelGGL((packed_direct_kernel<SH>), dim3((unsigned)(tm * tn)), dim3(SH::NT), 0, s,
                       p, tm, tn, group_m);
    return hipGetLastError();
}

hipError_t launch_pack(const float *X, int64_t ld, bool kc, int64_t rows, int64_t k, int vec,
                       __bf16 *out, hipStream_t s)
{
    const int64_t rp = pack_rows_pad(rows), kb = pack_kblocks(k);
    const dim3 grid((unsigned)(rp / 256), (unsigned)kb);
    if (kc)
        hipLaunchKernelGGL((pack_x3_kernel<true>), grid, dim3(256), 0, s, X, ld, rows, k, rp, vec,
                           out);
    else
        hipLaunchKernelGGL((pack_x3_kernel<false>), grid, dim3(256), 0, s, X, ld, rows, k, rp,
                           vec, out);
    return hipGetLastError();
}

// The packing of a whole batch: block b finds its job (the last one whose
// first_block <= b) by bisection, then packs one 256-row x 16-k unit of it.
__global__ __launch_bounds__(256) void pack_batch_kernel(const PackJob *__restrict__ jobs,
                                                         int njobs)
{
    const int64_t b = blockIdx.x;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (jobs[mid].first_block <= b) lo = mid;
        else hi = mid - 1;
    }
    const PackJob &j = jobs[lo];
    const int64_t local = b - j.first_block;
    const int64_t r = (local % j.row_blocks) * 256 + threadIdx.x;
    const int64_t kb = local / j.row_blocks;
    if (r >= j.rows_pad) return;
    if (j.kc) pack_unit<true>(j.X, j.ld, j.rows, j.kdim, j.rows_pad, j.vec, j.out, r, kb);
    else pack_unit<false>(j.X, j.ld, j.rows, j.kdim, j.rows_pad, j.vec, j.out, r, kb);
}

hipError_t launch_pack_batch(const PackJob *jobs, int njobs, int64_t blocks, hipStream_t s)
{
    if (njobs <= 0 || blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(pack_batch_kernel, dim3((unsigned)blocks), dim3(256), 0, s, jobs, njobs);
    return hipGetLastError();
}

// Persistent tile kernel over the tiles of a packed batch (the tile lists of
// batch_kernel: one list per XCD, longest tiles first).
template <class SH, bool DIRECT>
__global__ __launch_bounds__(SH::NT, SH::OCC) void packed_batch_kernel(
    const PackedArgs *__restrict__ probs, const TileDev *__restrict__ tiles, BatchSplit split)
{
    // three distinct stage arrays for the direct copies (as in
    // packed_direct_kernel), one buffer for the register-staged tile
    constexpr int SB = X3DTile<SH>::STAGE_BYTES;
    constexpr int HS = DIRECT ? SB / 2 : 8;
    __shared__ __attribute__((aligned(16))) __bf16 s0[HS];
    __shared__ __attribute__((aligned(16))) __bf16 s1[HS];
    __shared__ __attribute__((aligned(16))) __bf16 s2[HS];
    __shared__ __attribute__((aligned(16))) char smem[DIRECT ? 16 : X3KTile<SH>::LDS_BYTES];
    const int x = (int)(blockIdx.x % (unsigned)split.nx);
    const int64_t slot = blockIdx.x / (unsigned)split.nx, slots = gridDim.x / (unsigned)split.nx;
    const int64_t end = split.off[x + 1];
    for (int64_t t = split.off[x] + slot; t < end; t += slots) {
        const TileDev td = tiles[t];
        const PackedArgs p = probs[td.prob];
        const int64_t m0 = (int64_t)td.tm * SH::BM, n0 = (int64_t)td.tn * SH::BN;
        if constexpr (DIRECT) X3DTile<SH>::run(p, m0, n0, s0, s1, s2);
        else X3KTile<SH>::run(p, m0, n0, smem);
        __syncthreads();
    }
}

template <class SH, bool DIRECT>
hipError_t launch_packed_batch(const PackedArgs *probs, const TileDev *tiles,
                               const BatchSplit &split, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((packed_batch_kernel<SH, DIRECT>), dim3(grid), dim3(SH::NT), 0, s, probs,
                       tiles, split);
    return hipGetLastError();
}

template <class SH, bool DIRECT>
int packed_batch_occupancy()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, packed_batch_kernel<SH, DIRECT>,
                                                     SH::NT, 0) != hipSuccess)
        return 1;
    return blocks > 0 ? blocks : 1;
}

namespace {

template <class SH, bool DIRECT, bool BATCHED = false>
ConfigEntry make_x3k(const char *name)
{
    ConfigEntry e;
    memset(&e, 0, sizeof(e));
    e.desc.mode = MISGEMM_BF16X3;
    e.desc.bm = SH::BM;
    e.desc.bn = SH::BN;
    e.desc.bk = PACK_K;
    e.desc.wm = SH::WM;
    e.desc.wn = SH::WN;
    e.desc.threads = SH::NT;
    e.desc.lds_bytes = DIRECT ? 3 * X3DTile<SH>::STAGE_BYTES : X3KTile<SH>::LDS_BYTES;
    e.desc.packed = 1;
    strncpy(e.desc.name, name, sizeof(e.desc.name) - 1);
    e.packed = DIRECT ? launch_packed_direct<SH> : launch_packed<SH>;
    if constexpr (BATCHED) {
        e.packed_batch = launch_packed_batch<SH, DIRECT>;
        e.batch_occupancy = packed_batch_occupancy<SH, DIRECT>;
    }
    return e;
}

}  // namespace

void register_x3k(std::vector<ConfigEntry> &out)
{
    // direct global->LDS copies, three stages
    out.push_back(make_x3k<Shape<256, 256, 16, 128, 128>, true>("x3dl_256x256x16_w128x128"));
    out.push_back(make_x3k<Shape<256, 256, 16, 64, 128>, true>("x3dl_256x256x16_w64x128"));
    out.push_back(make_x3k<Shape<256, 256, 16, 128, 64>, true>("x3dl_256x256x16_w128x64"));
    out.push_back(make_x3k<Shape<128, 128, 16, 64, 64>, true, true>("x3dl_128x128x16_w64x64"));
    out.push_back(make_x3k<Shape<64, 64, 16, 32, 32>, true, true>("x3dl_64x64x16_w32x32"));
    // register-staged copies, two stages
    out.push_back(make_x3k<Shape<256, 256, 16, 64, 128>, false>("x3k_256x256x16_w64x128"));
    out.push_back(make_x3k<Shape<256, 256, 16, 128, 64>, false>("x3k_256x256x16_w128x64"));
    out.push_back(make_x3k<Shape<256, 256, 16, 128, 128>, false>("x3k_256x256x16_w128x128"));
    out.push_back(make_x3k<Shape<128, 128, 16, 64, 64>, false, true>("x3k_128x128x16_w64x64"));
    out.push_back(make_x3k<Shape<64, 64, 16, 32, 32>, false, true>("x3k_64x64x16_w32x32"));
}

}  // namespace misgemm
