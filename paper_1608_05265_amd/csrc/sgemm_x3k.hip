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

namespace {

template <class SH, bool DIRECT>
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
    return e;
}

}  // namespace

void register_x3k(std::vector<ConfigEntry> &out)
{
    // direct global->LDS copies, three stages
    out.push_back(make_x3k<Shape<256, 256, 16, 128, 128>, true>("x3dl_256x256x16_w128x128"));
    out.push_back(make_x3k<Shape<256, 256, 16, 64, 128>, true>("x3dl_256x256x16_w64x128"));
    out.push_back(make_x3k<Shape<256, 256, 16, 128, 64>, true>("x3dl_256x256x16_w128x64"));
    out.push_back(make_x3k<Shape<128, 128, 16, 64, 64>, true>("x3dl_128x128x16_w64x64"));
    // register-staged copies, two stages
    out.push_back(make_x3k<Shape<256, 256, 16, 64, 128>, false>("x3k_256x256x16_w64x128"));
    out.push_back(make_x3k<Shape<256, 256, 16, 128, 64>, false>("x3k_256x256x16_w128x64"));
    out.push_back(make_x3k<Shape<256, 256, 16, 128, 128>, false>("x3k_256x256x16_w128x128"));
    out.push_back(make_x3k<Shape<128, 128, 16, 64, 64>, false>("x3k_128x128x16_w64x64"));
}

}  // namespace misgemm
