// Split-precision configurations: three bf16 parts per FP32 operand, six
// part products on v_mfma_f32_32x32x16_bf16, FP32 accumulation.
#include <string.h>

#include "registry.hpp"

namespace misgemm {

namespace {

// one accumulator for all six products
template <class SH, bool TA, bool TB>
using X3S = X3Tile<SH, TA, TB, false>;
// the leading product a0*b0 in its own accumulator, the five small ones in another
template <class SH, bool TA, bool TB>
using X3D = X3Tile<SH, TA, TB, true>;

// pipelined: split/store of the next block starts after 1/3 of the MFMAs
template <class SH, bool TA, bool TB>
using X3P13 = X3PTile<SH, TA, TB, 1, 3>;
// the same with the order pinned by fences instead of group barriers
template <class SH, bool TA, bool TB>
using X3F13 = X3PTile<SH, TA, TB, 1, 3, true>;
// pipelined with the global loads two K blocks ahead (two register sets)
template <class SH, bool TA, bool TB>
using X3Q13 = X3PTile<SH, TA, TB, 1, 3, false, true>;

// small tiles, four waves splitting each tile's K steps
template <class SH, bool TA, bool TB>
using X3W = X3WTile<SH, TA, TB>;

// register tiles (16x16 blocks on v_mfma_f32_16x16x32_bf16, split in
// registers, no LDS staging) for latency-bound problems
template <class SH, bool TA, bool TB>
using X3R = X3RTile<SH, TA, TB>;

template <template <class, bool, bool> class T, class SH, bool BATCHED, bool SPLITK = false>
ConfigEntry make_x3(const char *name)
{
    ConfigEntry e;
    memset(&e, 0, sizeof(e));
    e.desc.mode = MISGEMM_BF16X3;
    e.desc.bm = SH::BM;
    e.desc.bn = SH::BN;
    e.desc.bk = SH::BK;
    e.desc.wm = SH::WM;
    e.desc.wn = SH::WN;
    e.desc.threads = SH::NT;
    e.desc.lds_bytes = T<SH, false, false>::LDS_BYTES;
    strncpy(e.desc.name, name, sizeof(e.desc.name) - 1);
    e.launch[0][0] = launch_tile_kernel<T<SH, false, false>, SH>;
    e.launch[0][1] = launch_tile_kernel<T<SH, false, true>, SH>;
    e.launch[1][0] = launch_tile_kernel<T<SH, true, false>, SH>;
    e.launch[1][1] = launch_tile_kernel<T<SH, true, true>, SH>;
    if constexpr (BATCHED) {
        e.batch = launch_batch_kernel<T, SH>;
        e.batch_occupancy = batch_occupancy<T, SH>;
    }
    if constexpr (SPLITK) {
        e.splitk[0][0] = launch_splitk_kernel<T<SH, false, false>, SH, false, false>;
        e.splitk[0][1] = launch_splitk_kernel<T<SH, false, true>, SH, false, true>;
        e.splitk[1][0] = launch_splitk_kernel<T<SH, true, false>, SH, true, false>;
        e.splitk[1][1] = launch_splitk_kernel<T<SH, true, true>, SH, true, true>;
    }
    return e;
}

}  // namespace

void register_x3(std::vector<ConfigEntry> &out)
{
    // 8 waves (two per SIMD): the other wave issues MFMAs while one splits
    out.push_back(make_x3<X3F13, Shape<256, 256, 16, 128, 64>, false>("x3f_256x256x16_w128x64"));
    out.push_back(make_x3<X3F13, Shape<256, 256, 16, 64, 128>, false>("x3f_256x256x16_w64x128"));
    out.push_back(make_x3<X3F13, Shape<256, 256, 16, 128, 128>, false>("x3f_256x256x16_w128x128"));
    out.push_back(make_x3<X3P13, Shape<128, 128, 16, 64, 64>, true, true>("x3p_128x128x16_w64x64"));
    out.push_back(make_x3<X3Q13, Shape<128, 128, 16, 64, 64>, true, true>("x3q_128x128x16_w64x64"));
    out.push_back(make_x3<X3S, Shape<128, 128, 32, 64, 64>, true>("x3_128x128x32_w64x64"));
    out.push_back(make_x3<X3D, Shape<128, 128, 32, 64, 64>, true, true>("x3d_128x128x32_w64x64"));
    out.push_back(make_x3<X3S, Shape<64, 64, 32, 32, 32>, true, true>("x3_64x64x32_w32x32"));
    out.push_back(make_x3<X3W, WShape<64, 64, 64, 4>, true>("x3w_64x64x64_k4"));
    out.push_back(make_x3<X3W, WShape<32, 32, 64, 4>, true>("x3w_32x32x64_k4"));
    // register tiles: four waves take 64-k chunks in turn
    out.push_back(make_x3<X3R, RShape<16, 16, 4>, false>("x3r_16x16x64_r4"));
    out.push_back(make_x3<X3R, RShape<32, 32, 4>, true>("x3r_32x32x64_r4"));
    // eight waves taking 32-k chunks in turn (half the loads per wave)
    out.push_back(make_x3<X3R, RShape<16, 16, 8, 8>, false>("x3r_16x16x32_r8"));
}

}  // namespace misgemm
