// FP32 matrix-core configurations (v_mfma_f32_32x32x2_f32; the register
// tiles v_mfma_f32_16x16x4_f32).
#include <string.h>

#include "registry.hpp"

namespace misgemm {

namespace {

template <class SH, bool TA, bool TB>
using F32 = F32Tile<SH, TA, TB>;
template <class SH, bool TA, bool TB>
using F32P = F32PTile<SH, TA, TB>;
template <class SH, bool TA, bool TB>
using F32W = F32WTile<SH, TA, TB>;
// global loads two K blocks ahead (two register sets)
template <class SH, bool TA, bool TB>
using F32Q = F32Tile<SH, TA, TB, true>;
// register tiles (16x16 blocks, no LDS staging) for latency-bound problems
template <class SH, bool TA, bool TB>
using F32R = F32RTile<SH, TA, TB>;

template <template <class, bool, bool> class T, class SH, bool BATCHED, bool SPLITK = false>
ConfigEntry make_f32(const char *name)
{
    ConfigEntry e;
    memset(&e, 0, sizeof(e));
    e.desc.mode = MISGEMM_FP32;
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

void register_f32(std::vector<ConfigEntry> &out)
{
    out.push_back(make_f32<F32P, Shape<256, 256, 16, 128, 64>, false>("fp32p_256x256x16_w128x64"));
    out.push_back(make_f32<F32P, Shape<256, 256, 32, 128, 64>, false>("fp32p_256x256x32_w128x64"));
    out.push_back(make_f32<F32P, Shape<256, 128, 16, 128, 64, 2>, false>("fp32p_256x128x16_w128x64"));
    out.push_back(make_f32<F32P, Shape<128, 128, 16, 64, 64>, true, true>("fp32p_128x128x16_w64x64"));
    out.push_back(make_f32<F32P, Shape<128, 128, 32, 64, 64>, true>("fp32p_128x128x32_w64x64"));
    out.push_back(make_f32<F32P, Shape<64, 64, 32, 32, 32>, true, true>("fp32p_64x64x32_w32x32"));
    out.push_back(make_f32<F32, Shape<128, 128, 16, 64, 64>, true, true>("fp32_128x128x16_w64x64"));
    out.push_back(make_f32<F32, Shape<128, 64, 16, 64, 32>, true>("fp32_128x64x16_w64x32"));
    out.push_back(make_f32<F32, Shape<64, 64, 16, 32, 32>, true, true>("fp32_64x64x16_w32x32"));
    out.push_back(make_f32<F32Q, Shape<64, 64, 16, 32, 32>, true, true>("fp32q_64x64x16_w32x32"));
    out.push_back(make_f32<F32Q, Shape<128, 128, 16, 64, 64>, true, true>("fp32q_128x128x16_w64x64"));
    out.push_back(make_f32<F32Q, Shape<128, 64, 16, 64, 32>, true>("fp32q_128x64x16_w64x32"));
    // small tiles, four waves splitting each tile's K steps
    out.push_back(make_f32<F32W, WShape<64, 64, 32, 4>, true>("fp32w_64x64x32_k4"));
    out.push_back(make_f32<F32W, WShape<32, 32, 32, 4>, true>("fp32w_32x32x32_k4"));
    // register tiles: four waves take 64-k chunks in turn
    out.push_back(make_f32<F32R, RShape<16, 16, 4>, false>("fp32r_16x16x64_r4"));
    out.push_back(make_f32<F32R, RShape<32, 32, 4>, true>("fp32r_32x32x64_r4"));
    // eight waves taking 32-k chunks in turn (half the loads per wave)
    out.push_back(make_f32<F32R, RShape<16, 16, 8, 8>, false>("fp32r_16x16x32_r8"));
}

}  // namespace misgemm
