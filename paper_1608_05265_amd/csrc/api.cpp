// The C-ABI of the library: argument checking, degenerate cases, choice of
// tile configuration, and the batched plan (see include/misgemm.h).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "dgemm.hpp"
#include "registry.hpp"

using namespace misgemm;

namespace {

std::vector<ConfigEntry> &configs()
{
    static std::vector<ConfigEntry> table;
    static std::once_flag once;
    std::call_once(once, [] {
        register_f32(table);
        register_x3(table);
        register_x3k(table);
    });
    return table;
}

// Per-device facts, read once per device.
struct DeviceInfo {
    bool checked = false;
    bool ok = false;
    int cus = 0;
};

constexpr int MAX_DEVICES = 64;
DeviceInfo g_devices[MAX_DEVICES];
std::mutex g_dev_mutex;

int current_device(DeviceInfo **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return MISGEMM_E_NO_DEVICE;
    if (dev < 0 || dev >= MAX_DEVICES) return MISGEMM_E_NO_DEVICE;
    std::lock_guard<std::mutex> lock(g_dev_mutex);
    DeviceInfo &d = g_devices[dev];
    if (!d.checked) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return MISGEMM_E_NO_DEVICE;
        d.ok = strncmp(prop.gcnArchName, "gfx950", 6) == 0;
        d.cus = prop.multiProcessorCount;
        d.checked = true;
    }
    if (!d.ok) return MISGEMM_E_NO_DEVICE;
    *out = &d;
    return 0;
}

int trans_flag(char t)
{
    if (t == 'N' || t == 'n') return 0;
    if (t == 'T' || t == 't' || t == 'C' || t == 'c') return 1;
    return -1;
}

// ---------------------------------------------------------------------------
// Tuning table (format in include/misgemm.h, misgemm_load_tuning).
// ---------------------------------------------------------------------------
struct TuneEntry {
    int mode, ta, tb;
    int64_t m, n, k;
    int config;
    int group_m;
    int splits;  // 0: automatic, 1: whole K per workgroup, >= 2: split-K factor
};
std::vector<TuneEntry> g_tuning;
int g_batch_config[2] = {-1, -1};  // per mode, from "batch" lines
// per mode, from "batch2" lines: problems with m and n >= threshold use
// config big, the others config small, in two concurrent launches
struct BatchRule {
    int threshold, big, small;
};
BatchRule g_batch_rule[2] = {{0, -1, -1}, {0, -1, -1}};
std::mutex g_tune_mutex;

int find_config(const char *name)
{
    const auto &t = configs();
    for (size_t i = 0; i < t.size(); ++i)
        if (strcmp(t[i].desc.name, name) == 0) return (int)i;
    return -1;
}

// Nearest tuned entry (same mode and transposes, every size within a factor
// 2, smallest summed log-distance; on equal distance the earlier line, so a
// table lists a key's packed winner before its best non-packed entry), among
// the non-packed configurations unless allow_packed; -1 when none.
int tuned_config(int mode, int ta, int tb, int64_t m, int64_t n, int64_t k, bool allow_packed,
                 int *group_m, int *splits)
{
    const auto &table = configs();
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    int best = -1;
    double best_d = 1e300;
    for (const TuneEntry &e : g_tuning) {
        if (e.mode != mode || e.ta != ta || e.tb != tb) continue;
        if (!allow_packed && table[e.config].desc.packed) continue;
        const double dm = fabs(log2((double)m / (double)e.m));
        const double dn = fabs(log2((double)n / (double)e.n));
        const double dk = fabs(log2((double)k / (double)e.k));
        if (dm > 1.0 || dn > 1.0 || dk > 1.0) continue;
        const double d = dm + dn + dk;
        if (d < best_d) {
            best_d = d;
            best = e.config;
            *group_m = e.group_m;
            *splits = e.splits;
        }
    }
    return best;
}

// Built-in choice: the largest tile that still gives every CU at least one
// tile (packed configurations first on equal area, when allowed); below that
// the smallest tile (fewest idle CUs).
int heuristic_config(int mode, int64_t m, int64_t n, int64_t k, int cus, bool allow_packed)
{
    (void)k;
    const auto &t = configs();
    int best = -1;
    int64_t best_key = -1;
    int smallest = -1;
    int64_t smallest_area = INT64_MAX;
    for (size_t i = 0; i < t.size(); ++i) {
        const misgemm_config_desc &d = t[i].desc;
        if (d.mode != mode || (d.packed && !allow_packed)) continue;
        const int64_t area = (int64_t)d.bm * d.bn;
        const int64_t key = 2 * area + (d.packed ? 1 : 0);
        const int64_t tiles = ((m + d.bm - 1) / d.bm) * ((n + d.bn - 1) / d.bn);
        if (tiles >= cus && key > best_key) { best_key = key; best = (int)i; }
        if (area < smallest_area) { smallest_area = area; smallest = (int)i; }
    }
    return best >= 0 ? best : smallest;
}

int select_config(int mode, int ta, int tb, int64_t m, int64_t n, int64_t k, int cus,
                  bool allow_packed, int *group_m, int *splits)
{
    *group_m = GROUP_M_DEFAULT;
    *splits = 0;
    const int c = tuned_config(mode, ta, tb, m, n, k, allow_packed, group_m, splits);
    if (c >= 0) return c;
    *group_m = GROUP_M_DEFAULT;
    *splits = 0;
    return heuristic_config(mode, m, n, k, cus, allow_packed);
}

// ---------------------------------------------------------------------------
// Workspace of the packed path.
// ---------------------------------------------------------------------------
int64_t packed_bytes(int64_t m, int64_t n, int64_t k)
{
    return 2 * (pack_halves(m, k) + pack_halves(n, k)) + 512;
}

// Library-owned scratch, one set per (device, stream): calls on one stream
// run in order, so they can share it; calls on different streams never do.
struct StreamWorkspace {
    void *ptr = nullptr;
    int64_t bytes = 0;
    bool captured = false;        // ptr was handed to a call under graph capture
    std::vector<void *> retired;  // outgrown buffers that captured graphs may reference
    int64_t retired_bytes = 0;
};
std::map<std::pair<int, void *>, StreamWorkspace> g_ws;
std::mutex g_ws_mutex;

bool capturing(hipStream_t s)
{
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone;
}

// Library-owned workspace of at least `bytes` for the current device and
// stream `s`.  Returns 0 and the buffer, MISGEMM_E_CAPTURING when it would
// have to grow while `s` is capturing, or the HIP error of a failed
// allocation.  An outgrown buffer is freed once the work queued on `s` has
// finished, unless it was handed to a call under capture: then a graph may
// still use it and it is kept until misgemm_release_workspace, so memory
// accumulates only across growths that follow captures.
int library_workspace(int64_t bytes, hipStream_t s, void **out)
{
    *out = nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MISGEMM_E_NO_DEVICE;
    std::lock_guard<std::mutex> lock(g_ws_mutex);
    StreamWorkspace &w = g_ws[{dev, (void *)s}];
    const bool cap = capturing(s);
    if (w.bytes >= bytes) {
        if (cap) w.captured = true;
        *out = w.ptr;
        return 0;
    }
    if (cap) return MISGEMM_E_CAPTURING;
    const int64_t want = std::max<int64_t>(bytes, w.bytes + w.bytes / 2);
    if (w.ptr) {
        if (w.captured) {
            w.retired.push_back(w.ptr);
            w.retired_bytes += w.bytes;
        } else {
            // only calls on `s` use it, and they run in order
            hipError_t e = hipStreamSynchronize(s);
            if (e == hipSuccess) e = hipFree(w.ptr);
            if (e != hipSuccess) return (int)e;
        }
        w.ptr = nullptr;
        w.bytes = 0;
        w.captured = false;
    }
    void *p = nullptr;
    const hipError_t e = hipMalloc(&p, (size_t)want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return (int)e;
    }
    w.ptr = p;
    w.bytes = want;
    *out = p;
    return 0;
}

// ---------------------------------------------------------------------------
// Static scratch of misgemm_sgemm_split_noalloc: one array per device, in
// the code object, so that calls need no allocation.  Host code uses the
// device address hipGetSymbolAddress returns for the current device, never
// the array's name (a host-side stand-in).
// ---------------------------------------------------------------------------
static __device__ __align__(256) float scratch[MISGEMM_STATIC_SCRATCH_BYTES / 4];
void *g_scratch_ptr[MAX_DEVICES];
std::mutex g_scratch_mutex;

// Device address of the current device's copy of `scratch`, looked up once
// per device.
int static_scratch(void **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
        return MISGEMM_E_NO_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            return e != hipSuccess ? (int)e : MISGEMM_E_NO_DEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

hipError_t launch_packed_path(const ConfigEntry &cfg, int ta, int tb, const GemmArgs &g,
                              void *ws, int group_m, hipStream_t s)
{
    __bf16 *ap = reinterpret_cast<__bf16 *>(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    __bf16 *bp = ap + pack_halves(g.m, g.k);
    hipError_t e = launch_pack(g.A, g.lda, ta != 0, g.m, g.k, g.vec_a, ap, s);
    if (e != hipSuccess) return e;
    e = launch_pack(g.B, g.ldb, tb == 0, g.n, g.k, g.vec_b, bp, s);
    if (e != hipSuccess) return e;
    PackedArgs p;
    p.g = g;
    p.Ap = ap;
    p.Bp = bp;
    p.mp = pack_rows_pad(g.m);
    p.np = pack_rows_pad(g.n);
    p.kblocks = pack_kblocks(g.k);
    return cfg.packed(p, group_m, s);
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

int validate(char transa, char transb, int64_t m, int64_t n, int64_t k, float alpha,
             const float *A, int64_t lda, const float *B, int64_t ldb, float *C, int64_t ldc,
             int mode)
{
    const int ta = trans_flag(transa), tb = trans_flag(transb);
    if (ta < 0) return -1;
    if (tb < 0) return -2;
    if (m < 0) return -3;
    if (n < 0) return -4;
    if (k < 0) return -5;
    const int64_t arows = ta ? k : m, brows = tb ? n : k;
    if (lda < std::max<int64_t>(1, arows)) return -8;
    if (ldb < std::max<int64_t>(1, brows)) return -10;
    if (ldc < std::max<int64_t>(1, m)) return -13;
    if (mode != MISGEMM_FP32 && mode != MISGEMM_BF16X3) return -14;
    const bool work = m > 0 && n > 0;
    const bool reads_ab = work && k > 0 && alpha != 0.0f;
    if (reads_ab && A == nullptr) return -7;
    if (reads_ab && B == nullptr) return -9;
    if (work && C == nullptr) return -12;
    // tile indices are 32-bit in the grid; offsets are 64-bit everywhere
    if (m > (int64_t)1 << 40 || n > (int64_t)1 << 40 || k > (int64_t)1 << 40)
        return MISGEMM_E_TOO_LARGE;
    return 0;
}

GemmArgs make_args(int64_t m, int64_t n, int64_t k, float alpha, const float *A, int64_t lda,
                   const float *B, int64_t ldb, float beta, float *C, int64_t ldc)
{
    GemmArgs g;
    g.m = m; g.n = n; g.k = k;
    g.A = A; g.B = B; g.C = C;
    g.lda = lda; g.ldb = ldb; g.ldc = ldc;
    g.alpha = alpha; g.beta = beta;
    g.vec_a = aligned16(A) && lda % 4 == 0;
    g.vec_b = aligned16(B) && ldb % 4 == 0;
    g.vec_c = aligned16(C) && ldc % 4 == 0;
    g.part = nullptr;
    g.tile = 0;
    g.split = 0;
    g.splits = 1;
    return g;
}

// Workspace policy of one call: library scratch grown on demand, a caller's
// workspace, none, or the static scratch (split-K partials only, at most
// MISGEMM_STATIC_SCRATCH_BYTES).
enum WsPolicy { WS_LIBRARY, WS_CALLER, WS_NONE, WS_STATIC };

// Split-K factor for a non-packed configuration when neither the caller nor
// the tuning table fixed one: only when the tiles leave CUs idle, enough
// splits for about two workgroups per CU, each split at least eight K blocks
// (shorter ranges lose more to the second launch and the partial traffic
// than they gain), at most 16.
int auto_splits(const ConfigEntry &e, int64_t tiles, int64_t k, int cus)
{
    if (e.splitk[0][0] == nullptr || tiles >= cus) return 1;
    const int64_t kt = (k + e.desc.bk - 1) / e.desc.bk;
    int64_t s = (2 * (int64_t)cus + tiles - 1) / tiles;
    s = std::min<int64_t>(s, std::min<int64_t>(kt / 8, 16));
    return s < 2 ? 1 : (int)s;
}

// Splits actually launched for a request: every split gets a non-empty,
// whole-block K range.
int effective_splits(int64_t k, int bk, int req)
{
    const int64_t kt = (k + bk - 1) / bk;
    if (req <= 1 || kt <= 1) return 1;
    const int64_t per = (kt + req - 1) / req;
    return (int)((kt + per - 1) / per);
}

// splits_req: 0 = automatic (tuning table, then auto_splits), >= 1 = forced.
int run_sgemm(char transa, char transb, int64_t m, int64_t n, int64_t k, float alpha,
              const float *A, int64_t lda, const float *B, int64_t ldb, float beta, float *C,
              int64_t ldc, int mode, int config_id, int group_m, void *stream,
              WsPolicy policy = WS_LIBRARY, void *workspace = nullptr, int64_t ws_bytes = 0,
              int splits_req = 0)
{
    int rc = validate(transa, transb, m, n, k, alpha, A, lda, B, ldb, C, ldc, mode);
    if (rc != 0) return rc;
    const auto &table = configs();
    if (config_id >= 0 &&
        (config_id >= (int)table.size() || table[config_id].desc.mode != mode))
        return -15;
    if (m == 0 || n == 0) return 0;
    if ((alpha == 0.0f || k == 0) && beta == 1.0f) return 0;
    DeviceInfo *dev = nullptr;
    rc = current_device(&dev);
    if (rc != 0) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (alpha == 0.0f || k == 0) return (int)launch_scale(beta, C, m, n, ldc, s);
    const int ta = trans_flag(transa), tb = trans_flag(transb);
    int gm = group_m > 0 ? group_m : GROUP_M_DEFAULT;
    // A packed configuration is chosen only when the caller passed its
    // workspace (misgemm_sgemm_ws): misgemm_sgemm allocates nothing for it.
    // One requested explicitly (misgemm_sgemm_config) uses the library scratch.
    const bool packable = mode == MISGEMM_BF16X3 && policy == WS_CALLER &&
                          pack_kblocks(k) <= 65535;
    int cfg = config_id;
    int splits = splits_req;
    int tuned_splits = 0;
    if (cfg < 0) cfg = select_config(mode, ta, tb, m, n, k, dev->cus, packable, &gm, &tuned_splits);
    if (cfg < 0) return MISGEMM_E_BAD_CONFIG;
    if (splits == 0) splits = tuned_splits;
    void *ws = nullptr;
    if (table[cfg].desc.packed) {
        if (pack_kblocks(k) > 65535) return MISGEMM_E_TOO_LARGE;
        if (policy == WS_STATIC) return -15;
        const int64_t need = packed_bytes(m, n, k);
        int wrc = 0;
        if (policy == WS_CALLER) ws = workspace;
        else if (policy == WS_LIBRARY) wrc = library_workspace(need, s, &ws);
        if (ws == nullptr) {
            // an explicitly requested packed configuration runs packed or not at all
            if (config_id >= 0 && policy == WS_LIBRARY) return wrc != 0 ? wrc : MISGEMM_E_CAPTURING;
            if (wrc != 0 && wrc != MISGEMM_E_CAPTURING) return wrc;
            // no workspace (capturing, or none given): a non-packed config
            cfg = heuristic_config(mode, m, n, k, dev->cus, false);
            gm = group_m > 0 ? group_m : GROUP_M_DEFAULT;
            splits = splits_req;
        }
    }
    const ConfigEntry &e = table[cfg];
    const misgemm_config_desc &d = e.desc;
    const int64_t tiles = ((m + d.bm - 1) / d.bm) * ((n + d.bn - 1) / d.bn);
    if (tiles > INT32_MAX) return MISGEMM_E_TOO_LARGE;
    GemmArgs g = make_args(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
    if (d.packed) return (int)launch_packed_path(e, ta, tb, g, ws, gm, s);
    const bool forced = splits_req >= 1;
    if (splits == 0) splits = policy == WS_LIBRARY ? auto_splits(e, tiles, k, dev->cus) : 1;
    splits = effective_splits(k, d.bk, splits);
    if (splits > 1) {
        if (e.splitk[0][0] == nullptr) return MISGEMM_E_BAD_CONFIG;
        const int64_t need = (int64_t)splits * tiles * d.bm * d.bn * 4;
        void *part = nullptr;
        int wrc = 0;
        if (policy == WS_LIBRARY) {
            wrc = library_workspace(need, s, &part);
        } else if (policy == WS_STATIC) {
            if (need > ws_bytes) return MISGEMM_E_SCRATCH;
            part = workspace;
        }
        if (part != nullptr) {
            g.part = (float *)part;
            g.splits = splits;
            return (int)e.splitk[ta][tb](g, gm, s);
        }
        if (forced) return wrc != 0 ? wrc : MISGEMM_E_CAPTURING;
        if (wrc != 0 && wrc != MISGEMM_E_CAPTURING) return wrc;
    }
    return (int)e.launch[ta][tb](g, gm, s);
}

}  // namespace

// ---------------------------------------------------------------------------
// Batched plan.
// ---------------------------------------------------------------------------
struct misgemm_batch {
    int config_id;
    int mode;
    int64_t count, ntiles;
    int grid;
    double flops, tile_flops;
    double part_imbalance;
    BatchSplit split;
    ProbDev *d_probs;
    TileDev *d_tiles;
    int device;
    // packed configurations: every operand split once into panels the plan
    // owns (one pack launch), then the tile kernel on the panels
    bool packed;
    PackedArgs *d_pprobs;
    PackJob *d_jobs;
    int njobs;
    int64_t pack_blocks;
    void *d_panels;
    int64_t panel_bytes;
    // two-part plans: the problems below the size threshold in their own
    // plan, launched on `side` between the fork and join events
    misgemm_batch *second;
    hipStream_t side;
    hipEvent_t fork, join;
};

// Build the plan of the problems listed in `index` (already validated) with
// configuration cfg: tiles, their partition over the XCDs, device tables.
int build_part(const misgemm_problem *problems, const std::vector<int64_t> &index, int mode,
               int cfg, const DeviceInfo *dev, misgemm_batch **out, int64_t *bad_index)
{
    const auto &table = configs();
    const misgemm_config_desc &d = table[cfg].desc;

    std::vector<ProbDev> probs;
    std::vector<TileDev> tiles;
    std::vector<int64_t> work;   // per-tile K (work of a full tile is bm*bn*k)
    std::vector<int64_t> first;  // per problem: index of its first tile
    probs.reserve(index.size());
    double flops = 0.0, tile_flops = 0.0;
    // packed: panel rows padded to the larger tile side (so every tile reads
    // inside its panels), panels 256-byte aligned in one plan-owned buffer
    const bool packed = d.packed != 0;
    const int64_t pad_rows = std::max(d.bm, d.bn);
    std::vector<PackedArgs> pprobs;
    std::vector<PackJob> jobs;
    std::vector<int64_t> a_off, b_off;  // panel offsets, in bf16 elements
    int64_t panel_halves = 0, pack_blocks = 0;
    auto round_up = [](int64_t x, int64_t q) { return (x + q - 1) / q * q; };
    for (const int64_t i : index) {
        const misgemm_problem &p = problems[i];
        if (p.m == 0 || p.n == 0) continue;
        if ((p.alpha == 0.0f || p.k == 0) && p.beta == 1.0f) continue;
        ProbDev pd;
        const bool ab = p.alpha != 0.0f && p.k > 0;
        pd.g = make_args(p.m, p.n, ab ? p.k : 0, p.alpha, p.A, p.lda, p.B, p.ldb, p.beta, p.C,
                         p.ldc);
        pd.ta = trans_flag(p.transa);
        pd.tb = trans_flag(p.transb);
        pd.tiles_m = (p.m + d.bm - 1) / d.bm;
        pd.tiles_n = (p.n + d.bn - 1) / d.bn;
        if (pd.tiles_m > INT32_MAX || pd.tiles_n > INT32_MAX || (int64_t)probs.size() >= INT32_MAX) {
            if (bad_index) *bad_index = i;
            return MISGEMM_E_TOO_LARGE;
        }
        const int32_t idx = (int32_t)probs.size();
        probs.push_back(pd);
        if (packed) {
            PackedArgs pa;
            pa.g = pd.g;
            pa.mp = round_up(p.m, pad_rows);
            pa.np = round_up(p.n, pad_rows);
            pa.kblocks = pack_kblocks(pd.g.k);
            pa.Ap = pa.Bp = nullptr;  // set once the panel buffer exists
            a_off.push_back(panel_halves);
            panel_halves += round_up(pa.kblocks * 3 * pa.mp * PACK_K, 128);
            b_off.push_back(panel_halves);
            panel_halves += round_up(pa.kblocks * 3 * pa.np * PACK_K, 128);
            if (pa.kblocks > 0) {
                // op(A) is k-contiguous when A is transposed, op(B) when B is not
                const PackJob ja = {p.A, nullptr, p.lda, p.m, pd.g.k, pa.mp, pack_blocks,
                                    (pa.mp + 255) / 256, pd.ta != 0, pd.g.vec_a};
                pack_blocks += ja.row_blocks * pa.kblocks;
                const PackJob jb = {p.B, nullptr, p.ldb, p.n, pd.g.k, pa.np, pack_blocks,
                                    (pa.np + 255) / 256, pd.tb == 0, pd.g.vec_b};
                pack_blocks += jb.row_blocks * pa.kblocks;
                jobs.push_back(ja);
                jobs.push_back(jb);
            }
            pprobs.push_back(pa);
        }
        first.push_back((int64_t)tiles.size());
        flops += 2.0 * (double)p.m * (double)p.n * (double)pd.g.k;
        tile_flops += 2.0 * (double)(pd.tiles_m * d.bm) * (double)(pd.tiles_n * d.bn) *
                      (double)pd.g.k;
        for (int64_t tn = 0; tn < pd.tiles_n; ++tn)
            for (int64_t tm = 0; tm < pd.tiles_m; ++tm) {
                tiles.push_back({idx, (int32_t)tm, (int32_t)tn, 0});
                work.push_back(pd.g.k);
            }
    }
    first.push_back((int64_t)tiles.size());
    const int64_t ntiles = (int64_t)tiles.size();
    const int occ = table[cfg].batch_occupancy ? table[cfg].batch_occupancy() : 1;
    int64_t grid = (int64_t)dev->cus * occ;
    if (grid > ntiles) grid = ntiles;
    if (grid < 1) grid = 1;
    const int nx = grid >= MAX_XCD ? MAX_XCD : 1;
    grid -= grid % nx;

    // Deal the tiles to the XCDs so that each XCD's L2 serves few problems:
    // problems are cut into chunks of consecutive tiles (tiles of a chunk
    // share operand panels) of at most 1/(4*nx) of the total work, the
    // chunks go longest first to the least-loaded XCD, and each XCD orders
    // its tiles by decreasing K (longest processing time first; stable, so
    // the tiles of a chunk stay together).
    int64_t total_work = 0;
    for (int64_t w : work) total_work += std::max<int64_t>(1, w);
    const int64_t chunk_cap = std::max<int64_t>(1, (total_work + 4 * nx - 1) / (4 * nx));
    struct Chunk { int64_t begin, end, work; };
    std::vector<Chunk> chunks;
    for (size_t p = 0; p + 1 < first.size(); ++p) {
        const int64_t b = first[p], e = first[p + 1];
        if (b == e) continue;
        const int64_t per = std::max<int64_t>(1, work[(size_t)b]);
        const int64_t pwork = (e - b) * per;
        const int64_t pieces = (pwork + chunk_cap - 1) / chunk_cap;
        const int64_t step = (e - b + pieces - 1) / pieces;
        for (int64_t c = b; c < e; c += step) {
            const int64_t ce = std::min(e, c + step);
            chunks.push_back({c, ce, (ce - c) * per});
        }
    }
    std::stable_sort(chunks.begin(), chunks.end(),
                     [](const Chunk &a, const Chunk &b) { return a.work > b.work; });
    std::vector<std::vector<int64_t>> part((size_t)nx);
    std::vector<int64_t> load((size_t)nx, 0);
    for (const Chunk &c : chunks) {
        int best = 0;
        for (int x = 1; x < nx; ++x)
            if (load[(size_t)x] < load[(size_t)best]) best = x;
        load[(size_t)best] += c.work;
        for (int64_t t = c.begin; t < c.end; ++t) part[(size_t)best].push_back(t);
    }
    std::vector<TileDev> sorted;
    sorted.reserve(tiles.size());
    BatchSplit split = {};
    split.nx = nx;
    int64_t max_load = 0;
    for (int x = 0; x < nx; ++x) {
        std::vector<int64_t> &pt = part[(size_t)x];
        std::stable_sort(pt.begin(), pt.end(),
                         [&](int64_t a, int64_t b) { return work[(size_t)a] > work[(size_t)b]; });
        split.off[x] = (int64_t)sorted.size();
        for (int64_t t : pt) sorted.push_back(tiles[(size_t)t]);
        max_load = std::max(max_load, load[(size_t)x]);
    }
    for (int x = nx; x <= MAX_XCD; ++x) split.off[x] = (int64_t)sorted.size();

    misgemm_batch *b = (misgemm_batch *)calloc(1, sizeof(misgemm_batch));
    if (!b) return (int)hipErrorOutOfMemory;
    b->config_id = cfg;
    b->mode = mode;
    b->count = (int64_t)index.size();
    b->ntiles = (int64_t)sorted.size();
    b->flops = flops;
    b->tile_flops = tile_flops;
    b->split = split;
    b->part_imbalance = total_work > 0 ? (double)max_load * nx / (double)total_work : 1.0;
    (void)hipGetDevice(&b->device);
    b->grid = (int)grid;
    b->packed = packed;
    if (packed && (pack_blocks > INT32_MAX || jobs.size() > (size_t)INT32_MAX)) {
        free(b);
        return MISGEMM_E_TOO_LARGE;
    }
    hipError_t e = hipSuccess;
    if (!probs.empty()) {
        e = hipMalloc((void **)&b->d_tiles, sorted.size() * sizeof(TileDev));
        if (e == hipSuccess)
            e = hipMemcpy(b->d_tiles, sorted.data(), sorted.size() * sizeof(TileDev),
                          hipMemcpyHostToDevice);
        if (!packed) {
            if (e == hipSuccess) e = hipMalloc((void **)&b->d_probs, probs.size() * sizeof(ProbDev));
            if (e == hipSuccess)
                e = hipMemcpy(b->d_probs, probs.data(), probs.size() * sizeof(ProbDev),
                              hipMemcpyHostToDevice);
        } else {
            b->panel_bytes = panel_halves * 2;
            if (e == hipSuccess && b->panel_bytes > 0) e = hipMalloc(&b->d_panels, (size_t)b->panel_bytes);
            __bf16 *base = reinterpret_cast<__bf16 *>(b->d_panels);
            size_t jn = 0;
            for (size_t i = 0; i < pprobs.size(); ++i) {
                pprobs[i].Ap = base + a_off[i];
                pprobs[i].Bp = base + b_off[i];
                if (pprobs[i].kblocks > 0) {
                    jobs[jn++].out = base + a_off[i];
                    jobs[jn++].out = base + b_off[i];
                }
            }
            b->njobs = (int)jobs.size();
            b->pack_blocks = pack_blocks;
            if (e == hipSuccess)
                e = hipMalloc((void **)&b->d_pprobs, pprobs.size() * sizeof(PackedArgs));
            if (e == hipSuccess)
                e = hipMemcpy(b->d_pprobs, pprobs.data(), pprobs.size() * sizeof(PackedArgs),
                              hipMemcpyHostToDevice);
            if (e == hipSuccess && !jobs.empty())
                e = hipMalloc((void **)&b->d_jobs, jobs.size() * sizeof(PackJob));
            if (e == hipSuccess && !jobs.empty())
                e = hipMemcpy(b->d_jobs, jobs.data(), jobs.size() * sizeof(PackJob),
                              hipMemcpyHostToDevice);
        }
    }
    if (e != hipSuccess) {
        if (b->d_probs) (void)hipFree(b->d_probs);
        if (b->d_tiles) (void)hipFree(b->d_tiles);
        if (b->d_pprobs) (void)hipFree(b->d_pprobs);
        if (b->d_jobs) (void)hipFree(b->d_jobs);
        if (b->d_panels) (void)hipFree(b->d_panels);
        free(b);
        return (int)e;
    }
    *out = b;
    return 0;
}


extern "C" {

int misgemm_sgemm(char transa, char transb, int64_t m, int64_t n, int64_t k, float alpha,
                  const float *A, int64_t lda, const float *B, int64_t ldb, float beta, float *C,
                  int64_t ldc, int mode, void *stream)
{
    return run_sgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, mode, -1, 0,
                     stream);
}

int misgemm_sgemm_config(char transa, char transb, int64_t m, int64_t n, int64_t k, float alpha,
                         const float *A, int64_t lda, const float *B, int64_t ldb, float beta,
                         float *C, int64_t ldc, int mode, int config_id, int group_m,
                         void *stream)
{
    if (config_id < 0) return -15;
    if (group_m < 0 || group_m > 4096) return -16;
    return run_sgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, mode,
                     config_id, group_m, stream, WS_LIBRARY, nullptr, 0, 1);
}

int misgemm_sgemm_split(char transa, char transb, int64_t m, int64_t n, int64_t k, float alpha,
                        const float *A, int64_t lda, const float *B, int64_t ldb, float beta,
                        float *C, int64_t ldc, int mode, int config_id, int group_m, int splits,
                        void *stream)
{
    if (group_m < 0 || group_m > 4096) return -16;
    if (splits < 1 || splits > 64) return -17;
    if (config_id < 0 && splits > 1) {
        // the split-capable configuration of the mode with the smallest tile
        const auto &t = configs();
        int64_t best = INT64_MAX;
        for (size_t i = 0; i < t.size(); ++i) {
            const int64_t area = (int64_t)t[i].desc.bm * t[i].desc.bn;
            if (t[i].desc.mode == mode && t[i].splitk[0][0] && area < best) {
                best = area;
                config_id = (int)i;
            }
        }
    }
    return run_sgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, mode,
                     config_id, group_m, stream, WS_LIBRARY, nullptr, 0, splits);
}

int misgemm_sgemm_split_noalloc(char transa, char transb, int64_t m, int64_t n, int64_t k,
                                float alpha, const float *A, int64_t lda, const float *B,
                                int64_t ldb, float beta, float *C, int64_t ldc, int mode,
                                int config_id, int group_m, int splits, void *stream)
{
    if (group_m < 0 || group_m > 4096) return -16;
    if (splits < 1 || splits > 64) return -17;
    const auto &t = configs();
    if (config_id >= 0 && config_id < (int)t.size() && t[config_id].desc.packed) return -15;
    if (config_id < 0 && splits > 1) {
        int64_t best = INT64_MAX;
        for (size_t i = 0; i < t.size(); ++i) {
            const int64_t area = (int64_t)t[i].desc.bm * t[i].desc.bn;
            if (t[i].desc.mode == mode && t[i].splitk[0][0] && area < best) {
                best = area;
                config_id = (int)i;
            }
        }
    }
    // argument errors first, so that C stays untouched on any of them
    int rc = validate(transa, transb, m, n, k, alpha, A, lda, B, ldb, C, ldc, mode);
    if (rc != 0) return rc;
    void *ptr = nullptr;
    rc = static_scratch(&ptr);
    if (rc != 0) return rc;
    return run_sgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, mode,
                     config_id, group_m, stream, WS_STATIC, ptr, MISGEMM_STATIC_SCRATCH_BYTES,
                     splits);
}

int64_t misgemm_workspace_held(void)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -(int64_t)MISGEMM_E_NO_DEVICE;
    std::lock_guard<std::mutex> lock(g_ws_mutex);
    int64_t held = 0;
    for (const auto &kv : g_ws)
        if (kv.first.first == dev) held += kv.second.bytes + kv.second.retired_bytes;
    return held;
}

int misgemm_dgemm(char transa, char transb, int64_t m, int64_t n, int64_t k, double alpha,
                  const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
                  double *C, int64_t ldc, int dmode, void *stream)
{
    const int ta = trans_flag(transa), tb = trans_flag(transb);
    if (ta < 0) return -1;
    if (tb < 0) return -2;
    if (m < 0) return -3;
    if (n < 0) return -4;
    if (k < 0) return -5;
    const int64_t arows = ta ? k : m, acols = ta ? m : k;
    const int64_t brows = tb ? n : k, bcols = tb ? k : n;
    if (lda < std::max<int64_t>(1, arows)) return -8;
    if (ldb < std::max<int64_t>(1, brows)) return -10;
    if (ldc < std::max<int64_t>(1, m)) return -13;
    if (dmode != MISGEMM_D_FP64 && dmode != MISGEMM_D_FP32) return -14;
    const bool work = m > 0 && n > 0;
    const bool reads_ab = work && k > 0 && alpha != 0.0;
    if (reads_ab && A == nullptr) return -7;
    if (reads_ab && B == nullptr) return -9;
    if (work && C == nullptr) return -12;
    if (m > (int64_t)1 << 40 || n > (int64_t)1 << 40 || k > (int64_t)1 << 40)
        return MISGEMM_E_TOO_LARGE;
    if (!work) return 0;
    if ((alpha == 0.0 || k == 0) && beta == 1.0) return 0;
    DeviceInfo *dev = nullptr;
    int rc = current_device(&dev);
    if (rc != 0) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (alpha == 0.0 || k == 0) return (int)launch_dscale(beta, C, m, n, ldc, s);
    if (dmode == MISGEMM_D_FP64)
        return (int)launch_dgemm_fp64(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                                      dev->cus, s);
    // FP32 compute: narrow the stored operands (every element up to the last
    // used one, padding included), sgemm into an m x n FP32 product, widen
    // with alpha and beta applied in FP64.
    const int64_t na = lda * (acols - 1) + arows, nb = ldb * (bcols - 1) + brows;
    const int64_t a_bytes = (na * 4 + 255) / 256 * 256, b_bytes = (nb * 4 + 255) / 256 * 256;
    char *ws = nullptr;
    rc = library_workspace(a_bytes + b_bytes + m * n * 4, s, (void **)&ws);
    if (rc != 0) return rc;
    float *a32 = (float *)ws, *b32 = (float *)(ws + a_bytes), *p32 = (float *)(ws + a_bytes + b_bytes);
    hipError_t e = launch_narrow(A, na, a32, s);
    if (e == hipSuccess) e = launch_narrow(B, nb, b32, s);
    if (e != hipSuccess) return (int)e;
    rc = run_sgemm(transa, transb, m, n, k, 1.0f, a32, lda, b32, ldb, 0.0f, p32, m,
                   MISGEMM_FP32, -1, 0, stream, WS_NONE, nullptr, 0, 1);
    if (rc != 0) return rc;
    return (int)launch_widen(p32, m, n, alpha, beta, C, ldc, s);
}

int64_t misgemm_workspace_size(char transa, char transb, int64_t m, int64_t n, int64_t k,
                               int mode)
{
    if (trans_flag(transa) < 0) return -1;
    if (trans_flag(transb) < 0) return -2;
    if (m < 0) return -3;
    if (n < 0) return -4;
    if (k < 0) return -5;
    if (mode != MISGEMM_FP32 && mode != MISGEMM_BF16X3) return -6;
    if (mode == MISGEMM_FP32 || m == 0 || n == 0 || k == 0) return 0;
    return packed_bytes(m, n, k);
}

int misgemm_sgemm_ws(char transa, char transb, int64_t m, int64_t n, int64_t k, float alpha,
                     const float *A, int64_t lda, const float *B, int64_t ldb, float beta,
                     float *C, int64_t ldc, int mode, void *workspace, int64_t workspace_bytes,
                     void *stream)
{
    int rc = validate(transa, transb, m, n, k, alpha, A, lda, B, ldb, C, ldc, mode);
    if (rc != 0) return rc;
    if (workspace == nullptr)
        return run_sgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, mode, -1,
                         0, stream, WS_NONE);
    if (((uintptr_t)workspace & 15u) != 0) return -15;
    if (mode == MISGEMM_BF16X3 && m > 0 && n > 0 && k > 0 &&
        workspace_bytes < packed_bytes(m, n, k))
        return -16;
    return run_sgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, mode, -1, 0,
                     stream, WS_CALLER, workspace, workspace_bytes);
}

int misgemm_release_workspace(void)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MISGEMM_E_NO_DEVICE;
    hipError_t e = hipDeviceSynchronize();
    std::lock_guard<std::mutex> lock(g_ws_mutex);
    for (auto it = g_ws.begin(); it != g_ws.end();) {
        if (it->first.first != dev) { ++it; continue; }
        StreamWorkspace &w = it->second;
        if (w.ptr) (void)hipFree(w.ptr);
        for (void *p : w.retired) (void)hipFree(p);
        it = g_ws.erase(it);
    }
    return (int)e;
}

int misgemm_num_configs(void) { return (int)configs().size(); }

int misgemm_config_info(int id, misgemm_config_desc *out)
{
    if (id < 0 || id >= (int)configs().size()) return -1;
    if (out == nullptr) return -2;
    *out = configs()[id].desc;
    out->splitk = configs()[id].splitk[0][0] != nullptr;
    return 0;
}

int misgemm_select_config(char transa, char transb, int64_t m, int64_t n, int64_t k, int mode)
{
    const int ta = trans_flag(transa), tb = trans_flag(transb);
    if (ta < 0) return -1;
    if (tb < 0) return -2;
    if (m < 0) return -3;
    if (n < 0) return -4;
    if (k < 0) return -5;
    if (mode != MISGEMM_FP32 && mode != MISGEMM_BF16X3) return -6;
    DeviceInfo *dev = nullptr;
    int cus = 256;
    if (current_device(&dev) == 0) cus = dev->cus;
    int gm = 0, splits = 0;
    return select_config(mode, ta, tb, m, n, k, cus, false, &gm, &splits);
}

int misgemm_load_tuning(const char *path)
{
    std::vector<TuneEntry> entries;
    int batch_cfg[2] = {-1, -1};
    BatchRule batch_rule[2] = {{0, -1, -1}, {0, -1, -1}};
    if (path != nullptr) {
        FILE *f = fopen(path, "r");
        if (!f) return MISGEMM_E_TUNING_FILE;
        char line[512];
        bool header = false;
        int rc = 0;
        while (fgets(line, sizeof line, f)) {
            if (line[0] == '#' || line[0] == '\n') continue;
            if (!header) {
                if (strncmp(line, "misgemm-tuning 1", 16) != 0) { rc = MISGEMM_E_TUNING_FILE; break; }
                header = true;
                continue;
            }
            char name[64];
            int mode;
            if (strncmp(line, "batch2 ", 7) == 0) {
                char name2[64];
                int thr = 0;
                if (sscanf(line + 7, "%d %d %63s %63s", &mode, &thr, name, name2) != 4 ||
                    mode < 0 || mode > 1 || thr <= 0) {
                    rc = MISGEMM_E_TUNING_FILE;
                    break;
                }
                const int b = find_config(name), sm = find_config(name2);
                if (b < 0 || sm < 0 || configs()[b].desc.mode != mode ||
                    configs()[sm].desc.mode != mode || !has_batch(configs()[b]) ||
                    !has_batch(configs()[sm])) {
                    rc = MISGEMM_E_TUNING_FILE;
                    break;
                }
                batch_rule[mode] = {thr, b, sm};
                continue;
            }
            if (strncmp(line, "batch ", 6) == 0) {
                if (sscanf(line + 6, "%d %63s", &mode, name) != 2 || mode < 0 || mode > 1) {
                    rc = MISGEMM_E_TUNING_FILE;
                    break;
                }
                const int id = find_config(name);
                if (id < 0 || configs()[id].desc.mode != mode || !has_batch(configs()[id])) {
                    rc = MISGEMM_E_TUNING_FILE;
                    break;
                }
                batch_cfg[mode] = id;
                continue;
            }
            char ta, tb;
            long long m, n, k;
            int gm = GROUP_M_DEFAULT, sp = 0;
            const int got = sscanf(line, "%d %c %c %lld %lld %lld %63s %d %d", &mode, &ta, &tb,
                                   &m, &n, &k, name, &gm, &sp);
            if (got < 7 || m <= 0 || n <= 0 || k <= 0 || trans_flag(ta) < 0 ||
                trans_flag(tb) < 0 || gm <= 0 || gm > 4096 || sp < 0 || sp > 64) {
                rc = MISGEMM_E_TUNING_FILE;
                break;
            }
            const int id = find_config(name);
            if (id < 0 || configs()[id].desc.mode != mode ||
                (sp > 1 && configs()[id].splitk[0][0] == nullptr)) {
                rc = MISGEMM_E_TUNING_FILE;
                break;
            }
            entries.push_back({mode, trans_flag(ta), trans_flag(tb), m, n, k, id, gm, sp});
        }
        fclose(f);
        if (rc == 0 && !header) rc = MISGEMM_E_TUNING_FILE;
        if (rc != 0) return rc;
    }
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tuning.swap(entries);
    g_batch_config[0] = batch_cfg[0];
    g_batch_config[1] = batch_cfg[1];
    g_batch_rule[0] = batch_rule[0];
    g_batch_rule[1] = batch_rule[1];
    return 0;
}

int misgemm_batch_plan(const misgemm_problem *problems, int64_t count, int mode, int config_id,
                       misgemm_batch **plan, int64_t *bad_index)
{
    if (bad_index) *bad_index = -1;
    if (plan == nullptr) return MISGEMM_E_NULL_PLAN;
    *plan = nullptr;
    if (count < 0 || (count > 0 && problems == nullptr)) return MISGEMM_E_BATCH;
    if (mode != MISGEMM_FP32 && mode != MISGEMM_BF16X3) return -14;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(nullptr, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone)
        return MISGEMM_E_CAPTURING;
    DeviceInfo *dev = nullptr;
    int rc = current_device(&dev);
    if (rc != 0) return rc;
    const auto &table = configs();

    // configuration: explicit, else the heuristic/tuned choice for the
    // problem carrying the most work, among configs with a batched variant
    int cfg = config_id;
    if (cfg >= 0) {
        if (cfg >= (int)table.size() || table[cfg].desc.mode != mode || !has_batch(table[cfg]))
            return MISGEMM_E_BAD_CONFIG;
    } else {
        {
            std::lock_guard<std::mutex> lock(g_tune_mutex);
            cfg = g_batch_config[mode];
        }
        int64_t smallest = INT64_MAX;
        for (size_t i = 0; i < table.size(); ++i) {
            const misgemm_config_desc &d = table[i].desc;
            if (d.mode != mode || !has_batch(table[i])) continue;
            // default: the 128x128 tile if compiled, else the smallest
            const int64_t area = (int64_t)d.bm * d.bn;
            if (d.bm == 128 && d.bn == 128 && cfg < 0) cfg = (int)i;
            if (area < smallest) smallest = area;
        }
        if (cfg < 0)
            for (size_t i = 0; i < table.size(); ++i)
                if (table[i].desc.mode == mode && has_batch(table[i]) &&
                    (int64_t)table[i].desc.bm * table[i].desc.bn == smallest) { cfg = (int)i; break; }
        if (cfg < 0) return MISGEMM_E_BAD_CONFIG;
    }
    for (int64_t i = 0; i < count; ++i) {
        const misgemm_problem &p = problems[i];
        rc = validate(p.transa, p.transb, p.m, p.n, p.k, p.alpha, p.A, p.lda, p.B, p.ldb, p.C,
                      p.ldc, mode);
        if (rc != 0) {
            if (bad_index) *bad_index = i;
            return rc;
        }
    }
    // A tuned two-part rule (no explicit config): the problems with m and n
    // at or above the threshold on one configuration, the rest on another,
    // launched concurrently; with only one side present, its configuration.
    BatchRule rule = {0, -1, -1};
    if (config_id < 0) {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        rule = g_batch_rule[mode];
    }
    std::vector<int64_t> all, big, small;
    for (int64_t i = 0; i < count; ++i) {
        all.push_back(i);
        if (rule.big >= 0)
            (problems[i].m >= rule.threshold && problems[i].n >= rule.threshold ? big : small)
                .push_back(i);
    }
    if (rule.big >= 0 && (big.empty() || small.empty()))
        return build_part(problems, all, mode, big.empty() ? rule.small : rule.big, dev, plan,
                          bad_index);
    if (rule.big < 0) return build_part(problems, all, mode, cfg, dev, plan, bad_index);
    misgemm_batch *p1 = nullptr, *p2 = nullptr;
    rc = build_part(problems, big, mode, rule.big, dev, &p1, bad_index);
    if (rc == 0) rc = build_part(problems, small, mode, rule.small, dev, &p2, bad_index);
    if (rc == 0) {
        p1->second = p2;
        p1->count = count;
        if (hipStreamCreateWithFlags(&p1->side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&p1->fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&p1->join, hipEventDisableTiming) != hipSuccess)
            rc = MISGEMM_E_NO_DEVICE;
    }
    if (rc != 0) {
        if (p1) misgemm_batch_destroy(p1);
        else if (p2) misgemm_batch_destroy(p2);
        return rc;
    }
    *plan = p1;
    return 0;
}

int misgemm_batch_launch(const misgemm_batch *plan, void *stream)
{
    if (plan == nullptr) return MISGEMM_E_NULL_PLAN;
    const hipStream_t s = (hipStream_t)stream;
    auto run = [](const misgemm_batch *p, hipStream_t st) -> int {
        if (p->ntiles == 0) return 0;
        const ConfigEntry &c = configs()[p->config_id];
        if (p->packed) {
            const hipError_t e = launch_pack_batch(p->d_jobs, p->njobs, p->pack_blocks, st);
            if (e != hipSuccess) return (int)e;
            return (int)c.packed_batch(p->d_pprobs, p->d_tiles, p->split, p->grid, st);
        }
        return (int)c.batch(p->d_probs, p->d_tiles, p->split, p->grid, st);
    };
    if (plan->second == nullptr) return run(plan, s);
    // fork the second part onto the plan's side stream and join it back, so
    // that the launch stays one unit on `stream` (and one graph when captured)
    hipError_t e = hipEventRecord(plan->fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(plan->side, plan->fork, 0);
    if (e != hipSuccess) return (int)e;
    int rc = run(plan, s);
    const int rc2 = run(plan->second, plan->side);
    if (rc == 0) rc = rc2;
    e = hipEventRecord(plan->join, plan->side);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, plan->join, 0);
    return rc != 0 ? rc : (int)e;
}

int misgemm_batch_info(const misgemm_batch *plan, misgemm_batch_desc *out)
{
    if (plan == nullptr) return MISGEMM_E_NULL_PLAN;
    if (out == nullptr) return -2;
    const misgemm_batch *q = plan->second;
    out->count = plan->count;
    out->tiles = plan->ntiles + (q ? q->ntiles : 0);
    out->grid = plan->grid;
    out->config_id = plan->config_id;
    out->flops = plan->flops + (q ? q->flops : 0.0);
    out->tile_flops = plan->tile_flops + (q ? q->tile_flops : 0.0);
    out->parts = plan->split.nx;
    out->part_imbalance = plan->part_imbalance;
    out->second_config_id = q ? q->config_id : -1;
    out->second_grid = q ? q->grid : 0;
    out->panel_bytes = plan->panel_bytes + (q ? q->panel_bytes : 0);
    return 0;
}

int misgemm_batch_destroy(misgemm_batch *plan)
{
    if (plan == nullptr) return MISGEMM_E_NULL_PLAN;
    hipError_t e = hipDeviceSynchronize();
    if (plan->second) misgemm_batch_destroy(plan->second);
    if (plan->fork) (void)hipEventDestroy(plan->fork);
    if (plan->join) (void)hipEventDestroy(plan->join);
    if (plan->side) (void)hipStreamDestroy(plan->side);
    if (plan->d_probs) (void)hipFree(plan->d_probs);
    if (plan->d_tiles) (void)hipFree(plan->d_tiles);
    if (plan->d_pprobs) (void)hipFree(plan->d_pprobs);
    if (plan->d_jobs) (void)hipFree(plan->d_jobs);
    if (plan->d_panels) (void)hipFree(plan->d_panels);
    free(plan);
    return (int)e;
}

int misgemm_bf16x3_split(const float *x, int64_t count, uint16_t *parts, void *stream)
{
    if (x == nullptr && count > 0) return -1;
    if (count < 0) return -2;
    if (parts == nullptr && count > 0) return -3;
    if (count == 0) return 0;
    DeviceInfo *dev = nullptr;
    const int rc = current_device(&dev);
    if (rc != 0) return rc;
    return (int)launch_split(x, count, parts, (hipStream_t)stream);
}

const char *misgemm_status_string(int status)
{
    static thread_local char buf[160];
    if (status == 0) return "success";
    if (status < 0) {
        snprintf(buf, sizeof buf, "invalid argument at position %d", -status);
        return buf;
    }
    switch (status) {
    case MISGEMM_E_NO_DEVICE: return "no gfx950 (MI355X) device is current";
    case MISGEMM_E_BAD_CONFIG: return "unknown kernel configuration for this mode";
    case MISGEMM_E_CAPTURING: return "call not allowed while a stream is capturing";
    case MISGEMM_E_TUNING_FILE: return "tuning file unreadable or malformed";
    case MISGEMM_E_BATCH: return "invalid batch description";
    case MISGEMM_E_NULL_PLAN: return "batch plan pointer is NULL";
    case MISGEMM_E_TOO_LARGE: return "a size exceeds the supported range";
    case MISGEMM_E_SCRATCH:
        return "split-K partial tiles exceed the static scratch (MISGEMM_STATIC_SCRATCH_BYTES)";
    default: break;
    }
    if (status < 1000) {
        snprintf(buf, sizeof buf, "HIP error %d: %s", status,
                 hipGetErrorString((hipError_t)status));
        return buf;
    }
    snprintf(buf, sizeof buf, "unknown status %d", status);
    return buf;
}

const char *misgemm_version(void) { return "misgemm 0.2 (gfx950)"; }

}  // extern "C"
