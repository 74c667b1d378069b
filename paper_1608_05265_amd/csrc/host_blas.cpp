// Host-pointer BLAS entry points: the classic Fortran sgemm_/dgemm_ symbols
// (every argument by reference) and their C forms with a status code.  The
// paper's library served unmodified BLAS callers and overlapped the
// host/co-processor transfers with the multiplications (Sections III-A and
// III-C); here the operands travel over PCIe into HBM, C is cut into column
// panels, and panel p+1 is copied in while panel p is multiplied and panel
// p-1 is copied back.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/misgemm.h"

namespace {

int trans_of(char t)
{
    if (t == 'N' || t == 'n') return 0;
    if (t == 'T' || t == 't' || t == 'C' || t == 'c') return 1;
    return -1;
}

// Per-device state: three streams (copies in, compute, copies out), grow-only device buffers
// for A, B and C, and grow-only pinned host buffers (two for C panels on
// their way in, two on their way out, two chunks through which A and B
// travel).  Calls on one device are serialized.
constexpr int NPIN = 6;
constexpr int HOST_COPY_THREADS = 8;               // host threads per large copy (16 measured no faster)
constexpr int PIN_UPLOAD = 4;                      // first of the two upload chunks
constexpr size_t UPLOAD_CHUNK = (size_t)64 << 20;  // bytes per upload chunk
struct HostState {
    std::mutex mu;
    bool init = false;
    hipStream_t copy = nullptr, comp = nullptr, out = nullptr;  // copies in, compute, copies out
    void *buf[3] = {nullptr, nullptr, nullptr};
    size_t cap[3] = {0, 0, 0};
    void *pin[NPIN] = {};
    size_t pin_cap[NPIN] = {};
};
constexpr int MAX_DEV = 64;
HostState g_host[MAX_DEV];

int ensure(HostState &h, int which, size_t bytes, void **out)
{
    if (h.cap[which] < bytes) {
        if (h.buf[which]) (void)hipFree(h.buf[which]);
        h.buf[which] = nullptr;
        h.cap[which] = 0;
        hipError_t e = hipMalloc(&h.buf[which], bytes);
        if (e != hipSuccess) return (int)e;
        h.cap[which] = bytes;
    }
    *out = h.buf[which];
    return 0;
}

// Pinned host buffer `which` of at least `bytes` (hipHostMalloc; the old one
// is freed after the copy stream has drained, so no transfer still uses it).
int ensure_pinned(HostState &h, int which, size_t bytes, void **out)
{
    if (h.pin_cap[which] < bytes) {
        if (h.pin[which]) {
            hipError_t e = hipStreamSynchronize(h.copy);
            if (e == hipSuccess) e = hipStreamSynchronize(h.out);
            if (e == hipSuccess) e = hipHostFree(h.pin[which]);
            if (e != hipSuccess) return (int)e;
        }
        h.pin[which] = nullptr;
        h.pin_cap[which] = 0;
        const hipError_t e = hipHostMalloc(&h.pin[which], bytes, hipHostMallocDefault);
        if (e != hipSuccess) return (int)e;
        h.pin_cap[which] = bytes;
    }
    *out = h.pin[which];
    return 0;
}

// The m rows of columns [0, cols) of a column-major host block (leading
// dimension ld) to or from a contiguous m x cols buffer, on several host
// threads for large blocks (plain memcpy per column).
template <class T>
void gather_columns(T *dst, const T *src, int64_t m, int64_t cols, int64_t ld, bool to_packed)
{
    const int64_t bytes = m * cols * (int64_t)sizeof(T);
    const int nt = bytes >= ((int64_t)8 << 20) ? HOST_COPY_THREADS : 1;
    auto work = [&](int t) {
        for (int64_t c = t; c < cols; c += nt) {
            if (to_packed) memcpy(dst + c * m, src + c * ld, (size_t)m * sizeof(T));
            else memcpy(dst + c * ld, src + c * m, (size_t)m * sizeof(T));
        }
    };
    if (nt == 1) {
        work(0);
        return;
    }
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) pool.emplace_back(work, t);
    work(0);
    for (auto &th : pool) th.join();
}

// bytes from src to dst on several host threads for large copies.
void parallel_memcpy(char *dst, const char *src, size_t bytes)
{
    const int nt = bytes >= ((size_t)8 << 20) ? HOST_COPY_THREADS : 1;
    const size_t part = (bytes / nt + 4095) / 4096 * 4096;
    auto work = [&](int t) {
        const size_t off = std::min(bytes, (size_t)t * part);
        const size_t len = std::min(part, bytes - off);
        if (len > 0) memcpy(dst + off, src + off, len);
    };
    if (nt == 1) {
        work(0);
        return;
    }
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) pool.emplace_back(work, t);
    work(0);
    for (auto &th : pool) th.join();
}

// The two pinned chunks through which read-only operands travel: host
// threads copy chunk i of the caller's (pageable) range into chunk buffer
// i % 2, once the transfer of chunk i-2 out of it has finished, and the DMA
// engine moves it to the device on the copy stream while the host fills the
// other buffer (handing pageable memory to the runtime directly moved about
// 20 GB/s).
struct Uploader {
    HostState &h;
    size_t chunk = 0;  // bytes per chunk (the pinned buffers hold at least this)
    hipEvent_t done[2] = {nullptr, nullptr};
    bool used[2] = {false, false};
    int next = 0;
    explicit Uploader(HostState &hs) : h(hs) {}
    ~Uploader()
    {
        for (hipEvent_t ev : done)
            if (ev) (void)hipEventDestroy(ev);
    }
    hipError_t init()
    {
        hipError_t e = hipSuccess;
        for (int i = 0; i < 2 && e == hipSuccess; ++i)
            e = hipEventCreateWithFlags(&done[i], hipEventDisableTiming);
        return e;
    }
    hipError_t put(void *dst, const void *src, size_t bytes)
    {
        for (size_t off = 0; off < bytes; off += chunk) {
            const size_t len = std::min(chunk, bytes - off);
            const int s = next;
            next ^= 1;
            if (used[s]) {
                const hipError_t e = hipEventSynchronize(done[s]);
                if (e != hipSuccess) return e;
            }
            char *pin = (char *)h.pin[PIN_UPLOAD + s];
            parallel_memcpy(pin, (const char *)src + off, len);
            hipError_t e = hipMemcpyAsync((char *)dst + off, pin, len, hipMemcpyHostToDevice, h.copy);
            if (e == hipSuccess) e = hipEventRecord(done[s], h.copy);
            if (e != hipSuccess) return e;
            used[s] = true;
        }
        return hipSuccess;
    }
};

// Copy the rows x cols column-major block with leading dimension ld
// between host and device, keeping the same leading dimension on the
// device.  Never past the last column's last row.  An operand that is only
// read may travel as one contiguous range, padding rows included (one large
// transfer instead of one per column); C (may_touch_padding false) moves
// as rows x cols, so that padding rows of the host C -- which may belong to
// a larger matrix that other code is using -- are never written.
template <class T>
hipError_t copy_block(T *dst, const T *src, int64_t rows, int64_t cols, int64_t ld,
                      hipMemcpyKind kind, hipStream_t s, bool may_touch_padding)
{
    if (rows == 0 || cols == 0) return hipSuccess;
    if (ld == rows || may_touch_padding)
        return hipMemcpyAsync(dst, src, (size_t)(ld * (cols - 1) + rows) * sizeof(T), kind, s);
    return hipMemcpy2DAsync(dst, (size_t)ld * sizeof(T), src, (size_t)ld * sizeof(T),
                            (size_t)rows * sizeof(T), (size_t)cols, kind, s);
}

// Panels of C columns: about four when n is large, so that copies overlap
// the multiplications, each at least 256 columns wide.
int64_t panel_width(int64_t n)
{
    if (n < 1024) return std::max<int64_t>(n, 1);
    return (n + 3) / 4;
}

template <class T, class GEMM>
int host_gemm(char transa, char transb, int64_t m, int64_t n, int64_t k, T alpha,
              const T *A, int64_t lda, const T *B, int64_t ldb, T beta, T *C, int64_t ldc,
              GEMM gemm)
{
    const int ta = trans_of(transa), tb = trans_of(transb);
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
    const bool reads_ab = m > 0 && n > 0 && k > 0 && alpha != T(0);
    if (reads_ab && A == nullptr) return -7;
    if (reads_ab && B == nullptr) return -9;
    if (m > 0 && n > 0 && C == nullptr) return -12;
    if (m == 0 || n == 0) return 0;
    if (!reads_ab && beta == T(1)) return 0;

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEV) return MISGEMM_E_NO_DEVICE;
    HostState &h = g_host[dev];
    std::lock_guard<std::mutex> lock(h.mu);
    if (!h.init) {
        if (hipStreamCreateWithFlags(&h.copy, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&h.comp, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&h.out, hipStreamNonBlocking) != hipSuccess)
            return MISGEMM_E_NO_DEVICE;
        h.init = true;
    }
    void *dA = nullptr, *dB = nullptr, *dC = nullptr;
    int rc = 0;
    if (reads_ab) {
        rc = ensure(h, 0, (size_t)(lda * (acols - 1) + arows) * sizeof(T), &dA);
        if (rc == 0) rc = ensure(h, 1, (size_t)(ldb * (bcols - 1) + brows) * sizeof(T), &dB);
    }
    if (rc == 0) rc = ensure(h, 2, (size_t)(ldc * (n - 1) + m) * sizeof(T), &dC);
    if (rc != 0) return rc;
    T *a = (T *)dA, *b = (T *)dB, *c = (T *)dC;

    hipError_t e = hipSuccess;
    const int64_t nb = panel_width(n);
    const int64_t panels = (n + nb - 1) / nb;
    // C's panels go through pinned buffers, gathered and scattered by host
    // threads (only the m rows of each column: the padding of a host C may
    // belong to a larger matrix and must not be written), so the DMA engines
    // move contiguous pinned data: a column-wise copy from pageable memory
    // ran at 4-6 GB/s, a contiguous one (tight ldc) at about 20 GB/s.  Panel
    // p's gather happens while panel p-1 is multiplied, its scatter while
    // panel p+1 is.
    const bool staged = true;
    T *pin_in[2] = {nullptr, nullptr}, *pin_out[2] = {nullptr, nullptr};
    if (staged) {
        const size_t pbytes = (size_t)m * nb * sizeof(T);
        for (int i = 0; i < 4 && rc == 0; ++i) {
            void *ptr = nullptr;
            if (i < 2 && beta == T(0)) continue;  // C0 is not read
            rc = ensure_pinned(h, i, pbytes, &ptr);
            (i < 2 ? pin_in[i] : pin_out[i - 2]) = (T *)ptr;
        }
        if (rc != 0) return rc;
    }
    // A whole; B whole when its stored columns are not C's columns (transb);
    // both are only read, so they travel as contiguous ranges (padding rows
    // included) through the pinned upload chunks
    Uploader up(h);
    if (reads_ab) {
        // chunks of UPLOAD_CHUNK bytes, smaller when the largest single
        // transfer (A, B whole, or one panel of B) is smaller
        const size_t a_bytes = (size_t)(lda * (acols - 1) + arows) * sizeof(T);
        const size_t b_bytes = tb ? (size_t)(ldb * (bcols - 1) + brows) * sizeof(T)
                                  : (size_t)(ldb * (std::min(nb, n) - 1) + brows) * sizeof(T);
        up.chunk = std::min(UPLOAD_CHUNK, std::max(a_bytes, b_bytes));
        for (int i = 0; i < 2 && rc == 0; ++i) {
            void *ptr = nullptr;
            rc = ensure_pinned(h, PIN_UPLOAD + i, up.chunk, &ptr);
        }
        if (rc != 0) return rc;
        e = up.init();
        if (e == hipSuccess)
            e = up.put(a, A, (size_t)(lda * (acols - 1) + arows) * sizeof(T));
        if (e == hipSuccess && tb)
            e = up.put(b, B, (size_t)(ldb * (bcols - 1) + brows) * sizeof(T));
    }
    constexpr int nev = 4;
    hipEvent_t in_done[nev] = {}, out_done[nev] = {}, pin_free[2] = {}, pin_full[2] = {};
    for (int i = 0; i < nev && e == hipSuccess; ++i) {
        e = hipEventCreateWithFlags(&in_done[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&out_done[i], hipEventDisableTiming);
    }
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipEventCreateWithFlags(&pin_free[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&pin_full[i], hipEventDisableTiming);
    }
    bool pin_in_used[2] = {false, false};
    auto scatter = [&](int64_t q) -> hipError_t {
        // panel q's result, copied into pin_out[q % 2], to the host C
        const int64_t q0 = q * nb, qc = std::min(nb, n - q0);
        const hipError_t se = hipEventSynchronize(pin_full[q % 2]);
        if (se == hipSuccess) gather_columns(C + q0 * ldc, pin_out[q % 2], m, qc, ldc, false);
        return se;
    };
    for (int64_t p = 0; p < panels && e == hipSuccess && rc == 0; ++p) {
        const int64_t j0 = p * nb, cols = std::min(nb, n - j0);
        const int slot = (int)(p % nev), ps = (int)(p % 2);
        // stage panel p (its own device columns, so no panel waits for
        // another): B columns (transb = N), C columns when beta != 0
        if (reads_ab && !tb)
            e = up.put(b + j0 * ldb, B + j0 * ldb, (size_t)(ldb * (cols - 1) + brows) * sizeof(T));
        if (e == hipSuccess && beta != T(0)) {
            if (staged) {
                // the pinned buffer's previous transfer (panel p-2) must be done
                if (pin_in_used[ps]) e = hipEventSynchronize(pin_free[ps]);
                if (e == hipSuccess) {
                    gather_columns(pin_in[ps], C + j0 * ldc, m, cols, ldc, true);
                    e = hipMemcpy2DAsync(c + j0 * ldc, (size_t)ldc * sizeof(T), pin_in[ps],
                                         (size_t)m * sizeof(T), (size_t)m * sizeof(T),
                                         (size_t)cols, hipMemcpyHostToDevice, h.copy);
                }
                if (e == hipSuccess) e = hipEventRecord(pin_free[ps], h.copy);
                pin_in_used[ps] = true;
            } else {
                e = copy_block(c + j0 * ldc, C + j0 * ldc, m, cols, ldc, hipMemcpyHostToDevice,
                               h.copy, false);
            }
        }
        if (e == hipSuccess) e = hipEventRecord(in_done[slot], h.copy);
        if (e == hipSuccess) e = hipStreamWaitEvent(h.comp, in_done[slot], 0);
        if (e != hipSuccess) break;
        // multiply panel p on the compute stream
        const T *bp = tb ? b + j0 : b + j0 * ldb;  // op(B)(:, j0:j0+cols)
        rc = gemm(transa, transb, m, cols, k, alpha, a, lda, bp, ldb, beta, c + j0 * ldc, ldc,
                  (void *)h.comp);
        if (rc != 0) break;
        // copy panel p back on its own stream (only its m rows: the host
        // padding stays untouched), so the next panel's inputs need not wait
        // for it
        e = hipEventRecord(out_done[slot], h.comp);
        if (e == hipSuccess) e = hipStreamWaitEvent(h.out, out_done[slot], 0);
        if (e == hipSuccess) {
            if (staged) {
                e = hipMemcpy2DAsync(pin_out[ps], (size_t)m * sizeof(T), c + j0 * ldc,
                                     (size_t)ldc * sizeof(T), (size_t)m * sizeof(T),
                                     (size_t)cols, hipMemcpyDeviceToHost, h.out);
                if (e == hipSuccess) e = hipEventRecord(pin_full[ps], h.out);
                // the previous panel's result goes to C while this one is computed
                if (e == hipSuccess && p > 0) e = scatter(p - 1);
            } else {
                e = copy_block(C + j0 * ldc, c + j0 * ldc, m, cols, ldc, hipMemcpyDeviceToHost,
                               h.out, false);
            }
        }
    }
    if (staged && e == hipSuccess && rc == 0 && panels > 0) e = scatter(panels - 1);
    const hipError_t s1 = hipStreamSynchronize(h.comp), s2 = hipStreamSynchronize(h.copy);
    const hipError_t s3 = hipStreamSynchronize(h.out);
    for (int i = 0; i < nev; ++i) {
        if (in_done[i]) (void)hipEventDestroy(in_done[i]);
        if (out_done[i]) (void)hipEventDestroy(out_done[i]);
    }
    for (int i = 0; i < 2; ++i) {
        if (pin_free[i]) (void)hipEventDestroy(pin_free[i]);
        if (pin_full[i]) (void)hipEventDestroy(pin_full[i]);
    }
    if (rc != 0) return rc;
    if (e != hipSuccess) return (int)e;
    if (s1 != hipSuccess) return (int)s1;
    if (s2 != hipSuccess) return (int)s2;
    return (int)s3;
}

void report(const char *name, int rc)
{
    if (rc < 0)
        fprintf(stderr, " ** On entry to %s parameter number %d had an illegal value\n", name,
                -rc);
    else if (rc > 0)
        fprintf(stderr, " ** %s failed: %s\n", name, misgemm_status_string(rc));
}

int host_mode()
{
    const char *e = getenv("MISGEMM_SGEMM_MODE");
    return e && strcmp(e, "bf16x3") == 0 ? MISGEMM_BF16X3 : MISGEMM_FP32;
}

}  // namespace

extern "C" {

int misgemm_sgemm_host(char transa, char transb, int64_t m, int64_t n, int64_t k, float alpha,
                       const float *A, int64_t lda, const float *B, int64_t ldb, float beta,
                       float *C, int64_t ldc, int mode)
{
    if (mode != MISGEMM_FP32 && mode != MISGEMM_BF16X3) return -14;
    return host_gemm<float>(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                            [mode](char ta, char tb, int64_t mm, int64_t nn, int64_t kk,
                                   float al, const float *a, int64_t la, const float *b,
                                   int64_t lb, float be, float *c, int64_t lc, void *s) {
                                return misgemm_sgemm(ta, tb, mm, nn, kk, al, a, la, b, lb, be,
                                                     c, lc, mode, s);
                            });
}

int misgemm_dgemm_host(char transa, char transb, int64_t m, int64_t n, int64_t k, double alpha,
                       const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
                       double *C, int64_t ldc, int dmode)
{
    if (dmode != MISGEMM_D_FP64 && dmode != MISGEMM_D_FP32) return -14;
    return host_gemm<double>(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                             [dmode](char ta, char tb, int64_t mm, int64_t nn, int64_t kk,
                                     double al, const double *a, int64_t la, const double *b,
                                     int64_t lb, double be, double *c, int64_t lc, void *s) {
                                 return misgemm_dgemm(ta, tb, mm, nn, kk, al, a, la, b, lb, be,
                                                      c, lc, dmode, s);
                             });
}

void sgemm_(const char *transa, const char *transb, const int *m, const int *n, const int *k,
            const float *alpha, const float *A, const int *lda, const float *B, const int *ldb,
            const float *beta, float *C, const int *ldc)
{
    report("SGEMM ", misgemm_sgemm_host(*transa, *transb, *m, *n, *k, *alpha, A, *lda, B, *ldb,
                                        *beta, C, *ldc, host_mode()));
}

void dgemm_(const char *transa, const char *transb, const int *m, const int *n, const int *k,
            const double *alpha, const double *A, const int *lda, const double *B,
            const int *ldb, const double *beta, double *C, const int *ldc)
{
    report("DGEMM ", misgemm_dgemm_host(*transa, *transb, *m, *n, *k, *alpha, A, *lda, B, *ldb,
                                        *beta, C, *ldc, MISGEMM_D_FP64));
}

}  // extern "C"
