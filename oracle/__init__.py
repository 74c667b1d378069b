"""CPU oracle for the single-precision GEMM problem: TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
use this package.  The GPU library never imports it, links it or calls it,
and it shares no code with the GPU library.

What it computes (Section III-A of the paper, restated for the inner
micro-kernel in Section III-C): ``C_out = alpha * op(A) * op(B) + beta * C_in``
for column-major FP32 storage with leading dimensions and N/T transposes, in
FP64, plus the error denominator ``den = |alpha| (|op(A)| |op(B)|) + |beta| |C_in|``.
The arithmetic lives in ``oracle_sgemm.c`` (plain loops, OpenMP over columns);
this module compiles it with gcc and exposes it through ``ctypes``.

Matrices are passed as the raw column-major storage: a 1-D float32 numpy
array in which element (r, c) sits at ``r + c * ld``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_sgemm.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

U32 = 2.0 ** -24  # unit roundoff of FP32 (round to nearest)
U64 = 2.0 ** -53  # unit roundoff of FP64


def build(force: bool = True) -> str:
    """Compile oracle_sgemm.c into liboracle.so next to it (gcc + OpenMP)."""
    global _lib
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    _lib = None
    return _LIB_PATH


def _bind(lib):
    i64, f32, i32 = ctypes.c_int64, ctypes.c_float, ctypes.c_int
    vp = ctypes.c_void_p
    lib.oracle_sgemm_f64.argtypes = [ctypes.c_char, ctypes.c_char, i64, i64, i64,
                                     f32, vp, i64, vp, i64, f32, vp, i64, vp, vp, i32]
    lib.oracle_sgemm_f64.restype = i32
    lib.oracle_sgemm_f64_entries.argtypes = [ctypes.c_char, ctypes.c_char, i64, i64, i64,
                                             f32, vp, i64, vp, i64, f32, vp, i64,
                                             i64, vp, vp, vp, vp, i32]
    lib.oracle_sgemm_f64_entries.restype = i32
    lib.oracle_sgemm_bf16x3_f64.argtypes = [ctypes.c_char, ctypes.c_char, i64, i64, i64,
                                            f32, vp, i64, vp, i64, f32, vp, i64, vp, i32]
    lib.oracle_sgemm_bf16x3_f64.restype = i32
    lib.oracle_bf16_rne.argtypes = [f32]
    lib.oracle_bf16_rne.restype = ctypes.c_uint16
    lib.oracle_bf16x3_split_array.argtypes = [vp, i64, vp]
    lib.oracle_bf16x3_split_array.restype = None
    lib.oracle_bf16x3_sweep.argtypes = [ctypes.c_uint64, ctypes.c_uint64, vp, vp, i32]
    lib.oracle_bf16x3_sweep.restype = None
    lib.oracle_bf16x3_split_digest.argtypes = [ctypes.c_uint64, ctypes.c_uint64, i32]
    lib.oracle_bf16x3_split_digest.restype = ctypes.c_uint64
    f64 = ctypes.c_double
    lib.oracle_dgemm_f128.argtypes = [ctypes.c_char, ctypes.c_char, i64, i64, i64,
                                      f64, vp, i64, vp, i64, f64, vp, i64, vp, vp, i32]
    lib.oracle_dgemm_f128.restype = i32
    lib.oracle_dgemm_f128_entries.argtypes = [ctypes.c_char, ctypes.c_char, i64, i64, i64,
                                              f64, vp, i64, vp, i64, f64, vp, i64,
                                              i64, vp, vp, vp, vp, i32]
    lib.oracle_dgemm_f128_entries.restype = i32
    lib.oracle_getrf_f64.argtypes = [i64, vp, i64, vp, vp, i32]
    lib.oracle_getrf_f64.restype = i32
    lib.oracle_getrs_f64.argtypes = [i64, vp, vp, vp]
    lib.oracle_getrs_f64.restype = i32
    lib.oracle_max_threads.argtypes = []
    lib.oracle_max_threads.restype = i32
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    if a is None:
        return None
    return np.ascontiguousarray(a, dtype=np.float32).reshape(-1)


def _f64(a):
    if a is None:
        return None
    return np.ascontiguousarray(a, dtype=np.float64).reshape(-1)


class Oracle:
    """The oracle functions bound to one compiled copy of oracle_sgemm.c.

    The default instance uses liboracle.so; tests also bind deliberately
    broken copies to show that the pins catch such mistakes.
    """

    def __init__(self, lib_path: str):
        self.path = lib_path
        self.lib = _bind(ctypes.CDLL(lib_path))

    def max_threads(self) -> int:
        return int(self.lib.oracle_max_threads())

    def sgemm_f64(self, transa: str, transb: str, m: int, n: int, k: int, alpha: float,
                  A: np.ndarray, lda: int, B: np.ndarray, ldb: int, beta: float,
                  C0: Optional[np.ndarray], ldc: int, nthreads: int = 0
                  ) -> Tuple[np.ndarray, np.ndarray]:
        """Return (Cref, den), each an (m, n) float64 array indexed [i, j].

        Section III-A: Cref = alpha*op(A)*op(B) + beta*C0 evaluated in FP64 from
        the FP32 inputs; den = |alpha|*(|op(A)||op(B)|) + |beta|*|C0|.
        """
        A, B, C0 = _f32(A), _f32(B), _f32(C0)
        cref = np.zeros((n, m), dtype=np.float64)  # column-major storage, ld = m
        den = np.zeros((n, m), dtype=np.float64)
        rc = self.lib.oracle_sgemm_f64(transa.encode(), transb.encode(), m, n, k, alpha,
                                       _ptr(A), lda, _ptr(B), ldb, beta, _ptr(C0), ldc,
                                       _ptr(cref), _ptr(den), nthreads)
        if rc != 0:
            raise ValueError("oracle_sgemm_f64 failed with code %d" % rc)
        return cref.T, den.T

    def sgemm_f64_entries(self, transa: str, transb: str, m: int, n: int, k: int,
                          alpha: float, A: np.ndarray, lda: int, B: np.ndarray, ldb: int,
                          beta: float, C0: Optional[np.ndarray], ldc: int,
                          rows: Sequence[int], cols: Sequence[int], nthreads: int = 0
                          ) -> Tuple[np.ndarray, np.ndarray]:
        """Oracle values (cref, den) at the entries (rows[e], cols[e])."""
        A, B, C0 = _f32(A), _f32(B), _f32(C0)
        r = np.ascontiguousarray(rows, dtype=np.int64)
        c = np.ascontiguousarray(cols, dtype=np.int64)
        cref = np.zeros(r.size, dtype=np.float64)
        den = np.zeros(r.size, dtype=np.float64)
        rc = self.lib.oracle_sgemm_f64_entries(transa.encode(), transb.encode(), m, n, k,
                                               alpha, _ptr(A), lda, _ptr(B), ldb, beta,
                                               _ptr(C0), ldc, r.size, _ptr(r), _ptr(c),
                                               _ptr(cref), _ptr(den), nthreads)
        if rc != 0:
            raise ValueError("oracle_sgemm_f64_entries failed with code %d" % rc)
        return cref, den

    def dgemm_f128(self, transa: str, transb: str, m: int, n: int, k: int, alpha: float,
                   A: np.ndarray, lda: int, B: np.ndarray, ldb: int, beta: float,
                   C0: Optional[np.ndarray], ldc: int, nthreads: int = 0
                   ) -> Tuple[np.ndarray, np.ndarray]:
        """Double-precision problem (Section IV-B): (Cref, den) as (m, n) float64
        arrays, evaluated in binary128 from the FP64 inputs and rounded once."""
        A, B, C0 = _f64(A), _f64(B), _f64(C0)
        cref = np.zeros((n, m), dtype=np.float64)
        den = np.zeros((n, m), dtype=np.float64)
        rc = self.lib.oracle_dgemm_f128(transa.encode(), transb.encode(), m, n, k, alpha,
                                        _ptr(A), lda, _ptr(B), ldb, beta, _ptr(C0), ldc,
                                        _ptr(cref), _ptr(den), nthreads)
        if rc != 0:
            raise ValueError("oracle_dgemm_f128 failed with code %d" % rc)
        return cref.T, den.T

    def dgemm_f128_entries(self, transa: str, transb: str, m: int, n: int, k: int,
                           alpha: float, A: np.ndarray, lda: int, B: np.ndarray, ldb: int,
                           beta: float, C0: Optional[np.ndarray], ldc: int,
                           rows: Sequence[int], cols: Sequence[int], nthreads: int = 0
                           ) -> Tuple[np.ndarray, np.ndarray]:
        """The dgemm oracle at the entries (rows[e], cols[e])."""
        A, B, C0 = _f64(A), _f64(B), _f64(C0)
        r = np.ascontiguousarray(rows, dtype=np.int64)
        c = np.ascontiguousarray(cols, dtype=np.int64)
        cref = np.zeros(r.size, dtype=np.float64)
        den = np.zeros(r.size, dtype=np.float64)
        rc = self.lib.oracle_dgemm_f128_entries(transa.encode(), transb.encode(), m, n, k,
                                                alpha, _ptr(A), lda, _ptr(B), ldb, beta,
                                                _ptr(C0), ldc, r.size, _ptr(r), _ptr(c),
                                                _ptr(cref), _ptr(den), nthreads)
        if rc != 0:
            raise ValueError("oracle_dgemm_f128_entries failed with code %d" % rc)
        return cref, den

    def getrf_f64(self, n: int, A: np.ndarray, lda: int, nthreads: int = 0):
        """LU with partial pivoting (Section IV-C, the factorization of the
        paper's Linpack run) of the n x n FP32 matrix, in FP64.

        Returns (LU as an (n, n) float64 array [i, j], ipiv int64 (0-based
        row swapped with row j at step j), info (0 or 1 + first zero pivot)).
        """
        A = _f32(A)
        lu = np.zeros((n, n), dtype=np.float64)  # column-major storage, ld = n
        ipiv = np.zeros(n, dtype=np.int64)
        info = self.lib.oracle_getrf_f64(n, _ptr(A), lda, _ptr(lu), _ptr(ipiv), nthreads)
        if info < 0:
            raise ValueError("oracle_getrf_f64 failed with code %d" % info)
        return lu.T, ipiv, int(info)

    def getrs_f64(self, lu: np.ndarray, ipiv: np.ndarray, b: np.ndarray) -> np.ndarray:
        """Solve A x = b from getrf_f64's factors (b is not modified)."""
        n = lu.shape[0]
        f = np.ascontiguousarray(np.asarray(lu, dtype=np.float64).T)  # column-major
        piv = np.ascontiguousarray(ipiv, dtype=np.int64)
        x = np.array(b, dtype=np.float64).reshape(-1).copy()
        rc = self.lib.oracle_getrs_f64(n, _ptr(f), _ptr(piv), _ptr(x))
        if rc != 0:
            raise ValueError("oracle_getrs_f64 failed with code %d" % rc)
        return x

    def sgemm_bf16x3_f64(self, transa: str, transb: str, m: int, n: int, k: int,
                         alpha: float, A: np.ndarray, lda: int, B: np.ndarray, ldb: int,
                         beta: float, C0: Optional[np.ndarray], ldc: int,
                         nthreads: int = 0) -> np.ndarray:
        """The split-precision method in FP64: six bf16 part products per term."""
        A, B, C0 = _f32(A), _f32(B), _f32(C0)
        cref = np.zeros((n, m), dtype=np.float64)
        rc = self.lib.oracle_sgemm_bf16x3_f64(transa.encode(), transb.encode(), m, n, k,
                                              alpha, _ptr(A), lda, _ptr(B), ldb, beta,
                                              _ptr(C0), ldc, _ptr(cref), nthreads)
        if rc != 0:
            raise ValueError("oracle_sgemm_bf16x3_f64 failed with code %d" % rc)
        return cref.T

    def bf16_rne(self, x: float) -> int:
        """bfloat16 bit pattern of round-to-nearest-even(x)."""
        return int(self.lib.oracle_bf16_rne(float(x)))

    def bf16x3_split(self, x: np.ndarray) -> np.ndarray:
        """uint16 array of shape x.shape + (3,): the three bf16 parts of each value."""
        flat = np.ascontiguousarray(x, dtype=np.float32).reshape(-1)
        parts = np.zeros((flat.size, 3), dtype=np.uint16)
        self.lib.oracle_bf16x3_split_array(_ptr(flat), flat.size, _ptr(parts))
        return parts.reshape(np.shape(x) + (3,))

    def bf16x3_sweep(self, lo: int = 0, hi: int = 1 << 32, nthreads: int = 0):
        """Exhaustive split-property sweep over bit patterns lo <= u < hi.

        Returns (checked, sum_failures, bound_failures, nonfinite,
        max|x1|/|x|, max|x2|/|x|).
        """
        counts = np.zeros(4, dtype=np.int64)
        rel = np.zeros(2, dtype=np.float64)
        self.lib.oracle_bf16x3_sweep(lo, hi, _ptr(counts), _ptr(rel), nthreads)
        return (int(counts[0]), int(counts[1]), int(counts[2]), int(counts[3]),
                float(rel[0]), float(rel[1]))

    def bf16x3_split_digest(self, lo: int, hi: int, nthreads: int = 0) -> int:
        """Sum mod 2^64 of (p0 | p1 << 16 | p2 << 32) * (2u + 1) over the bit
        patterns lo <= u < hi of the split's domain (finite, 2^-110 <= |x| <
        0x1.fefp127): a digest of the split for comparing implementations."""
        return int(self.lib.oracle_bf16x3_split_digest(lo, hi, nthreads))


def _default() -> Oracle:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or \
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        _lib = Oracle(_LIB_PATH)
    return _lib


def build_variant(source_text: str, out_path: str) -> str:
    """Compile a modified copy of the oracle source (used to show that the
    pins reject plausible mistakes) and bind it."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(source_text)
    subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                    "-o", out_path, src, "-lm"], check=True)
    return out_path


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()


def max_threads() -> int:
    return _default().max_threads()


def sgemm_f64(*args, **kw):
    return _default().sgemm_f64(*args, **kw)


def sgemm_f64_entries(*args, **kw):
    return _default().sgemm_f64_entries(*args, **kw)


def sgemm_bf16x3_f64(*args, **kw):
    return _default().sgemm_bf16x3_f64(*args, **kw)


def getrf_f64(*args, **kw):
    return _default().getrf_f64(*args, **kw)


def getrs_f64(*args, **kw):
    return _default().getrs_f64(*args, **kw)


def hpl_scaled_residual(A: np.ndarray, x: np.ndarray, b: np.ndarray, eps: float) -> float:
    """The residual check of the paper's Linpack run (Section IV-C, Table
    VII, its footnote): ||A x - b||_inf / (eps * (||A||_inf * ||x||_inf + ||b||_inf) * N),
    evaluated in FP64; A is the dense (n, n) matrix."""
    A = np.asarray(A, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    n = A.shape[0]
    r = np.max(np.abs(A @ x - b))
    norm_a = np.max(np.sum(np.abs(A), axis=1))
    return float(r / (eps * (norm_a * np.max(np.abs(x)) + np.max(np.abs(b))) * n))


def dgemm_f128(*args, **kw):
    return _default().dgemm_f128(*args, **kw)


def dgemm_f128_entries(*args, **kw):
    return _default().dgemm_f128_entries(*args, **kw)


def bf16_rne(x: float) -> int:
    return _default().bf16_rne(x)


def bf16x3_split(x: np.ndarray) -> np.ndarray:
    return _default().bf16x3_split(x)


def bf16x3_sweep(lo: int = 0, hi: int = 1 << 32, nthreads: int = 0):
    return _default().bf16x3_sweep(lo, hi, nthreads)


def bf16x3_split_digest(lo: int, hi: int, nthreads: int = 0) -> int:
    return _default().bf16x3_split_digest(lo, hi, nthreads)


def bf16_to_f32(h: np.ndarray) -> np.ndarray:
    """Widen bf16 bit patterns to float32 (exact)."""
    return (np.asarray(h, dtype=np.uint32) << 16).view(np.float32)


# --------------------------------------------------------------------------
# Acceptance metric (the bound every GPU result is held to).
# --------------------------------------------------------------------------

def tol(k: int) -> float:
    """Acceptance bound on the normalized error for a K-term sum.

    The target bound is 2*K*u (u = 2^-24).  A K-term FP32 dot product followed
    by the alpha scale, the beta scale and the final add has a worst-case
    error of (K + 3) u to first order, which exceeds 2*K*u only for K <= 2, so
    the bound used is max(2K, K + 3) * u: identical to 2*K*u for every K >= 3.
    """
    return max(2 * k, k + 3) * U32


def tol_d(k: int) -> float:
    """The same bound for an FP64 computation: max(2K, K + 3) * 2^-53."""
    return max(2 * k, k + 3) * U64


def tol_false_d(k: int) -> float:
    """Bound for the FP64 interface computed in FP32 (the paper's "false
    dgemm", Section IV-B): rounding a and b to FP32 (RNE, unit roundoff u)
    perturbs each product by at most (2u + u^2)|a||b|, and the FP32 sum of
    the rounded products is held to tol(k) times sum |fl(a)||fl(b)|, which
    is at most (1 + u)^2 sum |a||b|.  So the normalized error is at most
    tol(k) (1 + u)^2 + 2u + u^2 <= tol(k) (1 + 2^-22) + 2^-23 + 2^-47; the
    input-rounding term 2u is attained to within a factor 1 - 2^-22 by a
    one-term product whose factors both round down by almost u (pinned).
    """
    return tol(k) * (1.0 + 2.0 ** -22) + 2.0 ** -23 + 2.0 ** -47


def normalized_error(C: np.ndarray, cref: np.ndarray, den: np.ndarray):
    """Elementwise |C - Cref| / den, with den == 0 mapped to 0 where C == Cref
    exactly and to +inf where it does not (a zero denominator demands an exact
    result).  NaN in C gives +inf."""
    C = np.asarray(C, dtype=np.float64)
    diff = np.abs(C - cref)
    out = np.empty_like(diff)
    nz = den > 0
    out[nz] = diff[nz] / den[nz]
    out[~nz] = np.where(diff[~nz] == 0, 0.0, np.inf)
    out[~np.isfinite(C) & np.isfinite(cref)] = np.inf
    return out


def check(C: np.ndarray, cref: np.ndarray, den: np.ndarray, k: int, tol_fn=None):
    """Return (ok, max_err, mean_err, max_err / bound), bound = tol_fn(k)
    (tol by default)."""
    bound = (tol_fn or tol)(k)
    e = normalized_error(C, cref, den)
    if e.size == 0:
        return True, 0.0, 0.0, 0.0
    mx = float(np.max(e))
    return mx <= bound, mx, float(np.mean(e)), mx / bound
