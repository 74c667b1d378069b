"""MI355X-native single-precision GEMM: the BLAS sgemm hot path.

A thin ``ctypes`` binding of libmisgemm.so (include/misgemm.h).  Every entry
point keeps its C name without the ``misgemm_`` prefix and only marshals
arguments: device pointers come from torch tensors (or plain integers), the
stream defaults to torch's current stream, and a nonzero status raises
MisgemmError.  All arithmetic runs in the library's HIP kernels; there is no
fallback of any kind, and a missing library raises on first use.

Matrices are column-major storage buffers: a rows x cols matrix with leading
dimension ld is a float32 device tensor of ld * cols elements whose element
(r, c) sits at r + c * ld.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

__all__ = ["MisgemmError", "FP32", "BF16X3", "sgemm", "sgemm_config", "sgemm_ws",
           "sgemm_split", "sgemm_split_noalloc",
           "workspace_size", "release_workspace", "workspace_held", "num_configs",
           "config_info", "configs", "select_config", "load_tuning", "Batch", "bf16x3_split",
           "status_string", "version", "library_path"]

FP32 = 0
BF16X3 = 1
MODES = {"fp32": FP32, "bf16x3": BF16X3}

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmisgemm.so")
# Tuning table written by paper_1608_05265_amd.autotune on an MI355X; the
# MISGEMM_TUNING environment variable names another file, or "none".
TUNING_PATH = os.path.join(_HERE, "tuning_mi355x.txt")
_lib = None


class MisgemmError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s: %s (status %d)" % (where, status_string(status), status))


class ConfigDesc(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("bm", ctypes.c_int), ("bn", ctypes.c_int),
                ("bk", ctypes.c_int), ("wm", ctypes.c_int), ("wn", ctypes.c_int),
                ("threads", ctypes.c_int), ("lds_bytes", ctypes.c_int),
                ("packed", ctypes.c_int), ("splitk", ctypes.c_int), ("name", ctypes.c_char * 48)]


class Problem(ctypes.Structure):
    _fields_ = [("transa", ctypes.c_char), ("transb", ctypes.c_char),
                ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
                ("alpha", ctypes.c_float), ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("B", ctypes.c_void_p), ("ldb", ctypes.c_int64), ("beta", ctypes.c_float),
                ("C", ctypes.c_void_p), ("ldc", ctypes.c_int64)]


class BatchDesc(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int64), ("tiles", ctypes.c_int64), ("grid", ctypes.c_int64),
                ("config_id", ctypes.c_int), ("flops", ctypes.c_double),
                ("tile_flops", ctypes.c_double), ("parts", ctypes.c_int),
                ("part_imbalance", ctypes.c_double), ("second_config_id", ctypes.c_int),
                ("second_grid", ctypes.c_int64), ("panel_bytes", ctypes.c_int64)]


def library_path() -> str:
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError("libmisgemm.so is not built (%s); run "
                           "`python -m paper_1608_05265_amd.build` first" % _LIB_PATH)
    lib = ctypes.CDLL(_LIB_PATH)
    c, i64, f32, i32, vp = ctypes.c_char, ctypes.c_int64, ctypes.c_float, ctypes.c_int, \
        ctypes.c_void_p
    sig = [c, c, i64, i64, i64, f32, vp, i64, vp, i64, f32, vp, i64, i32]
    lib.misgemm_sgemm.argtypes = sig + [vp]
    lib.misgemm_sgemm.restype = i32
    lib.misgemm_sgemm_config.argtypes = sig + [i32, i32, vp]
    lib.misgemm_sgemm_config.restype = i32
    f64 = ctypes.c_double
    lib.misgemm_dgemm.argtypes = [c, c, i64, i64, i64, f64, vp, i64, vp, i64, f64, vp, i64,
                                  i32, vp]
    lib.misgemm_dgemm.restype = i32
    lib.misgemm_sgemm_host.argtypes = sig
    lib.misgemm_sgemm_host.restype = i32
    lib.misgemm_dgemm_host.argtypes = [c, c, i64, i64, i64, f64, vp, i64, vp, i64, f64, vp, i64,
                                       i32]
    lib.misgemm_dgemm_host.restype = i32
    lib.misgemm_sgetrf.argtypes = [i64, vp, i64, vp, vp, i32, vp]
    lib.misgemm_sgetrf.restype = i32
    lib.misgemm_sgetrs.argtypes = [i64, i64, vp, i64, vp, vp, i64, i32, vp]
    lib.misgemm_sgetrs.restype = i32
    lib.misgemm_sgemm_split.argtypes = sig + [i32, i32, i32, vp]
    lib.misgemm_sgemm_split.restype = i32
    lib.misgemm_sgemm_split_noalloc.argtypes = sig + [i32, i32, i32, vp]
    lib.misgemm_sgemm_split_noalloc.restype = i32
    lib.misgemm_sgemm_ws.argtypes = sig + [vp, i64, vp]
    lib.misgemm_sgemm_ws.restype = i32
    lib.misgemm_workspace_size.argtypes = [c, c, i64, i64, i64, i32]
    lib.misgemm_workspace_size.restype = i64
    lib.misgemm_release_workspace.argtypes = []
    lib.misgemm_release_workspace.restype = i32
    lib.misgemm_workspace_held.argtypes = []
    lib.misgemm_workspace_held.restype = i64
    lib.misgemm_num_configs.argtypes = []
    lib.misgemm_num_configs.restype = i32
    lib.misgemm_config_info.argtypes = [i32, ctypes.POINTER(ConfigDesc)]
    lib.misgemm_config_info.restype = i32
    lib.misgemm_select_config.argtypes = [c, c, i64, i64, i64, i32]
    lib.misgemm_select_config.restype = i32
    lib.misgemm_load_tuning.argtypes = [ctypes.c_char_p]
    lib.misgemm_load_tuning.restype = i32
    lib.misgemm_batch_plan.argtypes = [ctypes.POINTER(Problem), i64, i32, i32,
                                       ctypes.POINTER(vp), ctypes.POINTER(i64)]
    lib.misgemm_batch_plan.restype = i32
    lib.misgemm_batch_launch.argtypes = [vp, vp]
    lib.misgemm_batch_launch.restype = i32
    lib.misgemm_batch_info.argtypes = [vp, ctypes.POINTER(BatchDesc)]
    lib.misgemm_batch_info.restype = i32
    lib.misgemm_batch_destroy.argtypes = [vp]
    lib.misgemm_batch_destroy.restype = i32
    lib.misgemm_bf16x3_split.argtypes = [vp, i64, vp, vp]
    lib.misgemm_bf16x3_split.restype = i32
    lib.misgemm_status_string.argtypes = [i32]
    lib.misgemm_status_string.restype = ctypes.c_char_p
    lib.misgemm_version.argtypes = []
    lib.misgemm_version.restype = ctypes.c_char_p
    _lib = lib
    table = os.environ.get("MISGEMM_TUNING", TUNING_PATH)
    if table != "none" and os.path.exists(table):
        _check(lib.misgemm_load_tuning(table.encode()), "misgemm_load_tuning(%s)" % table)
    return lib


def _ptr(x) -> Optional[int]:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _mode(mode) -> int:
    return MODES[mode] if isinstance(mode, str) else int(mode)


def _check(rc: int, where: str) -> None:
    if rc != 0:
        raise MisgemmError(rc, where)


def status_string(status: int) -> str:
    return _load().misgemm_status_string(status).decode()


def version() -> str:
    return _load().misgemm_version().decode()


def sgemm(transa: str, transb: str, m: int, n: int, k: int, alpha: float, A, lda: int, B,
          ldb: int, beta: float, C, ldc: int, mode=FP32, stream=None) -> None:
    """C = alpha * op(A) * op(B) + beta * C (asynchronous on `stream`)."""
    rc = _load().misgemm_sgemm(transa.encode(), transb.encode(), m, n, k, alpha, _ptr(A), lda,
                               _ptr(B), ldb, beta, _ptr(C), ldc, _mode(mode), _stream(stream))
    _check(rc, "misgemm_sgemm")


def sgemm_config(transa: str, transb: str, m: int, n: int, k: int, alpha: float, A, lda: int,
                 B, ldb: int, beta: float, C, ldc: int, mode, config_id: int, group_m: int = 0,
                 stream=None) -> None:
    """sgemm with an explicit kernel configuration id and tile order."""
    rc = _load().misgemm_sgemm_config(transa.encode(), transb.encode(), m, n, k, alpha, _ptr(A),
                                      lda, _ptr(B), ldb, beta, _ptr(C), ldc, _mode(mode),
                                      config_id, group_m, _stream(stream))
    _check(rc, "misgemm_sgemm_config")


D_FP64 = 0
D_FP32 = 1


def dgemm(transa: str, transb: str, m: int, n: int, k: int, alpha: float, A, lda: int, B,
          ldb: int, beta: float, C, ldc: int, dmode=D_FP64, stream=None) -> None:
    """Double-precision GEMM on float64 tensors: dmode D_FP64 (FP64 matrix
    cores) or D_FP32 (the FP32-compute "false dgemm")."""
    rc = _load().misgemm_dgemm(transa.encode(), transb.encode(), m, n, k, float(alpha), _ptr(A),
                               lda, _ptr(B), ldb, float(beta), _ptr(C), ldc, int(dmode),
                               _stream(stream))
    _check(rc, "misgemm_dgemm")


def _host_ptr(a, dtype):
    import numpy as np
    if a is None:
        return None
    if not (isinstance(a, np.ndarray) and a.dtype == dtype and a.flags["C_CONTIGUOUS"]):
        raise TypeError("host operands must be contiguous numpy arrays of %s" % np.dtype(dtype))
    return a.ctypes.data


def sgemm_host(transa: str, transb: str, m: int, n: int, k: int, alpha: float, A, lda: int, B,
               ldb: int, beta: float, C, ldc: int, mode=FP32) -> None:
    """sgemm on host (numpy float32) column-major storage; C updated in place."""
    import numpy as np
    rc = _load().misgemm_sgemm_host(transa.encode(), transb.encode(), m, n, k, alpha,
                                    _host_ptr(A, np.float32), lda, _host_ptr(B, np.float32), ldb,
                                    beta, _host_ptr(C, np.float32), ldc, _mode(mode))
    _check(rc, "misgemm_sgemm_host")


def dgemm_host(transa: str, transb: str, m: int, n: int, k: int, alpha: float, A, lda: int, B,
               ldb: int, beta: float, C, ldc: int, dmode=D_FP64) -> None:
    """dgemm on host (numpy float64) column-major storage; C updated in place."""
    import numpy as np
    rc = _load().misgemm_dgemm_host(transa.encode(), transb.encode(), m, n, k, float(alpha),
                                    _host_ptr(A, np.float64), lda, _host_ptr(B, np.float64), ldb,
                                    float(beta), _host_ptr(C, np.float64), ldc, int(dmode))
    _check(rc, "misgemm_dgemm_host")


def sgetrf(n: int, A, lda: int, ipiv, info, mode=FP32, stream=None) -> None:
    """LU with partial pivoting of the n x n float32 device matrix A (in
    place); ipiv an int64 device tensor of n, info an int32 device tensor."""
    rc = _load().misgemm_sgetrf(n, _ptr(A), lda, _ptr(ipiv), _ptr(info), _mode(mode),
                                _stream(stream))
    _check(rc, "misgemm_sgetrf")


def sgetrs(n: int, nrhs: int, A, lda: int, ipiv, B, ldb: int, mode=FP32, stream=None) -> None:
    """Solve A X = B (B overwritten) with the factors of sgetrf."""
    rc = _load().misgemm_sgetrs(n, nrhs, _ptr(A), lda, _ptr(ipiv), _ptr(B), ldb, _mode(mode),
                                _stream(stream))
    _check(rc, "misgemm_sgetrs")


def sgemm_split(transa: str, transb: str, m: int, n: int, k: int, alpha: float, A, lda: int,
                B, ldb: int, beta: float, C, ldc: int, mode, config_id: int = -1,
                group_m: int = 0, splits: int = 1, stream=None) -> None:
    """sgemm with an explicit split-K factor (config_id -1: the split-capable
    configuration with the smallest tile)."""
    rc = _load().misgemm_sgemm_split(transa.encode(), transb.encode(), m, n, k, alpha, _ptr(A),
                                     lda, _ptr(B), ldb, beta, _ptr(C), ldc, _mode(mode),
                                     config_id, group_m, splits, _stream(stream))
    _check(rc, "misgemm_sgemm_split")


def sgemm_split_noalloc(transa: str, transb: str, m: int, n: int, k: int, alpha: float, A,
                        lda: int, B, ldb: int, beta: float, C, ldc: int, mode,
                        config_id: int = -1, group_m: int = 0, splits: int = 1,
                        stream=None) -> None:
    """sgemm_split with the partial tiles in the library's static device
    array: allocates nothing (for graph capture and callers that cannot
    allocate)."""
    rc = _load().misgemm_sgemm_split_noalloc(transa.encode(), transb.encode(), m, n, k, alpha,
                                             _ptr(A), lda, _ptr(B), ldb, beta, _ptr(C), ldc,
                                             _mode(mode), config_id, group_m, splits,
                                             _stream(stream))
    _check(rc, "misgemm_sgemm_split_noalloc")


def sgemm_ws(transa: str, transb: str, m: int, n: int, k: int, alpha: float, A, lda: int, B,
             ldb: int, beta: float, C, ldc: int, mode, workspace, workspace_bytes: int,
             stream=None) -> None:
    """sgemm with a caller-owned workspace (None: never use a packed config)."""
    rc = _load().misgemm_sgemm_ws(transa.encode(), transb.encode(), m, n, k, alpha, _ptr(A), lda,
                                  _ptr(B), ldb, beta, _ptr(C), ldc, _mode(mode), _ptr(workspace),
                                  workspace_bytes, _stream(stream))
    _check(rc, "misgemm_sgemm_ws")


def workspace_size(transa: str, transb: str, m: int, n: int, k: int, mode) -> int:
    rc = _load().misgemm_workspace_size(transa.encode(), transb.encode(), m, n, k, _mode(mode))
    if rc < 0:
        raise MisgemmError(int(rc), "misgemm_workspace_size")
    return int(rc)


def release_workspace() -> None:
    _check(_load().misgemm_release_workspace(), "misgemm_release_workspace")


def workspace_held() -> int:
    """Bytes of library-owned scratch held on the current device."""
    rc = _load().misgemm_workspace_held()
    if rc < 0:
        raise MisgemmError(int(-rc), "misgemm_workspace_held")
    return int(rc)


def num_configs() -> int:
    return _load().misgemm_num_configs()


def config_info(config_id: int) -> dict:
    d = ConfigDesc()
    _check(_load().misgemm_config_info(config_id, ctypes.byref(d)), "misgemm_config_info")
    return {"id": config_id, "mode": d.mode, "bm": d.bm, "bn": d.bn, "bk": d.bk, "wm": d.wm,
            "wn": d.wn, "threads": d.threads, "lds_bytes": d.lds_bytes,
            "packed": d.packed, "splitk": d.splitk, "name": d.name.decode()}


def configs(mode=None) -> List[dict]:
    out = [config_info(i) for i in range(num_configs())]
    if mode is not None:
        out = [c for c in out if c["mode"] == _mode(mode)]
    return out


def select_config(transa: str, transb: str, m: int, n: int, k: int, mode=FP32) -> int:
    rc = _load().misgemm_select_config(transa.encode(), transb.encode(), m, n, k, _mode(mode))
    if rc < 0:
        raise MisgemmError(rc, "misgemm_select_config")
    return rc


def load_tuning(path: Optional[str]) -> None:
    rc = _load().misgemm_load_tuning(None if path is None else path.encode())
    _check(rc, "misgemm_load_tuning")


def bf16x3_split(x, count: int, parts, stream=None) -> None:
    """parts[3*i + t] = bit pattern of the t-th bf16 part of x[i]."""
    rc = _load().misgemm_bf16x3_split(_ptr(x), count, _ptr(parts), _stream(stream))
    _check(rc, "misgemm_bf16x3_split")


class Batch:
    """A batched plan (misgemm_batch_plan ... misgemm_batch_destroy).

    problems: sequence of dicts or tuples with the misgemm_problem fields
    (transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc); A, B, C
    are device tensors or integer device pointers and must outlive the plan.
    """

    def __init__(self, problems: Sequence, mode=FP32, config_id: int = -1):
        lib = _load()
        arr = (Problem * max(1, len(problems)))()
        for i, p in enumerate(problems):
            if isinstance(p, dict):
                p = (p["transa"], p["transb"], p["m"], p["n"], p["k"], p["alpha"], p["A"],
                     p["lda"], p["B"], p["ldb"], p["beta"], p["C"], p["ldc"])
            ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc = p
            arr[i] = Problem(ta.encode(), tb.encode(), m, n, k, alpha, _ptr(A), lda, _ptr(B),
                             ldb, beta, _ptr(C), ldc)
        self._keep = problems
        handle = ctypes.c_void_p()
        bad = ctypes.c_int64(-1)
        rc = lib.misgemm_batch_plan(arr, len(problems), _mode(mode), config_id,
                                    ctypes.byref(handle), ctypes.byref(bad))
        if rc != 0:
            err = MisgemmError(rc, "misgemm_batch_plan")
            err.bad_index = bad.value
            raise err
        self._h = handle

    def launch(self, stream=None) -> None:
        _check(_load().misgemm_batch_launch(self._h, _stream(stream)), "misgemm_batch_launch")

    def info(self) -> dict:
        d = BatchDesc()
        _check(_load().misgemm_batch_info(self._h, ctypes.byref(d)), "misgemm_batch_info")
        return {"count": d.count, "tiles": d.tiles, "grid": d.grid, "config_id": d.config_id,
                "flops": d.flops, "tile_flops": d.tile_flops, "parts": d.parts,
                "part_imbalance": d.part_imbalance, "second_config_id": d.second_config_id,
                "second_grid": d.second_grid, "panel_bytes": d.panel_bytes}

    def destroy(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value is not None:
            _check(_load().misgemm_batch_destroy(self._h), "misgemm_batch_destroy")
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
