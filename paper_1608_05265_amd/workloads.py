"""Seeded synthetic workloads for the sgemm path.

This module only draws numbers and lays them out in column-major storage; it
holds none of the GEMM arithmetic, so that the GPU tests and the CPU oracle
can both take their inputs from it.

Storage convention (BLAS, column-major): a rows x cols matrix with leading
dimension ld >= rows is a 1-D float32 array of ld * cols values in which
element (r, c) sits at r + c * ld.  Rows r in [rows, ld) are padding.

Recipes (the paper's own workloads, the BLIS test-suite and HPL, are not
available; these stand in for them with their shapes):
  * seed = 160805265 + 1000 * config + case, numpy default_rng (PCG64);
  * values drawn in float64 and rounded to float32, in the order A, B, C0,
    each over its whole stored array including padding;
  * padding of A and B is then overwritten with NaN, padding of C with the
    canary bit pattern 0x7FC0DEAD, which the library must leave untouched;
  * C0 is NaN-filled when beta == 0 (it must not be read).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

SEED_BASE = 160805265
NAN_BITS = np.uint32(0x7FC00000)
CANARY_BITS = np.uint32(0x7FC0DEAD)
NAN_BITS64 = np.uint64(0x7FF8000000000000)
CANARY_BITS64 = np.uint64(0x7FF8DEADDEADDEAD)


def seed_for(config: int, case: int) -> int:
    return SEED_BASE + 1000 * config + case


def is_trans(t: str) -> bool:
    return t in ("T", "t", "C", "c")


@dataclasses.dataclass
class Problem:
    """One sgemm call: C = alpha * op(A) * op(B) + beta * C, column-major."""
    transa: str
    transb: str
    m: int
    n: int
    k: int
    alpha: float
    A: np.ndarray
    lda: int
    B: np.ndarray
    ldb: int
    beta: float
    C0: np.ndarray
    ldc: int
    label: str = ""

    @property
    def a_shape(self):
        """(rows, cols) of the stored A."""
        return (self.k, self.m) if is_trans(self.transa) else (self.m, self.k)

    @property
    def b_shape(self):
        return (self.n, self.k) if is_trans(self.transb) else (self.k, self.n)

    def flops(self) -> int:
        """Algorithmic flops 2*M*N*K (the paper's GFLOPS convention)."""
        return 2 * self.m * self.n * self.k

    def bytes(self) -> int:
        """Algorithmic HBM bytes: read op(A), op(B) once, read C0 when
        beta != 0, write C once."""
        c_terms = 2 if self.beta != 0.0 else 1
        return self.A.itemsize * (self.m * self.k + self.k * self.n + c_terms * self.m * self.n)


def storage_size(rows: int, cols: int, ld: int) -> int:
    return ld * cols if cols > 0 else 0


def fill_padding(buf: np.ndarray, rows: int, cols: int, ld: int, bits: np.uint32) -> None:
    """Overwrite rows [rows, ld) of every column with the given bit pattern."""
    if ld > rows and cols > 0:
        view = buf.view(np.uint32).reshape(cols, ld)
        view[:, rows:] = bits


def _draw(rng: np.random.Generator, size: int, dist: str) -> np.ndarray:
    if dist == "uniform":
        x = rng.uniform(-1.0, 1.0, size)
    elif dist == "normal":
        x = rng.standard_normal(size)
    elif dist == "unit":
        # same sign everywhere: |A||B| = A B, so the bound's denominator is
        # the result itself and no cancellation hides accumulation error
        x = rng.uniform(0.0, 1.0, size)
    elif dist == "wide":
        # random sign times 2^u with u continuous uniform in [-8, 8]
        s = np.where(rng.random(size) < 0.5, -1.0, 1.0)
        x = s * np.exp2(rng.uniform(-8.0, 8.0, size))
    else:
        raise ValueError(dist)
    return x.astype(np.float32)


def make_problem(transa: str, transb: str, m: int, n: int, k: int, alpha: float, beta: float,
                 seed: int, dist: str = "uniform", pad: int = 0, label: str = "",
                 c0_nan_when_beta0: bool = True) -> Problem:
    """Draw one problem.  pad is added to every leading dimension."""
    rng = np.random.default_rng(seed)
    ar, ac = (k, m) if is_trans(transa) else (m, k)
    br, bc = (n, k) if is_trans(transb) else (k, n)
    lda, ldb, ldc = max(1, ar + pad), max(1, br + pad), max(1, m + pad)
    A = _draw(rng, storage_size(ar, ac, lda), dist)
    B = _draw(rng, storage_size(br, bc, ldb), dist)
    C0 = _draw(rng, storage_size(m, n, ldc), dist)
    fill_padding(A, ar, ac, lda, NAN_BITS)
    fill_padding(B, br, bc, ldb, NAN_BITS)
    if beta == 0.0 and c0_nan_when_beta0:
        C0.view(np.uint32)[:] = NAN_BITS
    fill_padding(C0, m, n, ldc, CANARY_BITS)
    return Problem(transa, transb, m, n, k, float(alpha), A, lda, B, ldb, float(beta), C0, ldc,
                   label=label)


def fill_padding64(buf: np.ndarray, rows: int, cols: int, ld: int, bits: np.uint64) -> None:
    """fill_padding for FP64 storage."""
    if ld > rows and cols > 0:
        view = buf.view(np.uint64).reshape(cols, ld)
        view[:, rows:] = bits


def make_problem_d(transa: str, transb: str, m: int, n: int, k: int, alpha: float,
                   beta: float, seed: int, dist: str = "uniform", pad: int = 0,
                   label: str = "") -> Problem:
    """One double-precision problem: the draws of make_problem kept in FP64
    (A, then B, then C0, over the stored arrays), FP64 NaN in the A/B
    padding and in C0 when beta == 0, an FP64 canary in the C padding."""
    rng = np.random.default_rng(seed)
    ar, ac = (k, m) if is_trans(transa) else (m, k)
    br, bc = (n, k) if is_trans(transb) else (k, n)
    lda, ldb, ldc = max(1, ar + pad), max(1, br + pad), max(1, m + pad)
    draw = {"uniform": lambda size: rng.uniform(-1.0, 1.0, size),
            "normal": lambda size: rng.standard_normal(size)}[dist]
    A = draw(storage_size(ar, ac, lda)).astype(np.float64)
    B = draw(storage_size(br, bc, ldb)).astype(np.float64)
    C0 = draw(storage_size(m, n, ldc)).astype(np.float64)
    fill_padding64(A, ar, ac, lda, NAN_BITS64)
    fill_padding64(B, br, bc, ldb, NAN_BITS64)
    if beta == 0.0:
        C0.view(np.uint64)[:] = NAN_BITS64
    fill_padding64(C0, m, n, ldc, CANARY_BITS64)
    return Problem(transa, transb, m, n, k, float(alpha), A, lda, B, ldb, float(beta), C0, ldc,
                   label=label)


# --------------------------------------------------------------------------
# The five workload families.
# --------------------------------------------------------------------------

TRANS_PAIRS = [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")]
SQUARE_SIZES = [1024, 2048, 4096, 8192]
RANKK_KS = [128, 256, 512]


def config1(size: int = 256) -> Problem:
    """Single FP32 sgemm 256^3, NN, alpha=1, beta=0, uniform[-1,1], tight ld."""
    return make_problem("N", "N", size, size, size, 1.0, 0.0, seed_for(1, 0),
                        label="square%d_NN" % size)


def config2(size: int, transa: str, transb: str) -> Problem:
    """Square sweep: alpha=1.5, beta=-0.5, uniform[-1,1], every ld padded by 16."""
    case = SQUARE_SIZES.index(size) * 4 + TRANS_PAIRS.index((transa, transb)) \
        if size in SQUARE_SIZES else 100 + size
    return make_problem(transa, transb, size, size, size, 1.5, -0.5, seed_for(2, case),
                        pad=16, label="square%d_%s%s" % (size, transa, transb))


def config3(k: int, mn: int = 16384) -> Problem:
    """Linpack-style trailing update: M=N=16384, small K, alpha=-1, beta=1, normal(0,1)."""
    case = RANKK_KS.index(k) if k in RANKK_KS else 100 + k
    return make_problem("N", "N", mn, mn, k, -1.0, 1.0, seed_for(3, case), dist="normal",
                        label="rankk%d_%dx%d" % (k, mn, mn))


def config4(size: int = 8192) -> Problem:
    """Wide-dynamic-range entries (random sign x 2^U[-8,8]), NN, alpha=1, beta=0."""
    return make_problem("N", "N", size, size, size, 1.0, 0.0, seed_for(4, 0), dist="wide",
                        label="wide%d_NN" % size)


@dataclasses.dataclass
class BatchSpec:
    transa: str
    transb: str
    m: int
    n: int
    k: int
    beta: float


def batch_specs(count: int = 512, seed: Optional[int] = None, lo: int = 2, hi: int = 64,
                step: int = 16) -> List[BatchSpec]:
    """Sizes 16*U{2..64} for M, N, K; transposes uniform over NN/NT/TN;
    beta uniform over {0, 1}; alpha = 1."""
    rng = np.random.default_rng(seed_for(5, 0) if seed is None else seed)
    pairs = [("N", "N"), ("N", "T"), ("T", "N")]
    out = []
    for _ in range(count):
        m, n, k = (int(step * v) for v in rng.integers(lo, hi + 1, size=3))
        ta, tb = pairs[int(rng.integers(0, 3))]
        beta = float(rng.integers(0, 2))
        out.append(BatchSpec(ta, tb, m, n, k, beta))
    return out


def config5(count: int = 512, seed_case: int = 0, lo: int = 2, hi: int = 64,
            step: int = 16) -> List[Problem]:
    """The batch of independent GEMMs, each with its own seed."""
    specs = batch_specs(count, seed_for(5, seed_case), lo, hi, step)
    return [make_problem(s.transa, s.transb, s.m, s.n, s.k, 1.0, s.beta,
                         seed_for(5, 1 + seed_case * 100000 + i),
                         label="batch%d_%d" % (seed_case, i))
            for i, s in enumerate(specs)]


SKINNY_SHAPES = [(512, 512, 512), (128, 512, 8192), (512, 512, 16384)]


def config7(m: int, n: int, k: int) -> Problem:
    """Under-filled grids, the split-K regime: few output tiles and a long K
    (the small square case and skinny outputs of long inner products),
    alpha=1.5, beta=-0.5, uniform[-1,1], tight ld."""
    case = SKINNY_SHAPES.index((m, n, k)) if (m, n, k) in SKINNY_SHAPES else 1000 + m
    return make_problem("N", "N", m, n, k, 1.5, -0.5, seed_for(7, case),
                        label="skinny%dx%dx%d_NN" % (m, n, k))


DGEMM_SIZES = [2048, 4096, 8192]


def config6(size: int, transa: str = "N", transb: str = "N") -> Problem:
    """Double-precision square problem (the paper's dgemm, Section IV-B, at
    the square-sweep settings): alpha=1.5, beta=-0.5, uniform[-1,1], every
    leading dimension padded by 16."""
    case = DGEMM_SIZES.index(size) * 4 + TRANS_PAIRS.index((transa, transb)) \
        if size in DGEMM_SIZES else 1000 + size
    return make_problem_d(transa, transb, size, size, size, 1.5, -0.5, seed_for(6, case),
                          pad=16, label="dgemm%d_%s%s" % (size, transa, transb))


def gflops_rate(m: int, n: int, k: int, seconds: float) -> float:
    """GFLOP/s = 2*m*n*k / t / 1e9 (the convention behind the paper's tables)."""
    return 2.0 * m * n * k / seconds / 1e9
