"""Double-precision GEMM (the paper's dgemm variants, Section IV-B) against
the binary128 oracle: FP64 matrix cores within max(2K, K+3) * 2^-53, the
FP32-compute form ("false dgemm") within tol(K)(1 + 2^-22) + 2^-23 +
2^-47, every transpose, ragged sizes and padded leading dimensions,
degenerate cases, exactness on integer data, and untouched C padding."""
import numpy as np
import pytest

import oracle
from paper_1608_05265_amd import workloads as wl

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1


def _mg():
    import paper_1608_05265_amd as mg
    return mg


def _dev(p):
    import torch
    d = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(a.copy()).to(d) if a.size else torch.empty(1, dtype=torch.float64, device=d)
    return t(p.A), t(p.B), t(p.C0)


def _run(p, dmode, tensors=None):
    import torch
    mg = _mg()
    A, B, C = tensors if tensors is not None else _dev(p)
    mg.dgemm(p.transa, p.transb, p.m, p.n, p.k, p.alpha, A, p.lda, B, p.ldb, p.beta, C, p.ldc,
             dmode)
    torch.cuda.synchronize()
    return C.cpu().numpy()[:p.C0.size]


def _dense(p, out):
    return out.reshape(p.n, p.ldc).T[:p.m, :]


def _padding_ok(p, out):
    if p.ldc == p.m or p.n == 0:
        return True
    a = out.reshape(p.n, p.ldc)[:, p.m:].view(np.uint64)
    b = p.C0.reshape(p.n, p.ldc)[:, p.m:].view(np.uint64)
    return bool(np.array_equal(a, b))


def _check(p, out, dmode, label):
    cref, den = oracle.dgemm_f128(p.transa, p.transb, p.m, p.n, p.k, p.alpha, p.A, p.lda, p.B,
                                  p.ldb, p.beta, p.C0, p.ldc)
    tol_fn = oracle.tol_d if dmode == FP64 else oracle.tol_false_d
    ok, mx, mean, ratio = oracle.check(_dense(p, out), cref, den, p.k, tol_fn)
    assert _padding_ok(p, out), "C padding written " + label
    assert ok, "%s: max normalized error %.3e, bound %.3e" % (label, mx, tol_fn(p.k))
    return mx


@pytest.mark.parametrize("dmode", [FP64, FP32], ids=["fp64", "fp32-compute"])
def test_dgemm_against_oracle(dmode):
    """Ragged shapes (several tiles plus tails) in both tile sizes, every
    transpose pair, padded leading dimensions, alpha/beta variety."""
    cases = [(150, 97, 211, 1.5, -0.5), (300, 260, 64, -1.0, 1.0), (129, 385, 37, 0.3, 0.0),
             (1000, 640, 300, 1.0, 0.25)]
    for ci, (m, n, k, alpha, beta) in enumerate(cases):
        for ti, (ta, tb) in enumerate(wl.TRANS_PAIRS):
            p = wl.make_problem_d(ta, tb, m, n, k, alpha, beta, 7000 + 10 * ci + ti,
                                  pad=(ci + ti) % 3)
            _check(p, _run(p, dmode), dmode, "%s%s %dx%dx%d" % (ta, tb, m, n, k))


def test_dgemm_fp64_large_sampled_and_errors_of_both_forms():
    """A 2048 x 2048 x 2048 problem, entries sampled against the oracle: the
    FP64 form's error is orders of magnitude below the FP32-compute form's
    (which carries FP32 rounding, as the paper's false dgemm does)."""
    p = wl.make_problem_d("N", "T", 2048, 2048, 2048, 1.0, -1.0, 7100)
    rng = np.random.default_rng(5)
    rows = rng.integers(0, p.m, 256)
    cols = rng.integers(0, p.n, 256)
    cref, den = oracle.dgemm_f128_entries(p.transa, p.transb, p.m, p.n, p.k, p.alpha, p.A,
                                          p.lda, p.B, p.ldb, p.beta, p.C0, p.ldc, rows, cols)
    errs = {}
    for dmode, tol_fn in ((FP64, oracle.tol_d), (FP32, oracle.tol_false_d)):
        out = _run(p, dmode)
        got = out[rows + cols * p.ldc]
        ok, mx, mean, ratio = oracle.check(got, cref, den, p.k, tol_fn)
        assert ok, (dmode, mx)
        errs[dmode] = mx
    assert errs[FP64] < 1e-13 and errs[FP32] > 1e-9


def test_dgemm_integer_inputs_exact():
    """Integers below 2^20 with K = 64: every sum is exact in FP64, so the
    FP64 form equals the oracle bit for bit."""
    rng = np.random.default_rng(11)
    for ta, tb in wl.TRANS_PAIRS:
        p = wl.make_problem_d(ta, tb, 200, 136, 64, 1.0, 0.0, 7200)
        p.A[:] = rng.integers(-2 ** 20, 2 ** 20, size=p.A.size)
        p.B[:] = rng.integers(-2 ** 20, 2 ** 20, size=p.B.size)
        out = _run(p, FP64)
        cref, _ = oracle.dgemm_f128(ta, tb, p.m, p.n, p.k, 1.0, p.A, p.lda, p.B, p.ldb, 0.0,
                                    None, p.ldc)
        assert np.array_equal(_dense(p, out), cref)


@pytest.mark.parametrize("dmode", [FP64, FP32], ids=["fp64", "fp32-compute"])
def test_dgemm_degenerate_and_deterministic(dmode):
    import torch
    mg = _mg()
    # alpha = 0: C = beta * C0, A and B not read (NaN there)
    p = wl.make_problem_d("N", "N", 70, 50, 30, 0.0, -2.0, 7300, pad=1)
    A, B, C = _dev(p)
    A.fill_(float("nan"))
    B.fill_(float("nan"))
    out = _run(p, dmode, (A, B, C))
    assert np.array_equal(_dense(p, out), -2.0 * wl_dense(p))
    assert _padding_ok(p, out)
    # k = 0 with beta = 0: zeros, NaN C0 cleared
    p = wl.make_problem_d("T", "N", 33, 17, 0, 1.0, 0.0, 7301)
    out = _run(p, dmode)
    assert np.array_equal(_dense(p, out), np.zeros((33, 17)))
    # m = 0: nothing to do, no device needed for that
    mg.dgemm("N", "N", 0, 5, 5, 1.0, None, 1, None, 5, 0.0, None, 1, dmode)
    # two runs give the same bits
    p = wl.make_problem_d("N", "T", 333, 222, 111, 1.25, 0.5, 7302, pad=2)
    t = _dev(p)
    a = _run(p, dmode, t).copy()
    t[2].copy_(torch.from_numpy(p.C0.copy()).to(t[2].device))
    b = _run(p, dmode, t)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def wl_dense(p):
    return p.C0.reshape(p.n, p.ldc).T[:p.m, :]
