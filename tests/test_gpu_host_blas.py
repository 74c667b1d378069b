"""Host-pointer BLAS: the Fortran sgemm_/dgemm_ symbols and their C forms on
matrices in host memory, against the oracles -- single and multi-panel
shapes, every transpose, padded leading dimensions whose padding must stay
untouched, degenerate cases, and the reference-BLAS argument message."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1608_05265_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _mg():
    import paper_1608_05265_amd as mg
    return mg


def _fortran_sgemm(p, C):
    """Call sgemm_ the way a Fortran program does: every argument by address."""
    lib = ctypes.CDLL(_mg().library_path())
    i = lambda v: ctypes.byref(ctypes.c_int(v))
    f = lambda v: ctypes.byref(ctypes.c_float(v))
    fp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    lib.sgemm_(ctypes.c_char_p(p.transa.encode()), ctypes.c_char_p(p.transb.encode()),
               i(p.m), i(p.n), i(p.k), f(p.alpha), fp(p.A), i(p.lda), fp(p.B), i(p.ldb),
               f(p.beta), fp(C), i(p.ldc))


@pytest.mark.parametrize("mode", [0, 1], ids=["fp32", "bf16x3"])
def test_sgemm_host_against_oracle(mode):
    """One panel (n < 1024) and four panels (n >= 1024), every transpose,
    padded leading dimensions (C padding is a canary that must survive)."""
    mg = _mg()
    shapes = [(300, 200, 150), (517, 1100, 260)]
    for si, (m, n, k) in enumerate(shapes):
        for ti, (ta, tb) in enumerate(wl.TRANS_PAIRS):
            p = wl.make_problem(ta, tb, m, n, k, 1.5, -0.5, 8000 + 10 * si + ti, pad=3)
            C = p.C0.copy()
            mg.sgemm_host(ta, tb, m, n, k, p.alpha, p.A, p.lda, p.B, p.ldb, p.beta, C, p.ldc,
                          mode)
            gu.check_full(p, C, "host %s%s %dx%dx%d mode %d" % (ta, tb, m, n, k, mode))


@pytest.mark.parametrize("mode", [0, 1], ids=["fp32", "bf16x3"])
def test_sgemm_host_operands_over_several_upload_chunks(mode):
    """Operands larger than the pinned upload chunks (64 MB): op(A) of
    6003 x 6000 floats (144 MB, three chunks, so that a chunk buffer is
    refilled after its previous transfer), B whole (transposed) or in four
    column panels; sampled entries against the oracle, C padding intact."""
    mg = _mg()
    m, n, k = 6000, 2100, 6000
    pairs = wl.TRANS_PAIRS if mode == 0 else [("N", "N"), ("N", "T")]
    for ti, (ta, tb) in enumerate(pairs):
        p = wl.make_problem(ta, tb, m, n, k, 1.5, -0.5, 8100 + ti, pad=3)
        C = p.C0.copy()
        mg.sgemm_host(ta, tb, m, n, k, p.alpha, p.A, p.lda, p.B, p.ldb, p.beta, C, p.ldc, mode)
        gu.check_sampled(p, C, count=2048, seed=ti, label="host %s%s mode %d" % (ta, tb, mode))


def test_fortran_sgemm_symbol():
    """sgemm_ with by-reference arguments; beta = 0 clears a NaN C."""
    for ta, tb in wl.TRANS_PAIRS:
        p = wl.make_problem(ta, tb, 257, 1030, 97, -1.0, 0.0, 8100, pad=1)
        C = p.C0.copy()  # NaN where it is read-only data (beta = 0), canary in padding
        _fortran_sgemm(p, C)
        gu.check_full(p, C, "sgemm_ %s%s" % (ta, tb))


def test_fortran_sgemm_degenerate_and_errors(capfd):
    # alpha = 0: C = beta * C, A and B never read (NULL is fine)
    p = wl.make_problem("N", "N", 40, 30, 20, 0.0, 2.0, 8200, pad=2)
    C = p.C0.copy()
    mg = _mg()
    mg.sgemm_host("N", "N", 40, 30, 20, 0.0, None, p.lda, None, p.ldb, 2.0, C, p.ldc)
    gu.check_full(p, C, "alpha=0")
    # invalid lda: reference-BLAS message, C untouched
    p = wl.make_problem("N", "N", 40, 30, 20, 1.0, 1.0, 8201)
    p.lda = 10
    C = p.C0.copy()
    _fortran_sgemm(p, C)
    assert np.array_equal(C.view(np.uint32), p.C0.view(np.uint32))
    err = capfd.readouterr().err
    assert "On entry to SGEMM" in err and "parameter number 8" in err


def test_dgemm_host_against_oracle():
    mg = _mg()
    for ta, tb in wl.TRANS_PAIRS:
        p = wl.make_problem_d(ta, tb, 333, 1050, 129, 1.25, 0.5, 8300, pad=2)
        C = p.C0.copy()
        mg.dgemm_host(ta, tb, p.m, p.n, p.k, p.alpha, p.A, p.lda, p.B, p.ldb, p.beta, C, p.ldc)
        cref, den = oracle.dgemm_f128(ta, tb, p.m, p.n, p.k, p.alpha, p.A, p.lda, p.B, p.ldb,
                                      p.beta, p.C0, p.ldc)
        got = C.reshape(p.n, p.ldc).T[:p.m, :]
        ok, mx, _, _ = oracle.check(got, cref, den, p.k, oracle.tol_d)
        assert ok, (ta, tb, mx)
        pad_now = C.reshape(p.n, p.ldc)[:, p.m:].view(np.uint64)
        pad_was = p.C0.reshape(p.n, p.ldc)[:, p.m:].view(np.uint64)
        assert np.array_equal(pad_now, pad_was)


def test_fortran_dgemm_symbol_and_sgemm_mode_switch(monkeypatch):
    """dgemm_ with by-reference arguments against the binary128 oracle; and
    sgemm_ in the bf16x3 form when MISGEMM_SGEMM_MODE says so (read at each
    call), within the same bound."""
    lib = ctypes.CDLL(_mg().library_path())
    i = lambda v: ctypes.byref(ctypes.c_int(v))
    d = lambda v: ctypes.byref(ctypes.c_double(v))
    fp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    for ta, tb in wl.TRANS_PAIRS:
        p = wl.make_problem_d(ta, tb, 150, 1100, 77, -0.5, 1.5, 8500, pad=1)
        C = p.C0.copy()
        lib.dgemm_(ctypes.c_char_p(ta.encode()), ctypes.c_char_p(tb.encode()), i(p.m), i(p.n),
                   i(p.k), d(p.alpha), fp(p.A), i(p.lda), fp(p.B), i(p.ldb), d(p.beta), fp(C),
                   i(p.ldc))
        cref, den = oracle.dgemm_f128(ta, tb, p.m, p.n, p.k, p.alpha, p.A, p.lda, p.B, p.ldb,
                                      p.beta, p.C0, p.ldc)
        ok, mx, _, _ = oracle.check(C.reshape(p.n, p.ldc).T[:p.m, :], cref, den, p.k,
                                    oracle.tol_d)
        assert ok, ("dgemm_", ta, tb, mx)
    p = wl.make_problem("T", "N", 200, 1030, 300, 1.0, -1.0, 8501, pad=2)
    c32 = p.C0.copy()
    _fortran_sgemm(p, c32)
    gu.check_full(p, c32, "sgemm_ fp32")
    monkeypatch.setenv("MISGEMM_SGEMM_MODE", "bf16x3")
    cx3 = p.C0.copy()
    _fortran_sgemm(p, cx3)
    gu.check_full(p, cx3, "sgemm_ bf16x3")
    # the two forms round differently on random data: the switch took effect
    assert not np.array_equal(c32.view(np.uint32), cx3.view(np.uint32))
