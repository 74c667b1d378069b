"""Non-finite operands in the FP32 form (IEEE arithmetic on the matrix
cores, through the split-K reduction and the alpha/beta epilogue of
Section III-C): a NaN in row r of op(A) makes row r of C NaN, +inf in row
s of op(A) times a strictly positive op(B) makes row s of C +inf, and every
other entry stays finite and within the error bound against the oracle run
on the same data with those two rows of op(A) set to zero.  Every FP32
configuration, both staging orders of A (NN and TN), and split-K.  The
bf16x3 form takes finite inputs below the bf16 rounding-overflow threshold
only (its split of an infinity is not a sum of parts), so it is not run
here."""
import numpy as np
import pytest

import oracle
from paper_1608_05265_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

NAN_ROW, INF_ROW = 37, 142
M, N, K = 197, 131, 263


def _problem(transa):
    p = wl.make_problem(transa, "N", M, N, K, 1.0, 0.5, seed=880 + (transa == "T"), pad=3)
    rng = np.random.default_rng(881)
    B = p.B.reshape(N, p.ldb)  # column-major: B[col][row]
    B[:, :K] = (0.5 + 0.5 * rng.random((N, K))).astype(np.float32)  # op(B) > 0
    clean = p.A.copy()

    def at(r, kk):  # storage index of op(A)(r, kk)
        return kk + r * p.lda if transa == "T" else r + kk * p.lda
    for kk in range(K):
        clean[at(NAN_ROW, kk)] = 0.0
        clean[at(INF_ROW, kk)] = 0.0
    p.A[at(NAN_ROW, 17)] = np.float32(np.nan)
    p.A[at(INF_ROW, 201)] = np.float32(np.inf)
    # the oracle's reference: the same problem with the two rows of op(A) zero
    cref, den = oracle.sgemm_f64(p.transa, p.transb, M, N, K, p.alpha, clean, p.lda, p.B, p.ldb,
                                 p.beta, p.C0, p.ldc)
    return p, cref, den


def _check(p, out, cref, den, label):
    c = gu.c_dense(p, out)
    assert np.all(np.isnan(c[NAN_ROW])), label + ": NaN row"
    assert np.all(np.isposinf(c[INF_ROW])), label + ": +inf row"
    keep = np.ones(M, dtype=bool)
    keep[[NAN_ROW, INF_ROW]] = False
    assert np.all(np.isfinite(c[keep])), label + ": other rows finite"
    ok, mx, _, _ = oracle.check(c[keep], cref[keep], den[keep], K)
    assert ok, "%s: max normalized error %.3e" % (label, mx)
    assert gu.padding_untouched(p, out), label + ": padding"


@pytest.mark.parametrize("transa", ["N", "T"])
def test_fp32_nan_and_inf_propagate_every_config(transa):
    import paper_1608_05265_amd as mg
    p, cref, den = _problem(transa)
    for cfg in [None] + mg.configs(mg.FP32):
        out = gu.run(p, mg.FP32, config_id=None if cfg is None else cfg["id"])
        _check(p, out, cref, den, "%s%s %s" % (transa, "N", "default" if cfg is None
                                                else cfg["name"]))


def test_fp32_nan_and_inf_propagate_split_k():
    import torch
    import paper_1608_05265_amd as mg
    p, cref, den = _problem("N")
    for splits in (2, 5):
        A, B, C = gu.dev_problem(p)
        mg.sgemm_split(p.transa, p.transb, M, N, K, p.alpha, A, p.lda, B, p.ldb, p.beta, C,
                       p.ldc, mg.FP32, splits=splits)
        torch.cuda.synchronize()
        _check(p, C.cpu().numpy()[:p.C0.size], cref, den, "split-K %d" % splits)
