"""GPU parity at sizes the full oracle finishes in seconds: every compiled
configuration, every transpose pair, ragged edges, padded leading
dimensions, both arithmetic forms."""
import numpy as np
import pytest

import oracle
from paper_1608_05265_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1, 1), (7, 5, 3), (33, 17, 65), (64, 64, 64), (257, 129, 300), (300, 520, 97),
          (1000, 999, 37)]


def _mg():
    import paper_1608_05265_amd as mg
    return mg


@pytest.mark.parametrize("mode", [0, 1], ids=["fp32", "bf16x3"])
def test_config1_square256(mode):
    p = wl.config1()
    out = gu.run(p, mode)
    mx, mean, ratio = gu.check_full(p, out, "c1 mode %d" % mode)
    print("c1 mode=%d max=%.3e mean=%.3e ratio=%.3e" % (mode, mx, mean, ratio))


@pytest.mark.parametrize("mode", [0, 1], ids=["fp32", "bf16x3"])
@pytest.mark.parametrize("ta,tb", wl.TRANS_PAIRS, ids=["NN", "NT", "TN", "TT"])
def test_shapes_default_config(mode, ta, tb):
    for i, (m, n, k) in enumerate(SHAPES):
        p = wl.make_problem(ta, tb, m, n, k, 1.5, -0.5, 1000 + i, pad=3)
        out = gu.run(p, mode)
        gu.check_full(p, out, "%s%s %dx%dx%d mode %d" % (ta, tb, m, n, k, mode))


def test_every_config_every_transpose():
    mg = _mg()
    for cfg in mg.configs():
        for ti, (ta, tb) in enumerate(wl.TRANS_PAIRS):
            # spans several tiles of this config and leaves a ragged tail
            m = 2 * cfg["bm"] + 13
            n = cfg["bn"] + 7
            k = 3 * cfg["bk"] + 5
            p = wl.make_problem(ta, tb, m, n, k, -1.25, 0.5, 2000 + 4 * cfg["id"] + ti, pad=5)
            out = gu.run(p, cfg["mode"], config_id=cfg["id"])
            gu.check_full(p, out, "%s %s%s" % (cfg["name"], ta, tb))


def test_every_config_whole_blocks_with_beta():
    """Every configuration on a problem of whole tiles and whole K blocks
    (the unmasked load path) with beta != 0, each transpose pair: the paths
    that read C0 early, fold it into the accumulators or skip masking are
    all taken here."""
    mg = _mg()
    for cfg in mg.configs():
        for ti, (ta, tb) in enumerate(wl.TRANS_PAIRS):
            m, n, k = 2 * cfg["bm"], 2 * cfg["bn"], 8 * cfg["bk"]
            p = wl.make_problem(ta, tb, m, n, k, -1.5, 0.75, 3000 + 4 * cfg["id"] + ti)
            out = gu.run(p, cfg["mode"], config_id=cfg["id"])
            gu.check_full(p, out, "%s %s%s whole blocks" % (cfg["name"], ta, tb))


@pytest.mark.parametrize("mode", [0, 1], ids=["fp32", "bf16x3"])
def test_integer_inputs_bit_exact(mode):
    """Entries in {-4..4}, K <= 1024: every partial sum is an exact integer
    in FP32 (and every entry is exact in bf16), so the GPU must equal the
    oracle bit for bit in both forms."""
    rng = np.random.default_rng(3)
    for ta, tb in wl.TRANS_PAIRS:
        p = wl.make_problem(ta, tb, 300, 260, 1024, 1.0, 0.0, 7)
        p.A[:] = rng.integers(-4, 5, size=p.A.size)
        p.B[:] = rng.integers(-4, 5, size=p.B.size)
        out = gu.run(p, mode)
        cref, _ = oracle.sgemm_f64(ta, tb, p.m, p.n, p.k, 1.0, p.A, p.lda, p.B, p.ldb, 0.0, None,
                                   p.ldc)
        assert np.array_equal(gu.c_dense(p, out).astype(np.float64), cref)


def test_random_shapes_default_dispatch():
    """Seeded random problems through the default dispatch (tuned entries,
    the size heuristic and automatic split-K for under-filled grids):
    sizes from 1 to 400 with K log-uniform up to 4096, every transpose pair,
    alpha and beta including 0, padded leading dimensions, both forms --
    every entry against the full oracle, C padding untouched."""
    rng = np.random.default_rng(160805)
    for case in range(48):
        m, n = (int(v) for v in rng.integers(1, 401, size=2))
        k = int(np.exp(rng.uniform(0.0, np.log(4096.0))))
        ta, tb = wl.TRANS_PAIRS[int(rng.integers(0, 4))]
        alpha = float(rng.choice([1.0, -0.75, 2.5, 0.0], p=[0.4, 0.25, 0.25, 0.1]))
        beta = float(rng.choice([0.0, 1.0, 0.5, -2.0]))
        pad = int(rng.integers(0, 6))
        p = wl.make_problem(ta, tb, m, n, k, alpha, beta, 9000 + case, pad=pad)
        for mode in (0, 1):
            out = gu.run(p, mode)
            gu.check_full(p, out, "case %d %s%s %dx%dx%d a=%g b=%g pad=%d mode %d"
                          % (case, ta, tb, m, n, k, alpha, beta, pad, mode))
