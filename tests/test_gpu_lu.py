"""LU with partial pivoting and the solve (the Linpack workload of the
paper's Section IV-C) on the sgemm path, against the FP64 oracle: identical
pivots and factors where the pivot choice is unique, exact results on data
that factors exactly, and for general random matrices (where rounding may
legitimately pick another of two nearly equal pivots) valid pivots, the
backward error of P A = L U, bounded multipliers and the HPL scaled
residual of the solve."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

EPS32 = 2.0 ** -24


def _mg():
    import paper_1608_05265_amd as mg
    return mg


def _factor(a, mode, lda=None):
    """GPU sgetrf of the dense float32 matrix a; returns (LU dense, ipiv, info)."""
    import torch
    mg = _mg()
    n = a.shape[0]
    lda = lda or n
    buf = np.zeros((n, lda), dtype=np.float32)  # column-major storage with padding rows
    buf[:, :n] = a.T
    d = torch.device("cuda:0")
    A = torch.from_numpy(buf.reshape(-1).copy()).to(d)
    ipiv = torch.zeros(max(n, 1), dtype=torch.int64, device=d)
    info = torch.zeros(1, dtype=torch.int32, device=d)
    mg.sgetrf(n, A, lda, ipiv, info, mode)
    torch.cuda.synchronize()
    lu = A.cpu().numpy().reshape(n, lda)[:, :n].T
    pad = A.cpu().numpy().reshape(n, lda)[:, n:]
    assert np.array_equal(pad, buf[:, n:]), "padding rows written"
    return lu.astype(np.float64), ipiv.cpu().numpy()[:n], int(info.item()), A, ipiv


def _solve(A, ipiv, n, b, mode):
    import torch
    mg = _mg()
    B = torch.from_numpy(np.asarray(b, dtype=np.float32).copy()).to(A.device)
    mg.sgetrs(n, 1, A, n, ipiv, B, n, mode)
    torch.cuda.synchronize()
    return B.cpu().numpy().astype(np.float64)


def _permuted(a, ipiv):
    pa = np.array(a, dtype=np.float64)
    for j, p in enumerate(ipiv):
        pa[[j, p]] = pa[[p, j]]
    return pa


@pytest.mark.parametrize("mode", [0, 1], ids=["fp32", "bf16x3"])
def test_lu_unique_pivots_match_oracle(mode):
    """Permuted diagonally dominant matrices: every pivot is unique by a wide
    margin, so the GPU pivots equal the oracle's and the factors agree to
    FP32 accuracy; sizes around the leaf widths and with several levels."""
    rng = np.random.default_rng(50)
    for n in (1, 7, 8, 9, 31, 32, 33, 100, 257, 600, 1100):
        d = rng.uniform(-1, 1, (n, n)) + np.diag(rng.uniform(n, 2 * n, n))
        a = d[rng.permutation(n)].astype(np.float32)
        lu, ipiv, info = _factor(a, mode)[:3]
        lu_o, ipiv_o, info_o = oracle.getrf_f64(n, a.T.reshape(-1), n)
        assert info == 0 and info_o == 0
        assert np.array_equal(ipiv, ipiv_o), n
        scale = np.max(np.abs(lu_o))
        assert np.max(np.abs(lu - lu_o)) <= 8 * n * EPS32 * scale, n


def test_lu_exact_data_is_exact():
    """A = P T with T upper triangular and power-of-two entries: every
    operation of the factorization and the solve is exact."""
    rng = np.random.default_rng(51)
    n = 96
    t = np.triu(2.0 ** rng.integers(-3, 4, (n, n))) * rng.choice([-1.0, 1.0], (n, n))
    t += np.eye(n) * 256.0
    a = (np.eye(n)[rng.permutation(n)] @ t).astype(np.float32)
    lu, ipiv, info, A, dpiv = _factor(a, 0)
    lu_o, ipiv_o, _ = oracle.getrf_f64(n, a.T.reshape(-1), n)
    assert np.array_equal(ipiv, ipiv_o) and np.array_equal(lu, lu_o)
    x = rng.integers(-5, 6, n).astype(np.float64)
    b = a.astype(np.float64) @ x
    assert np.array_equal(_solve(A, dpiv, n, b, 0), x)


@pytest.mark.parametrize("mode", [0, 1], ids=["fp32", "bf16x3"])
@pytest.mark.parametrize("lda", [8232, 8235], ids=["lda8232", "lda8235"])
def test_lu_exact_data_tall_panels(mode, lda):
    """A = P T at n = 8232 (T upper triangular, power-of-two entries off the
    diagonal, 256 +- a power of two on it): the leaves of the first 36
    columns are taller than 8192 rows (4 columns, 16 rows per thread; four
    fused pairs, whose right leaf takes its sibling's update), the later ones
    hold at most 8 rows per thread, and every pivot is unique; lda 8232 takes the leaves' 16-byte
    row groups, lda 8235 their one-row accesses.  Partial pivoting then
    takes at step j the row that holds row j of T, so the pivots follow
    from P alone, L = I and U = T exactly; the factors are compared bit for
    bit."""
    rng = np.random.default_rng(58)
    n = 8232
    t = np.triu(np.exp2(rng.integers(-3, 4, (n, n))).astype(np.float32))
    t *= rng.choice(np.array([-1.0, 1.0], dtype=np.float32), (n, n))
    t[np.arange(n), np.arange(n)] = 256.0 + np.exp2(rng.integers(-3, 4, n)).astype(np.float32)
    perm = rng.permutation(n)
    a = t[perm]  # row r of A is row perm[r] of T
    del t
    # the pivots partial pivoting takes: the current position of row j of T
    pos = np.empty(n, dtype=np.int64)
    pos[perm] = np.arange(n)
    at = perm.copy()  # at[r]: the row of T now at position r
    want = np.empty(n, dtype=np.int64)
    for j in range(n):
        p = pos[j]
        want[j] = p
        tj, tp = at[j], at[p]
        at[j], at[p] = tp, tj
        pos[tp], pos[tj] = j, p
    lu, ipiv, info = _factor(a, mode, lda)[:3]
    assert info == 0
    assert np.array_equal(ipiv, want)
    u = np.triu(lu)
    assert np.array_equal(u, np.triu(a[np.argsort(perm)]).astype(np.float64))
    assert not np.any(np.tril(lu, -1))


@pytest.mark.parametrize("mode", [0, 1], ids=["fp32", "bf16x3"])
def test_lu_random_backward_error_and_residual(mode):
    """Random uniform[-1,1] matrices (uniform entries, as HPL uses):
    valid pivots, |L| <= 1, ||P A - L U|| small against n eps ||L|| ||U||
    and each entry within 4 n eps (|L| |U|)_ij, and the solve passes HPL's
    check (scaled residual < 16 with FP32 eps)."""
    rng = np.random.default_rng(52)
    for n in (200, 1000, 2048):
        a = rng.uniform(-1, 1, (n, n)).astype(np.float32)
        lu, ipiv, info, A, dpiv = _factor(a, mode, lda=n + 5 if n == 200 else None)
        assert info == 0
        assert np.all(ipiv >= np.arange(n)) and np.all(ipiv < n)
        L = np.tril(lu, -1) + np.eye(n)
        U = np.triu(lu)
        assert np.max(np.abs(L)) <= 1.0 + 1e-6
        resid = np.abs(_permuted(a, ipiv) - L @ U)
        err = np.max(resid)
        bound = 4 * n * EPS32 * np.max(np.sum(np.abs(L), 1)) * np.max(np.sum(np.abs(U), 0))
        assert err <= bound, (n, err, bound)
        # entry by entry: gamma_n (|L| |U|)_ij, gamma_n about n eps (4 n eps here)
        assert np.all(resid <= 4 * n * EPS32 * (np.abs(L) @ np.abs(U))), n
        if n == 200:
            continue  # padded lda: solve takes ld = n
        b = rng.uniform(-1, 1, n)
        x = _solve(A, dpiv, n, b.astype(np.float32), mode)
        r = oracle.hpl_scaled_residual(a, x, b.astype(np.float32), EPS32)
        assert r < 16.0, (n, r)


@pytest.mark.parametrize("mode", [0, 1], ids=["fp32", "bf16x3"])
@pytest.mark.parametrize("lda", [8232, 8235], ids=["lda8232", "lda8235"])
def test_lu_random_tall_leaf_pairs(mode, lda):
    """Uniform[-1,1] at n = 8232, so that the leaves of the first 36 columns
    are taller than 8192 rows (16 rows per thread; four fused pairs, the
    right leaf applying its sibling's solve and update in registers) with
    both panel layouts (lda
    8232: 16-byte row groups; 8235: one row per access): valid pivots,
    |L| <= 1, and every entry of P A - L U on 300 rows (the first 40, whose
    columns those pairs factor, and 260 drawn at random) within the
    componentwise backward-error bound of LU in floating point,
    gamma_n (|L| |U|)_ij with gamma_n about n eps, here 4 n eps (FP32's eps;
    the bf16x3 products' dropped terms add a few eps per product)."""
    rng = np.random.default_rng(59)
    n = 8232
    a = rng.uniform(-1, 1, (n, n)).astype(np.float32)
    lu, ipiv, info = _factor(a, mode, lda)[:3]
    assert info == 0
    assert np.all(ipiv >= np.arange(n)) and np.all(ipiv < n)
    L = np.tril(lu, -1)
    L[np.arange(n), np.arange(n)] = 1.0
    U = np.triu(lu)
    del lu
    assert np.max(np.abs(L)) <= 1.0 + 1e-6
    rows = np.concatenate([np.arange(40), rng.choice(np.arange(40, n), 260, replace=False)])
    pa = _permuted(a, ipiv)[rows]
    err = np.abs(pa - L[rows] @ U)
    bound = 4 * n * EPS32 * (np.abs(L[rows]) @ np.abs(U))
    worst = np.unravel_index(np.argmax(err - bound), err.shape)
    assert np.all(err <= bound), (rows[worst[0]], worst[1], err[worst], bound[worst])


def test_lu_singular_and_errors():
    """A zero column: info names it (1-based) and the rest is factored; a
    zero matrix reports column 1; n = 0 clears info."""
    import torch
    mg = _mg()
    rng = np.random.default_rng(53)
    n = 70
    a = rng.uniform(-1, 1, (n, n)).astype(np.float32)
    a[:, 40] = 0.0
    lu, ipiv, info = _factor(a, 0)[:3]
    assert info == 41
    assert _factor(np.zeros((5, 5), np.float32), 0)[2] == 1
    # n = 0: nothing to factor; info still cleared
    info_t = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    mg.sgetrf(0, None, 1, None, info_t, 0)
    torch.cuda.synchronize()
    assert int(info_t.item()) == 0


def test_getrs_row_swaps_any_pivots():
    """Identity factors (L = U = I), so sgetrs only applies the interchanges:
    row k with row ipiv[k] for k = 0 .. n-1 in order, for pivot lists a
    factorization never makes (targets above k, repeats, rows inside and
    outside a block of interchanges, entries outside [0, n) that must be
    skipped), several right-hand sides and a padded ldb; the result must be
    exactly the sequential swaps done here."""
    import torch
    mg = _mg()
    rng = np.random.default_rng(54)
    d = torch.device("cuda:0")
    for n, nrhs, ldb in ((1, 1, 1), (37, 3, 40), (300, 70, 300), (1000, 1, 1003)):
        eye = torch.from_numpy(np.eye(n, dtype=np.float32).T.reshape(-1).copy()).to(d)
        piv = rng.integers(0, n, n)
        piv[::7] = n - 1                     # one row named many times
        piv[3::11] = np.arange(3, n, 11) + 1  # the next row (inside a block)
        piv[5::13] = -1                       # skipped
        piv[6::17] = n                        # skipped
        piv = np.clip(piv, -1, n)
        b = rng.standard_normal((nrhs, ldb)).astype(np.float32)  # column-major, padded
        B = torch.from_numpy(b.reshape(-1).copy()).to(d)
        mg.sgetrs(n, nrhs, eye, n, torch.from_numpy(piv.astype(np.int64)).to(d), B, ldb, 0)
        torch.cuda.synchronize()
        want = b.copy()
        for k in range(n):
            p = int(piv[k])
            if 0 <= p < n:
                want[:, [k, p]] = want[:, [p, k]]
        assert np.array_equal(B.cpu().numpy().reshape(nrhs, ldb), want), n


@pytest.mark.parametrize("n", [300, 2100, 9000])
def test_lu_pivot_ties_take_first_row(n):
    """Equal largest magnitudes (both signs) in rows held by different
    threads, register slots and wavefronts of the leaf panel: the pivot is
    the first of them, as in the oracle; the sizes give one, four and
    sixteen panel rows per thread."""
    rng = np.random.default_rng(55)
    a = rng.uniform(-1, 1, (n, n)).astype(np.float32)
    rows = sorted({n // 7, n // 3, n // 2 + 1, n - 2, (n // 7) + 1024 if n > 1100 else n - 3})
    a[rows, 0] = [4.0 if i % 2 else -4.0 for i in range(len(rows))]
    ipiv = _factor(a, 0)[1]
    assert ipiv[0] == rows[0], (ipiv[0], rows)
    lu_o, ipiv_o, _ = oracle.getrf_f64(min(n, 300), a[:300, :300].T.reshape(-1), min(n, 300)) if n == 300 else (None, None, None)
    if ipiv_o is not None:
        assert ipiv_o[0] == rows[0]


def test_lu_tall_panels_through_the_solve():
    """n = 16500: the first panels are taller than the register-resident
    leaf takes (16384 rows), so the in-memory leaf factors them.  At this
    size the check is the solve: valid pivots and HPL's scaled residual
    (matrix-vector products only on the CPU)."""
    import torch
    mg = _mg()
    n = 16500
    rng = np.random.default_rng(56)
    a = rng.uniform(-1, 1, (n, n)).astype(np.float32)  # a[i, j], stored column-major below
    d = torch.device("cuda:0")
    A = torch.from_numpy(np.ascontiguousarray(a.T).reshape(-1)).to(d)
    ipiv = torch.zeros(n, dtype=torch.int64, device=d)
    info = torch.zeros(1, dtype=torch.int32, device=d)
    mg.sgetrf(n, A, n, ipiv, info, 0)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    piv = ipiv.cpu().numpy()
    assert np.all(piv >= np.arange(n)) and np.all(piv < n)
    b = rng.uniform(-1, 1, n).astype(np.float32)
    x = _solve(A, ipiv, n, b, 0)
    r = oracle.hpl_scaled_residual(a, x, b, EPS32)
    assert r < 16.0, r


@pytest.mark.parametrize("mode", [0, 1], ids=["fp32", "bf16x3"])
def test_lu_solve_many_rhs_padded_ldb(mode):
    """sgetrs with 7 right-hand sides and ldb = n + 9: every column passes
    HPL's check, and the padding rows of B are never written."""
    import torch
    mg = _mg()
    rng = np.random.default_rng(57)
    n, nrhs, ldb = 1500, 7, 1509
    a = rng.uniform(-1, 1, (n, n)).astype(np.float32)
    lu, ipiv, info, A, dpiv = _factor(a, mode)
    assert info == 0
    b = rng.uniform(-1, 1, (nrhs, ldb)).astype(np.float32)  # column-major B with padding
    b[:, n:] = np.float32(7.25)
    B = torch.from_numpy(b.reshape(-1).copy()).to(A.device)
    mg.sgetrs(n, nrhs, A, n, dpiv, B, ldb, mode)
    torch.cuda.synchronize()
    x = B.cpu().numpy().reshape(nrhs, ldb)
    assert np.all(x[:, n:] == np.float32(7.25))
    for j in range(nrhs):
        r = oracle.hpl_scaled_residual(a, x[j, :n], b[j, :n], EPS32)
        assert r < 16.0, (j, r)


def test_lu_at_the_papers_size():
    """The paper's Linpack size, N = 4608 (Section IV-C, Table VII), both
    forms: on a permuted diagonally dominant matrix the pivots equal the
    oracle's and the factors agree to FP32 accuracy; on uniform[-1,1] data
    (the benchmark's matrix) the solve passes HPL's scaled-residual check
    (below 16, with FP32's eps)."""
    n = 4608
    rng = np.random.default_rng(4608)
    d = rng.uniform(-1, 1, (n, n)) + np.diag(rng.uniform(n, 2 * n, n))
    a = d[rng.permutation(n)].astype(np.float32)
    lu_o, ipiv_o, info_o = oracle.getrf_f64(n, a.T.reshape(-1), n)
    assert info_o == 0
    scale = np.max(np.abs(lu_o))
    for mode in (0, 1):
        lu, ipiv, info = _factor(a, mode)[:3]
        assert info == 0
        assert np.array_equal(ipiv, ipiv_o), "mode %d" % mode
        err = np.max(np.abs(lu - lu_o))
        assert err <= 8 * n * EPS32 * scale, "mode %d: %.3e" % (mode, err / scale)
        print("N=4608 mode %d: max factor deviation %.3e of max |LU|" % (mode, err / scale))
    a = rng.uniform(-1, 1, (n, n)).astype(np.float32)
    b = rng.uniform(-1, 1, n).astype(np.float32)
    for mode in (0, 1):
        lu, ipiv, info, A, ipiv_t = _factor(a, mode)
        assert info == 0
        assert np.all((ipiv >= np.arange(n)) & (ipiv < n))
        x = _solve(A, ipiv_t, n, b, mode)
        r = oracle.hpl_scaled_residual(a, x, b, EPS32)
        assert r < 16.0, "mode %d: scaled residual %.3f" % (mode, r)
        print("N=4608 mode %d: HPL scaled residual %.4f (eps 2^-24)" % (mode, r))
