"""Pins of the CPU oracle: checks against facts that the paper's problem
statement (Section III-A) and plain mathematics fix, each computed by a route
other than the oracle's own loops.

Every function takes an ``oracle.Oracle`` instance and raises AssertionError
on a mismatch, so the same pins run against the real oracle (they must pass)
and against deliberately broken copies of it (at least one must fail).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from paper_1608_05265_amd import workloads as wl

U53 = 2.0 ** -53


def dense(buf, rows, cols, ld):
    """Stored column-major buffer -> rows x cols float64 array, via numpy's
    Fortran-order reshape (an indexing route independent of the oracle's)."""
    if rows == 0 or cols == 0:
        return np.zeros((rows, cols))
    return np.asarray(buf, dtype=np.float32).reshape(cols, ld).T[:rows, :].astype(np.float64)


def op_dense(buf, trans, rows, cols, ld):
    d = dense(buf, rows, cols, ld)
    return d.T if wl.is_trans(trans) else d


def problem_dense(p: wl.Problem):
    ar, ac = p.a_shape
    br, bc = p.b_shape
    a = op_dense(p.A, p.transa, ar, ac, p.lda)
    b = op_dense(p.B, p.transb, br, bc, p.ldb)
    c0 = dense(p.C0, p.m, p.n, p.ldc)
    return a, b, c0


def run(o, p: wl.Problem):
    return o.sgemm_f64(p.transa, p.transb, p.m, p.n, p.k, p.alpha, p.A, p.lda, p.B, p.ldb,
                       p.beta, p.C0, p.ldc)


# ---------------------------------------------------------------------------

def pin_fraction_bruteforce(o, seed=1):
    """Exact rational arithmetic on tiny problems: |Cref - exact| and
    |den - exact den| within (k + 2) * 2^-53 * den."""
    rng = np.random.default_rng(seed)
    for case in range(24):
        ta, tb = wl.TRANS_PAIRS[case % 4]
        m, n, k = (int(v) for v in rng.integers(1, 7, size=3))
        alpha = [1.0, -1.5, 0.75, 2.0][case % 4]
        beta = [0.0, 1.0, -0.5, 0.25][(case // 4) % 4]
        p = wl.make_problem(ta, tb, m, n, k, alpha, beta, seed * 1000 + case, pad=case % 3)
        cref, den = run(o, p)
        a, b, c0 = problem_dense(p)
        for i in range(m):
            for j in range(n):
                s = sum((Fraction(a[i, q]) * Fraction(b[q, j]) for q in range(k)), Fraction(0))
                sa = sum((abs(Fraction(a[i, q]) * Fraction(b[q, j])) for q in range(k)),
                         Fraction(0))
                ex = Fraction(alpha) * s
                exd = abs(Fraction(alpha)) * sa
                if beta != 0.0:
                    ex += Fraction(beta) * Fraction(c0[i, j])
                    exd += abs(Fraction(beta)) * abs(Fraction(c0[i, j]))
                bound = (k + 2) * U53 * float(exd) * 1.0001
                assert abs(Fraction(cref[i, j]) - ex) <= Fraction(bound), (case, i, j)
                assert abs(Fraction(den[i, j]) - exd) <= Fraction(bound), (case, i, j)


def pin_numpy_matmul(o, sizes=((67, 45, 129), (130, 70, 33), (1, 90, 17), (40, 1, 300))):
    """Against numpy's float64 matmul (an independent library) with padded
    leading dimensions and NaN padding, every transpose pair."""
    for idx, (m, n, k) in enumerate(sizes):
        for ti, (ta, tb) in enumerate(wl.TRANS_PAIRS):
            p = wl.make_problem(ta, tb, m, n, k, 1.5, -0.5, 77 + 10 * idx + ti, pad=5)
            cref, den = run(o, p)
            a, b, c0 = problem_dense(p)
            ref = 1.5 * (a @ b) + (-0.5) * c0
            refden = 1.5 * (np.abs(a) @ np.abs(b)) + 0.5 * np.abs(c0)
            bound = 4 * (k + 2) * U53 * refden
            assert np.all(np.abs(cref - ref) <= bound), (m, n, k, ta, tb)
            assert np.all(np.abs(den - refden) <= bound), (m, n, k, ta, tb)


def pin_identity_and_permutation(o):
    """A = I gives C = op(B) bit-exactly; a permutation P gives the permuted
    rows; B = P permutes the columns of op(A)."""
    rng = np.random.default_rng(5)
    m = 37
    for tb in ("N", "T"):
        p = wl.make_problem("N", tb, m, 23, m, 1.0, 0.0, 11, pad=3)
        eye = np.zeros((m, m), dtype=np.float32)
        perm = rng.permutation(m)
        eye[np.arange(m), perm] = 1.0  # row i of P picks column perm[i]
        A = np.full(p.lda * m, np.nan, dtype=np.float32)
        A.reshape(m, p.lda)[:, :m] = eye.T  # column-major storage of P
        cref, _ = o.sgemm_f64("N", tb, m, 23, m, 1.0, A, p.lda, p.B, p.ldb, 0.0, None, m)
        _, b, _ = problem_dense(p)
        assert np.array_equal(cref, b[perm, :])
    # B a permutation: C = op(A) with columns permuted
    n = 29
    for ta in ("N", "T"):
        p = wl.make_problem(ta, "N", 31, n, n, 1.0, 0.0, 12, pad=2)
        perm = rng.permutation(n)
        P = np.zeros((n, n), dtype=np.float32)
        P[perm, np.arange(n)] = 1.0  # column j of P selects row perm[j]
        B = np.ascontiguousarray(P.T).reshape(-1)  # column-major, ld = n
        cref, _ = o.sgemm_f64(ta, "N", 31, n, n, 1.0, p.A, p.lda, B, n, 0.0, None, 31)
        a, _, _ = problem_dense(p)
        assert np.array_equal(cref, a[:, perm])


def pin_rank1_closed_form(o):
    """A = u 1^T, B = 1 v^T with small integers: C = alpha k u_i v_j + beta C0."""
    rng = np.random.default_rng(9)
    for ta, tb in wl.TRANS_PAIRS:
        m, n, k = 19, 13, 4096
        u = rng.integers(-8, 9, size=m).astype(np.float32)
        v = rng.integers(-8, 9, size=n).astype(np.float32)
        opa = np.repeat(u[:, None], k, axis=1)  # m x k
        opb = np.repeat(v[None, :], k, axis=0)  # k x n
        sa = opa.T if wl.is_trans(ta) else opa
        sb = opb.T if wl.is_trans(tb) else opb
        A = np.asfortranarray(sa).reshape(-1, order="F")
        B = np.asfortranarray(sb).reshape(-1, order="F")
        C0 = np.random.default_rng(3).uniform(-1, 1, m * n).astype(np.float32)
        for alpha, beta in ((1.0, 0.0), (-2.0, 0.5)):
            cref, den = o.sgemm_f64(ta, tb, m, n, k, alpha, A, sa.shape[0], B, sb.shape[0],
                                    beta, C0, m)
            c0 = C0.reshape(n, m).T.astype(np.float64)
            closed = alpha * k * np.outer(u, v) + (beta * c0 if beta != 0.0 else 0.0)
            assert np.array_equal(cref, closed), (ta, tb, alpha, beta)
            closed_den = abs(alpha) * k * np.outer(np.abs(u), np.abs(v)) + abs(beta) * np.abs(c0)
            assert np.array_equal(den, closed_den)


def pin_integer_regime(o):
    """Entries in {-4..4}: every sum is an exact integer, equal to numpy's
    int64 matmul."""
    rng = np.random.default_rng(21)
    for ta, tb in wl.TRANS_PAIRS:
        m, n, k = 41, 35, 1024
        a = rng.integers(-4, 5, size=(m, k))
        b = rng.integers(-4, 5, size=(k, n))
        sa = a.T if wl.is_trans(ta) else a
        sb = b.T if wl.is_trans(tb) else b
        A = np.asfortranarray(sa, dtype=np.float32).reshape(-1, order="F")
        B = np.asfortranarray(sb, dtype=np.float32).reshape(-1, order="F")
        cref, den = o.sgemm_f64(ta, tb, m, n, k, 1.0, A, sa.shape[0], B, sb.shape[0], 0.0,
                                None, m)
        assert np.array_equal(cref, (a @ b).astype(np.float64))
        assert np.array_equal(den, (np.abs(a) @ np.abs(b)).astype(np.float64))


def pin_degenerate_cases(o):
    """alpha = 0 never reads A or B (NaN there has no effect); beta = 0 never
    reads C0 (NaN there has no effect); k = 0 leaves beta * C0; an empty m or
    n is accepted."""
    m, n, k = 9, 7, 5
    nanA = np.full(m * k, np.nan, dtype=np.float32)
    nanB = np.full(k * n, np.nan, dtype=np.float32)
    C0 = np.linspace(-1, 1, m * n).astype(np.float32)
    c0 = C0.reshape(n, m).T.astype(np.float64)
    cref, den = o.sgemm_f64("N", "N", m, n, k, 0.0, nanA, m, nanB, k, -0.5, C0, m)
    assert np.array_equal(cref, -0.5 * c0) and np.array_equal(den, 0.5 * np.abs(c0))
    cref, den = o.sgemm_f64("N", "N", m, n, 0, 2.0, None, m, None, 1, 3.0, C0, m)
    assert np.array_equal(cref, 3.0 * c0)
    A = np.ones(m * k, dtype=np.float32)
    B = np.ones(k * n, dtype=np.float32)
    nanC = np.full(m * n, np.nan, dtype=np.float32)
    cref, den = o.sgemm_f64("N", "N", m, n, k, 2.0, A, m, B, k, 0.0, nanC, m)
    assert np.array_equal(cref, np.full((m, n), 2.0 * k)) and np.all(np.isfinite(den))
    cref, den = o.sgemm_f64("N", "N", 0, n, k, 1.0, A, 1, B, k, 0.0, None, 1)
    assert cref.shape == (0, n)
    cref, den = o.sgemm_f64("T", "T", m, 0, k, 1.0, A, k, B, 1, 0.0, None, m)
    assert cref.shape == (m, 0)


def pin_transpose_identities(o):
    """(1) 'T' on an explicitly transposed copy equals 'N' on the original,
    bit for bit; (2) (A B)^T = B^T A^T, i.e. sgemm(T, T, n, m, k, B, A) is the
    transpose of sgemm(N, N, m, n, k, A, B), bit for bit (same products, same
    order of summation)."""
    m, n, k = 45, 38, 77
    p = wl.make_problem("N", "N", m, n, k, 1.25, 0.0, 31, pad=4)
    cref, _ = run(o, p)
    a, b, _ = problem_dense(p)
    At = np.asfortranarray(a.T.astype(np.float32)).reshape(-1, order="F")  # k x m, ld = k
    Bt = np.asfortranarray(b.T.astype(np.float32)).reshape(-1, order="F")  # n x k, ld = n
    c2, _ = o.sgemm_f64("T", "T", m, n, k, 1.25, At, k, Bt, n, 0.0, None, m)
    assert np.array_equal(cref, c2)
    c3, _ = o.sgemm_f64("T", "N", m, n, k, 1.25, At, k, p.B, p.ldb, 0.0, None, m)
    assert np.array_equal(cref, c3)
    c4, _ = o.sgemm_f64("N", "T", m, n, k, 1.25, p.A, p.lda, Bt, n, 0.0, None, m)
    assert np.array_equal(cref, c4)
    ct, _ = o.sgemm_f64("T", "T", n, m, k, 1.25, p.B, p.ldb, p.A, p.lda, 0.0, None, n)
    assert np.array_equal(cref, ct.T)
    # the transpose characters: case-insensitive, 'C' (conjugate transpose)
    # equals 'T' for real data
    for ca, cb in (("c", "C"), ("t", "c"), ("C", "t")):
        cc, _ = o.sgemm_f64(ca, cb, m, n, k, 1.25, At, k, Bt, n, 0.0, None, m)
        assert np.array_equal(cref, cc)
    cn, _ = o.sgemm_f64("n", "n", m, n, k, 1.25, p.A, p.lda, p.B, p.ldb, 0.0, None, m)
    assert np.array_equal(cref, cn)


def pin_den_nonnegative_inputs(o):
    """With nonnegative A, B, C0 and alpha, beta >= 0, den equals Cref exactly;
    flipping the sign of A leaves den unchanged."""
    rng = np.random.default_rng(4)
    m, n, k = 23, 19, 211
    A = rng.uniform(0, 1, m * k).astype(np.float32)
    B = rng.uniform(0, 1, k * n).astype(np.float32)
    C0 = rng.uniform(0, 1, m * n).astype(np.float32)
    cref, den = o.sgemm_f64("N", "N", m, n, k, 0.5, A, m, B, k, 2.0, C0, m)
    assert np.array_equal(cref, den)
    cref2, den2 = o.sgemm_f64("N", "N", m, n, k, 0.5, -A, m, B, k, 2.0, C0, m)
    assert np.array_equal(den2, den)
    assert not np.array_equal(cref2, cref)


def pin_entries_match_full(o):
    """The single-entry oracle returns the same numbers as the full oracle."""
    for ta, tb in wl.TRANS_PAIRS:
        p = wl.make_problem(ta, tb, 50, 44, 97, -1.0, 1.0, 55, pad=7)
        cref, den = run(o, p)
        rows = np.repeat(np.arange(p.m), p.n)
        cols = np.tile(np.arange(p.n), p.m)
        ce, de = o.sgemm_f64_entries(p.transa, p.transb, p.m, p.n, p.k, p.alpha, p.A, p.lda,
                                     p.B, p.ldb, p.beta, p.C0, p.ldc, rows, cols)
        assert np.array_equal(ce, cref[rows, cols]) and np.array_equal(de, den[rows, cols])


ALL_SGEMM_PINS = [pin_fraction_bruteforce, pin_numpy_matmul, pin_identity_and_permutation,
                  pin_rank1_closed_form, pin_integer_regime, pin_degenerate_cases,
                  pin_transpose_identities, pin_den_nonnegative_inputs, pin_entries_match_full]


# ---------------------------------------------------------------------------
# bf16 split and the split-precision method
# ---------------------------------------------------------------------------

def pin_bf16_rne_vs_torch(o, count=1 << 22, seed=7):
    """Round-to-nearest-even to bfloat16 equals torch's float32 -> bfloat16
    conversion (a library routine) on random bit patterns, on every exact
    tie and on the edge cases (zeros, infinities, the largest finite value,
    subnormals)."""
    import torch
    rng = np.random.default_rng(seed)
    bits = rng.integers(0, 1 << 32, size=count, dtype=np.uint64).astype(np.uint32)
    ties = (rng.integers(0, 1 << 16, size=4096, dtype=np.uint64).astype(np.uint32) << 16) \
        | np.uint32(0x8000)
    special = np.array([0, 0x80000000, 0x7F800000, 0xFF800000, 0x7F7FFFFF, 0x7F7F7FFF,
                        0x7F7F8000, 0x00000001, 0x00008000, 0x00018000, 0x007FFFFF,
                        0x3F808000, 0x3F818000, 0xBF808000], dtype=np.uint32)
    allbits = np.concatenate([bits, ties, special])
    x = allbits.view(np.float32)
    finite = np.isfinite(x)
    x = x[finite]
    parts = o.bf16x3_split(x)
    ref = torch.from_numpy(x.copy()).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(parts[:, 0], ref)


def pin_bf16x3_exhaustive(o, lo=0, hi=1 << 32):
    """Over every FP32 bit pattern in [lo, hi) inside the split's domain the
    three parts sum to x exactly, stay finite and obey the round-to-nearest
    residual bounds 2^-8 and 2^-16."""
    checked, bad_sum, bad_bound, nonfinite, r1, r2 = o.bf16x3_sweep(lo, hi)
    assert checked > 0
    assert bad_sum == 0 and bad_bound == 0 and nonfinite == 0, (bad_sum, bad_bound, nonfinite)
    assert r1 <= 2.0 ** -8 and r2 <= 2.0 ** -16
    return checked, r1, r2


def pin_bf16x3_digest(o, lo=0x3F000000, hi=0x3F000000 + (1 << 18)):
    """The split digest equals its definition evaluated with numpy on the
    oracle's own parts (the split is pinned above), on a range that also
    holds patterns outside the domain (negative zero side, NaN/Inf are
    excluded by the domain test)."""
    total = 0
    for a, b in ((lo, hi), (0x7F7F0000, 0x7F800010), (0x00000000, 0x00040000)):
        u = np.arange(a, b, dtype=np.uint64)
        x = u.astype(np.uint32).view(np.float32)
        with np.errstate(invalid="ignore"):
            ax = np.abs(x.astype(np.float64))
        keep = (ax >= 2.0 ** -110) & (ax < float(np.uint32(0x7F7F8000).view(np.float32)))
        parts = o.bf16x3_split(x[keep]).astype(np.uint64)
        key = parts[:, 0] | (parts[:, 1] << np.uint64(16)) | (parts[:, 2] << np.uint64(32))
        want = int(np.sum(key * (np.uint64(2) * u[keep] + np.uint64(1)), dtype=np.uint64))
        got = o.bf16x3_split_digest(a, b)
        assert got == want, (hex(a), got, want)
        total += int(keep.sum())
    assert total > 0


def pin_bf16x3_method(o):
    """The split-precision oracle: (1) equals the FP64 oracle exactly on small
    integers (every part past the first is zero and all sums are exact);
    (2) with 16-bit significands the third parts vanish, so no term is dropped
    and the two agree to FP64 rounding; (3) on general data the difference is
    bounded by the dropped terms, (2 * 2^-8 * 2^-16 + 2^-32) |a||b| each."""
    rng = np.random.default_rng(13)
    m, n, k = 33, 29, 150
    for ta, tb in wl.TRANS_PAIRS:
        a = rng.integers(-256, 257, size=m * k).astype(np.float32)
        b = rng.integers(-256, 257, size=k * n).astype(np.float32)
        lda = k if wl.is_trans(ta) else m
        ldb = n if wl.is_trans(tb) else k
        c0 = rng.uniform(-1, 1, m * n).astype(np.float32)
        x = o.sgemm_bf16x3_f64(ta, tb, m, n, k, 1.0, a, lda, b, ldb, 0.0, None, m)
        y, _ = o.sgemm_f64(ta, tb, m, n, k, 1.0, a, lda, b, ldb, 0.0, None, m)
        assert np.array_equal(x, y)
        # 16-bit significands: integers below 2^16 scaled by powers of two
        a16 = (rng.integers(-(1 << 16) + 1, 1 << 16, size=m * k) *
               np.exp2(rng.integers(-20, 0, size=m * k))).astype(np.float32)
        b16 = (rng.integers(-(1 << 16) + 1, 1 << 16, size=k * n) *
               np.exp2(rng.integers(-20, 0, size=k * n))).astype(np.float32)
        x = o.sgemm_bf16x3_f64(ta, tb, m, n, k, 1.5, a16, lda, b16, ldb, -0.5, c0, m)
        y, den = o.sgemm_f64(ta, tb, m, n, k, 1.5, a16, lda, b16, ldb, -0.5, c0, m)
        assert np.all(np.abs(x - y) <= 8 * (k + 2) * U53 * den)
        # general data: bounded by the dropped terms
        p = wl.make_problem(ta, tb, m, n, k, 1.0, 0.0, 99, dist="wide")
        x = o.sgemm_bf16x3_f64(p.transa, p.transb, m, n, k, 1.0, p.A, p.lda, p.B, p.ldb,
                               0.0, None, m)
        y, den = run(o, p)
        drop = (2 * 2.0 ** -24 + 2.0 ** -32) * den + 8 * (k + 2) * U53 * den
        assert np.all(np.abs(x - y) <= drop)
        # and the dropped terms are not all zero on such data
        assert np.any(x != y)


# ---------------------------------------------------------------------------
# Double-precision oracle (Section IV-B): the same facts for FP64 inputs, and
# a cancellation case that an FP64 (not binary128) accumulation gets wrong.
# ---------------------------------------------------------------------------

def dense_d(buf, rows, cols, ld):
    if rows == 0 or cols == 0:
        return np.zeros((rows, cols))
    return np.asarray(buf, dtype=np.float64).reshape(cols, ld).T[:rows, :]


def problem_dense_d(p: wl.Problem):
    ar, ac = p.a_shape
    br, bc = p.b_shape
    a = dense_d(p.A, ar, ac, p.lda)
    b = dense_d(p.B, br, bc, p.ldb)
    a = a.T if wl.is_trans(p.transa) else a
    b = b.T if wl.is_trans(p.transb) else b
    return a, b, dense_d(p.C0, p.m, p.n, p.ldc)


def run_d(o, p: wl.Problem):
    return o.dgemm_f128(p.transa, p.transb, p.m, p.n, p.k, p.alpha, p.A, p.lda, p.B, p.ldb,
                        p.beta, p.C0, p.ldc)


def pin_dgemm_fraction_bruteforce(o, seed=2):
    """Exact rational arithmetic on tiny FP64 problems with full 53-bit
    significands: Cref and den are the exact values rounded once (within
    half an ulp, plus nothing measurable from the binary128 sum)."""
    rng = np.random.default_rng(seed)
    for case in range(24):
        ta, tb = wl.TRANS_PAIRS[case % 4]
        m, n, k = (int(v) for v in rng.integers(1, 7, size=3))
        alpha = [1.0, -1.5, 0.1, 3.0][case % 4]
        beta = [0.0, 1.0, -0.3, 0.25][(case // 4) % 4]
        p = wl.make_problem_d(ta, tb, m, n, k, alpha, beta, seed * 1000 + case, pad=case % 3)
        cref, den = run_d(o, p)
        a, b, c0 = problem_dense_d(p)
        for i in range(m):
            for j in range(n):
                s = sum((Fraction(a[i, q]) * Fraction(b[q, j]) for q in range(k)), Fraction(0))
                sa = sum((abs(Fraction(a[i, q]) * Fraction(b[q, j])) for q in range(k)),
                         Fraction(0))
                ex = Fraction(alpha) * s
                exd = abs(Fraction(alpha)) * sa
                if beta != 0.0:
                    ex += Fraction(beta) * Fraction(c0[i, j])
                    exd += abs(Fraction(beta)) * abs(Fraction(c0[i, j]))
                for got, want in ((cref[i, j], ex), (den[i, j], exd)):
                    ulp = np.spacing(abs(float(want)))
                    assert abs(Fraction(got) - want) <= Fraction(0.5001 * ulp), (case, i, j)


def pin_dgemm_cancellation(o):
    """Sums whose FP64 accumulation loses everything: 1 + 2^-60 - 1 is
    2^-60, and 2^60 + 1 - 2^60 + x is 1 + x."""
    A = np.array([1.0, 2.0 ** -60, -1.0, 2.0 ** 60, 1.0, -2.0 ** 60, 0.375])
    B = np.ones(7)
    cref, _ = o.dgemm_f128("N", "N", 1, 1, 3, 1.0, A[:3], 1, B[:3], 3, 0.0, None, 1)
    assert cref[0, 0] == 2.0 ** -60
    cref, _ = o.dgemm_f128("T", "N", 1, 1, 4, 2.0, A[3:], 4, B[3:], 4, 0.0, None, 1)
    assert cref[0, 0] == 2.0 * 1.375


def pin_dgemm_numpy(o, sizes=((67, 45, 129), (1, 90, 17), (40, 1, 300))):
    """numpy's FP64 matmul (an independent library) agrees within the FP64
    bound of its own rounding; NaN padding is never read."""
    for idx, (m, n, k) in enumerate(sizes):
        for ta, tb in wl.TRANS_PAIRS:
            p = wl.make_problem_d(ta, tb, m, n, k, 1.25, -0.5, 500 + idx, pad=2)
            cref, den = run_d(o, p)
            a, b, c0 = problem_dense_d(p)
            ref = 1.25 * (a @ b) - 0.5 * c0
            assert np.all(np.isfinite(cref))
            assert np.all(np.abs(cref - ref) <= (k + 3) * U53 * den * 1.0001 + 1e-300), (m, n, k)


def pin_dgemm_integer_regime(o):
    """Integers up to 2^20, K = 64: every partial sum is below 2^53, so the
    result is exact and equals numpy's int64 matmul."""
    rng = np.random.default_rng(22)
    for ta, tb in wl.TRANS_PAIRS:
        m, n, k = 23, 17, 64
        a = rng.integers(-2 ** 20, 2 ** 20, size=(m, k))
        b = rng.integers(-2 ** 20, 2 ** 20, size=(k, n))
        sa = a.T if wl.is_trans(ta) else a
        sb = b.T if wl.is_trans(tb) else b
        A = np.asfortranarray(sa, dtype=np.float64).reshape(-1, order="F")
        B = np.asfortranarray(sb, dtype=np.float64).reshape(-1, order="F")
        cref, den = o.dgemm_f128(ta, tb, m, n, k, 1.0, A, sa.shape[0], B, sb.shape[0], 0.0,
                                 None, m)
        assert np.array_equal(cref, (a @ b).astype(np.float64))
        assert np.array_equal(den, (np.abs(a) @ np.abs(b)).astype(np.float64))


def pin_dgemm_identity_and_degenerate(o):
    """A permutation times op(B) is op(B) with rows permuted, bit for bit;
    alpha = 0 or k = 0 never reads A, B; beta = 0 never reads C0."""
    rng = np.random.default_rng(23)
    m, k, n = 9, 9, 7
    perm = rng.permutation(m)
    P = np.zeros((m, k))
    P[np.arange(m), perm] = 1.0
    b = rng.uniform(-1, 1, size=(k, n))
    for tb in ("N", "T"):
        sb = b.T if tb == "T" else b
        B = np.asfortranarray(sb).reshape(-1, order="F")
        cref, _ = o.dgemm_f128("N", tb, m, n, k, 1.0, P.reshape(-1, order="F"), m, B,
                               sb.shape[0], 0.0, None, m)
        assert np.array_equal(cref, b[perm, :])
    nan = np.full(64, np.nan)
    c0 = rng.uniform(-1, 1, 12)
    cref, den = o.dgemm_f128("N", "N", 3, 4, 5, 0.0, nan, 3, nan, 5, -2.0, c0, 3)
    assert np.array_equal(cref, -2.0 * c0.reshape(4, 3).T)
    cref, den = o.dgemm_f128("T", "N", 3, 4, 0, 1.0, nan, 1, nan, 1, 0.5, c0, 3)
    assert np.array_equal(cref, 0.5 * c0.reshape(4, 3).T)
    p = wl.make_problem_d("N", "N", 5, 6, 7, 1.0, 0.0, 24)   # C0 is NaN
    cref, _ = run_d(o, p)
    assert np.all(np.isfinite(cref))


def pin_dgemm_transpose_and_entries(o):
    """T on an explicitly transposed copy equals N bit for bit ('c' as 't');
    the single-entry oracle equals the full one bit for bit."""
    p = wl.make_problem_d("N", "N", 31, 29, 37, -0.75, 0.5, 25, pad=1)
    cref, den = run_d(o, p)
    a, b, _ = problem_dense_d(p)
    at = np.asfortranarray(a.T).reshape(-1, order="F")
    bt = np.asfortranarray(b.T).reshape(-1, order="F")
    c2, d2 = o.dgemm_f128("c", "t", p.m, p.n, p.k, p.alpha, at, p.k, bt, p.n, p.beta, p.C0,
                          p.ldc)
    assert np.array_equal(cref, c2) and np.array_equal(den, d2)
    rows = np.array([0, 30, 5, 17])
    cols = np.array([0, 28, 11, 3])
    ce, de = o.dgemm_f128_entries(p.transa, p.transb, p.m, p.n, p.k, p.alpha, p.A, p.lda,
                                  p.B, p.ldb, p.beta, p.C0, p.ldc, rows, cols)
    assert np.array_equal(ce, cref[rows, cols]) and np.array_equal(de, den[rows, cols])


ALL_DGEMM_PINS = [pin_dgemm_fraction_bruteforce, pin_dgemm_cancellation, pin_dgemm_numpy,
                  pin_dgemm_integer_regime, pin_dgemm_identity_and_degenerate,
                  pin_dgemm_transpose_and_entries]


# ---------------------------------------------------------------------------
# LU with partial pivoting (the factorization of the paper's Linpack run,
# Section IV-C): against LAPACK through scipy, exact rational elimination,
# the reconstruction P A = L U, ties, zero pivots and exact solves.
# ---------------------------------------------------------------------------

def _lu_fraction(a):
    """Textbook elimination with partial pivoting in exact rationals."""
    n = len(a)
    m = [[Fraction(float(v)) for v in row] for row in a]
    piv = []
    for j in range(n):
        p = max(range(j, n), key=lambda i: (abs(m[i][j]), -i))
        piv.append(p)
        m[j], m[p] = m[p], m[j]
        if m[j][j] == 0:
            continue
        for i in range(j + 1, n):
            m[i][j] /= m[j][j]
            for c in range(j + 1, n):
                m[i][c] -= m[i][j] * m[j][c]
    return m, piv


def pin_lu_lapack(o):
    """Same pivots as LAPACK's dgetrf (scipy.linalg.lu_factor), factors
    equal to FP64 rounding."""
    import scipy.linalg as sl
    rng = np.random.default_rng(41)
    for n in (1, 2, 7, 64, 129):
        a = rng.uniform(-1, 1, (n, n)).astype(np.float32)
        lu, piv, info = o.getrf_f64(n, a.reshape(-1, order="F"), n)
        lu2, piv2 = sl.lu_factor(a.astype(np.float64))
        assert info == 0 and np.array_equal(piv, piv2), n
        assert np.max(np.abs(lu - lu2)) <= 1e-12 * max(1.0, np.max(np.abs(lu2))), n


def pin_lu_fraction(o):
    """Exact rational elimination on small integer matrices: identical
    pivots, factors within a few FP64 ulps."""
    rng = np.random.default_rng(42)
    for n in (2, 3, 5, 6):
        for _ in range(3):
            a = rng.integers(-9, 10, (n, n)).astype(np.float32)
            m, piv = _lu_fraction(a)
            lu, ipiv, info = o.getrf_f64(n, a.reshape(-1, order="F"), n)
            assert list(ipiv) == piv
            for i in range(n):
                for j in range(n):
                    want = float(m[i][j])
                    assert abs(lu[i, j] - want) <= 8 * np.spacing(max(abs(want), 1e-300)), (n, i, j)


def pin_lu_reconstruct_ties_singular(o):
    """P A = L U to FP64 roundoff; the first of equal magnitudes is the
    pivot; a zero column reports its 1-based index and leaves the rest
    factored."""
    rng = np.random.default_rng(43)
    n = 40
    a = rng.standard_normal((n, n)).astype(np.float32)
    lu, ipiv, info = o.getrf_f64(n, a.reshape(-1, order="F"), n)
    L = np.tril(lu, -1) + np.eye(n)
    U = np.triu(lu)
    pa = a.astype(np.float64).copy()
    for j, p in enumerate(ipiv):
        pa[[j, p]] = pa[[p, j]]
    assert np.max(np.abs(L @ U - pa)) <= n * 2.0 ** -50 * np.max(np.abs(a))
    t = np.array([[1, 2, 0], [-1, 3, 1], [1, 1, 2]], dtype=np.float32)
    _, ipiv, info = o.getrf_f64(3, t.reshape(-1, order="F"), 3)
    assert ipiv[0] == 0 and info == 0
    s = np.array([[2, 0, 1], [4, 0, 3], [1, 0, 5]], dtype=np.float32)  # zero column 1
    _, _, info = o.getrf_f64(3, s.reshape(-1, order="F"), 3)
    assert info == 2


def pin_lu_exact_solve(o):
    """A = P T with T upper triangular, power-of-two entries: the solve
    reproduces the integer solution exactly."""
    rng = np.random.default_rng(44)
    n = 12
    t = np.triu(2.0 ** rng.integers(-3, 4, (n, n))) * rng.choice([-1.0, 1.0], (n, n))
    t += np.eye(n) * 64.0
    p = np.eye(n)[rng.permutation(n)]
    a = (p @ t).astype(np.float32)
    x = rng.integers(-5, 6, n).astype(np.float64)
    b = a.astype(np.float64) @ x
    lu, ipiv, info = o.getrf_f64(n, a.reshape(-1, order="F"), n)
    assert np.array_equal(o.getrs_f64(lu, ipiv, b), x)


ALL_LU_PINS = [pin_lu_lapack, pin_lu_fraction, pin_lu_reconstruct_ties_singular,
               pin_lu_exact_solve]
