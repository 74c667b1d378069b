"""Helpers for the GPU tests: move a seeded problem to the device, run the
library through its C-ABI binding, and check the result against the oracle."""
from __future__ import annotations

import numpy as np

import oracle
from paper_1608_05265_amd import workloads as wl


def dev_problem(p: wl.Problem):
    import torch
    d = torch.device("cuda:0")
    A = torch.from_numpy(p.A).to(d) if p.A.size else torch.empty(1, device=d)
    B = torch.from_numpy(p.B).to(d) if p.B.size else torch.empty(1, device=d)
    C = torch.from_numpy(p.C0.copy()).to(d) if p.C0.size else torch.empty(1, device=d)
    return A, B, C


def run(p: wl.Problem, mode, config_id=None, tensors=None):
    """Run p on the GPU; returns the C storage as a float32 numpy array."""
    import torch
    import paper_1608_05265_amd as mg
    A, B, C = tensors if tensors is not None else dev_problem(p)
    if config_id is None:
        mg.sgemm(p.transa, p.transb, p.m, p.n, p.k, p.alpha, A, p.lda, B, p.ldb, p.beta, C,
                 p.ldc, mode=mode)
    else:
        mg.sgemm_config(p.transa, p.transb, p.m, p.n, p.k, p.alpha, A, p.lda, B, p.ldb,
                        p.beta, C, p.ldc, mode, config_id)
    torch.cuda.synchronize()
    return C.cpu().numpy()[:p.C0.size]


def c_dense(p: wl.Problem, out: np.ndarray) -> np.ndarray:
    return out.reshape(p.n, p.ldc).T[:p.m, :] if p.m and p.n else np.zeros((p.m, p.n))


def padding_untouched(p: wl.Problem, out: np.ndarray) -> bool:
    if p.ldc == p.m or p.n == 0:
        return True
    a = out.reshape(p.n, p.ldc)[:, p.m:].view(np.uint32)
    b = p.C0.reshape(p.n, p.ldc)[:, p.m:].view(np.uint32)
    return bool(np.array_equal(a, b))


def check_full(p: wl.Problem, out: np.ndarray, label=""):
    cref, den = oracle.sgemm_f64(p.transa, p.transb, p.m, p.n, p.k, p.alpha, p.A, p.lda, p.B,
                                 p.ldb, p.beta, p.C0, p.ldc)
    ok, mx, mean, ratio = oracle.check(c_dense(p, out), cref, den, p.k)
    assert padding_untouched(p, out), "C padding written " + label
    assert ok, "%s: max normalized error %.3e exceeds bound %.3e" % (label, mx, oracle.tol(p.k))
    return mx, mean, ratio


def sample_entries(p: wl.Problem, count: int, seed: int):
    """Random entries plus the corners and last row/column of every edge."""
    rng = np.random.default_rng(seed)
    rows = list(rng.integers(0, p.m, size=count))
    cols = list(rng.integers(0, p.n, size=count))
    for r in (0, p.m - 1):
        for c in range(0, p.n, max(1, p.n // 64)):
            rows.append(r)
            cols.append(c)
    for c in (0, p.n - 1):
        for r in range(0, p.m, max(1, p.m // 64)):
            rows.append(r)
            cols.append(c)
    return np.array(rows, dtype=np.int64), np.array(cols, dtype=np.int64)


def check_sampled(p: wl.Problem, out: np.ndarray, count=2048, seed=0, label=""):
    rows, cols = sample_entries(p, count, seed)
    cref, den = oracle.sgemm_f64_entries(p.transa, p.transb, p.m, p.n, p.k, p.alpha, p.A, p.lda,
                                         p.B, p.ldb, p.beta, p.C0, p.ldc, rows, cols)
    got = out[rows + cols * p.ldc]
    ok, mx, mean, ratio = oracle.check(got, cref, den, p.k)
    assert padding_untouched(p, out), "C padding written " + label
    assert ok, "%s: max normalized error %.3e exceeds bound %.3e" % (label, mx, oracle.tol(p.k))
    return mx, mean, ratio
