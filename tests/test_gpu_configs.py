"""GPU parity at the full workload sizes (sampled outputs checked one by one
against the oracle), the split on its own, degenerate cases, argument errors,
determinism and transposed-copy invariance."""
import os

import numpy as np
import pytest

import oracle
from paper_1608_05265_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _mg():
    import paper_1608_05265_amd as mg
    return mg


def _free():
    import torch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("size", wl.SQUARE_SIZES)
def test_square_sweep_full_size(size):
    """The benchmark's square sweep, every transpose pair, both forms, in the
    launch configuration the benchmark uses (the tuned default)."""
    for ta, tb in wl.TRANS_PAIRS:
        p = wl.config2(size, ta, tb)
        tensors = gu.dev_problem(p)
        for mode in (0, 1):
            tensors[2].copy_(tensors[2].new_tensor(p.C0))
            out = gu.run(p, mode, tensors=tensors)
            label = "%s mode %d" % (p.label, mode)
            if size <= 1024:
                mx, mean, ratio = gu.check_full(p, out, label)
            else:
                mx, mean, ratio = gu.check_sampled(p, out, count=1024, seed=size, label=label)
            print("%s max/bound %.3e" % (label, ratio))
        del tensors
        _free()


@pytest.mark.parametrize("k", wl.RANKK_KS)
def test_rankk_full_size(k):
    p = wl.config3(k)
    tensors = gu.dev_problem(p)
    for mode in (0, 1):
        tensors[2].copy_(tensors[2].new_tensor(p.C0))
        out = gu.run(p, mode, tensors=tensors)
        mx, mean, ratio = gu.check_sampled(p, out, count=1024, seed=k, label="%s mode %d" %
                                           (p.label, mode))
        print("%s mode %d max/bound %.3e" % (p.label, mode, ratio))
    del tensors
    _free()


# Equal measured error (the split form against native FP32 on the same
# inputs): the split form's maximum and mean normalized error may exceed the
# native ones by at most this factor.
EQUAL_ERROR_RATIO = 1.5


def test_wide_range_both_forms():
    """Entries of both signs spread over 2^-8..2^8, 8192^3: both forms within
    the bound on the same inputs, and the split form's maximum and mean
    normalized error at most EQUAL_ERROR_RATIO times the native form's."""
    p = wl.config4()
    tensors = gu.dev_problem(p)
    stats = {}
    for mode in (0, 1):
        out = gu.run(p, mode, tensors=tensors)
        stats[mode] = gu.check_sampled(p, out, count=2048, seed=4, label="wide mode %d" % mode)
    print("wide 8192^3: fp32 max %.3e mean %.3e | bf16x3 max %.3e mean %.3e"
          % (stats[0][0], stats[0][1], stats[1][0], stats[1][1]))
    assert stats[1][0] <= EQUAL_ERROR_RATIO * stats[0][0], "max error not equal"
    assert stats[1][1] <= EQUAL_ERROR_RATIO * stats[0][1], "mean error not equal"
    del tensors
    _free()


def test_same_sign_long_k_every_config():
    """Entries uniform in [0, 1] (same sign: the bound's denominator equals
    the result, so no cancellation hides accumulation error) at K = 8192,
    ragged M and N over several tiles: every compiled configuration of both
    forms within the bound, and the split form's error equal to the native
    one's (EQUAL_ERROR_RATIO) on the same K schedule: every whole-K split-form
    configuration against the native whole-K sum (one FP32 accumulator in k
    order, the same bits for every native configuration), the small tiles
    whose waves split the k steps against their native counterpart, and the
    default choices (split-K for this few-tile shape) against each other."""
    mg = _mg()
    p = wl.make_problem("N", "N", 300, 270, 8192, 1.0, 0.0, wl.seed_for(8, 1), dist="unit")
    cref, den = oracle.sgemm_f64(p.transa, p.transb, p.m, p.n, p.k, p.alpha, p.A, p.lda, p.B,
                                 p.ldb, p.beta, p.C0, p.ldc)
    tensors = gu.dev_problem(p)
    err = {}
    for mode in (0, 1):
        for cfg in [None] + mg.configs(mode):
            out = gu.run(p, mode, config_id=None if cfg is None else cfg["id"], tensors=tensors)
            ok, mx, mean, ratio = oracle.check(gu.c_dense(p, out), cref, den, p.k)
            name = "default" if cfg is None else cfg["name"]
            assert ok, "%s mode %d: max/bound %.3e" % (name, mode, ratio)
            assert gu.padding_untouched(p, out)
            err[(mode, name)] = (mx, mean)
            print("same-sign K=8192 %s mode %d: max %.3e mean %.3e (%.2e of bound)"
                  % (name, mode, mx, mean, ratio))
    # K schedules: "default" (the dispatcher's choice), "kW" for the small
    # tiles whose W waves take every W-th k step (names ending in _kW), "rW"
    # for the register tiles whose W waves take every W-th 64-k chunk (names
    # ending in _rW), and "whole" (one accumulator over k in order) for every
    # other tile; native configurations with the same schedule give the same
    # bits
    def schedule(name):
        if name == "default":
            return name
        tail = name.rsplit("_", 1)[-1]
        return tail if tail[0] in "kr" and tail[1:].isdigit() else "whole"
    native = {}
    for (mode, name), v in err.items():
        if mode == 0:
            native.setdefault(schedule(name), v)
            assert v == native[schedule(name)], "%s differs from its schedule's bits" % name
    for (mode, name), (mx, mean) in err.items():
        if mode != 1:
            continue
        ref = native[schedule(name)]
        assert mx <= EQUAL_ERROR_RATIO * ref[0], "%s: max %.3e vs native %.3e" % (name, mx, ref[0])
        assert mean <= EQUAL_ERROR_RATIO * ref[1], "%s: mean %.3e vs native %.3e" % (
            name, mean, ref[1])
    del tensors
    _free()


def test_split_matches_oracle_bit_exact():
    """The GPU split (v_cvt_pk_bf16_f32 + FP32 residuals) equals the oracle's
    split bit for bit: every significand at several binades, random bit
    patterns over the whole domain, and edge values."""
    import torch
    mg = _mg()
    mant = np.arange(1 << 23, dtype=np.uint32)
    blocks = [((np.uint32(e) << 23) | mant) for e in (1, 17, 126, 127, 128, 200, 253)]
    rng = np.random.default_rng(5)
    rnd = rng.integers(0, 1 << 32, size=1 << 22, dtype=np.uint64).astype(np.uint32)
    edge = np.array([0x7F7F7FFF, 0x0C800000, 0x3F808000, 0x3F818000, 0x00000000, 0x80000000],
                    dtype=np.uint32)
    bits = np.concatenate(blocks + [rnd, edge])
    bits = np.concatenate([bits, bits | np.uint32(0x80000000)])
    x = bits.view(np.float32)
    ax = np.abs(x)
    keep = np.isfinite(x) & ((ax >= 2.0 ** -110) | (ax == 0)) & (ax < np.float32(3.3e38))
    x = np.ascontiguousarray(x[keep])
    xd = torch.from_numpy(x).cuda()
    parts = torch.empty(3 * x.size, dtype=torch.int16, device="cuda")
    mg.bf16x3_split(xd, x.size, parts)
    torch.cuda.synchronize()
    got = parts.cpu().numpy().view(np.uint16).reshape(-1, 3)
    ref = oracle.bf16x3_split(x)
    bad = np.nonzero(np.any(got != ref, axis=1))[0]
    assert bad.size == 0, "first mismatch at x=%r: gpu %s oracle %s" % (
        x[bad[0]], got[bad[0]], ref[bad[0]])


def test_split_exhaustive_against_oracle_digest():
    """All 2^32 FP32 bit patterns through the GPU split, in chunks: for every
    chunk the digest of the GPU parts over the split's domain (finite,
    2^-110 <= |x| < 0x1.fefp127) equals the oracle's digest of its own
    parts (sum mod 2^64 of (p0 | p1 << 16 | p2 << 32) * (2u + 1)); a
    single differing part changes it."""
    import torch
    mg = _mg()
    dev = torch.device("cuda:0")
    chunk = 1 << 26
    lo_mag = torch.tensor(2.0 ** -110, dtype=torch.float32, device=dev)
    hi_mag = torch.tensor([0x7F7F8000], dtype=torch.int32).view(torch.float32).to(dev)
    mod = 1 << 64
    bad = []
    for c in range((1 << 32) // chunk):
        lo = c * chunk
        u = torch.arange(lo, lo + chunk, dtype=torch.int64, device=dev)
        x = torch.where(u >= (1 << 31), u - (1 << 32), u).to(torch.int32).view(torch.float32)
        parts = torch.empty(3 * chunk, dtype=torch.int16, device=dev)
        mg.bf16x3_split(x, chunk, parts)
        ax = x.abs()
        keep = (ax >= lo_mag) & (ax < hi_mag)
        p = parts.view(chunk, 3).to(torch.int64) & 0xFFFF
        key = p[:, 0] | (p[:, 1] << 16) | (p[:, 2] << 32)
        got = int(torch.where(keep, key * (2 * u + 1), torch.zeros_like(key)).sum().item()) % mod
        want = oracle.bf16x3_split_digest(lo, lo + chunk)
        if got != want:
            bad.append(hex(lo))
        del u, x, parts, ax, keep, p, key
    assert not bad, "split digests differ in the chunks starting at %s" % bad


@pytest.mark.parametrize("mode", [0, 1], ids=["fp32", "bf16x3"])
def test_degenerate_cases(mode):
    import torch
    mg = _mg()
    m, n, k = 37, 29, 23
    p = wl.make_problem("N", "N", m, n, k, 1.0, 0.5, 3, pad=2)
    A, B, C = gu.dev_problem(p)
    nanA = torch.full_like(A, float("nan"))
    nanB = torch.full_like(B, float("nan"))
    # alpha = 0: A and B are not read
    mg.sgemm("N", "N", m, n, k, 0.0, nanA, p.lda, nanB, p.ldb, -2.0, C, p.ldc, mode=mode)
    out = C.cpu().numpy()
    c0 = gu.c_dense(p, p.C0).astype(np.float64)
    assert np.array_equal(gu.c_dense(p, out), (-2.0 * c0).astype(np.float32))
    assert gu.padding_untouched(p, out)
    # alpha = 0, beta = 1: quick return, C bit-identical
    C.copy_(C.new_tensor(p.C0))
    mg.sgemm("N", "N", m, n, k, 0.0, nanA, p.lda, nanB, p.ldb, 1.0, C, p.ldc, mode=mode)
    assert np.array_equal(C.cpu().numpy().view(np.uint32), p.C0.view(np.uint32))
    # k = 0, beta = 0: C = 0 even over NaN
    C.fill_(float("nan"))
    mg.sgemm("N", "N", m, n, 0, 1.0, A, p.lda, B, 1, 0.0, C, p.ldc, mode=mode)
    out = C.cpu().numpy()
    assert np.all(gu.c_dense(p, out) == 0)
    # beta = 0 with NaN in C: C = alpha * A * B, no NaN
    C.fill_(float("nan"))
    mg.sgemm("N", "N", m, n, k, 1.0, A, p.lda, B, p.ldb, 0.0, C, p.ldc, mode=mode)
    out = C.cpu().numpy()
    cref, den = oracle.sgemm_f64("N", "N", m, n, k, 1.0, p.A, p.lda, p.B, p.ldb, 0.0, None,
                                 p.ldc)
    ok, mx, _, _ = oracle.check(gu.c_dense(p, out), cref, den, k)
    assert ok
    # m = 0 / n = 0: nothing touched
    C.copy_(C.new_tensor(p.C0))
    mg.sgemm("N", "N", 0, n, k, 1.0, A, 1, B, p.ldb, 0.0, C, 1, mode=mode)
    mg.sgemm("N", "N", m, 0, k, 1.0, A, p.lda, B, p.ldb, 0.0, C, p.ldc, mode=mode)
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy().view(np.uint32), p.C0.view(np.uint32))


def test_argument_errors_leave_c_untouched():
    import torch
    mg = _mg()
    p = wl.make_problem("N", "N", 16, 16, 16, 1.0, 0.0, 4)
    A, B, C = gu.dev_problem(p)
    before = C.clone()
    for kwargs, code in ((dict(lda=8), -8), (dict(ldb=8), -10), (dict(ldc=8), -13),
                         (dict(transa="Z"), -1), (dict(mode=5), -14)):
        args = dict(transa="N", transb="N", lda=16, ldb=16, ldc=16, mode=0)
        args.update(kwargs)
        with pytest.raises(mg.MisgemmError) as ei:
            mg.sgemm(args["transa"], args["transb"], 16, 16, 16, 1.0, A, args["lda"], B,
                     args["ldb"], 0.0, C, args["ldc"], mode=args["mode"])
        assert ei.value.status == code
    torch.cuda.synchronize()
    assert torch.equal(C.view(torch.int32), before.view(torch.int32))


@pytest.mark.parametrize("mode", [0, 1], ids=["fp32", "bf16x3"])
def test_run_to_run_bitwise_determinism(mode):
    """Same inputs, same configuration, same bits (also guards against LDS
    races, which would show up as nondeterminism)."""
    mg = _mg()
    for cfg in mg.configs(mode):
        p = wl.make_problem("T", "N", 3 * cfg["bm"] + 5, 2 * cfg["bn"] + 3, 257, 1.0, 0.0,
                            70 + cfg["id"])
        tensors = gu.dev_problem(p)
        first = gu.run(p, mode, config_id=cfg["id"], tensors=tensors).copy()
        for _ in range(2):
            again = gu.run(p, mode, config_id=cfg["id"], tensors=tensors)
            assert np.array_equal(first.view(np.uint32), again.view(np.uint32)), cfg["name"]


@pytest.mark.parametrize("mode", [0, 1], ids=["fp32", "bf16x3"])
def test_transposed_copy_gives_same_bits(mode):
    """Staging canonicalizes the operands: 'T' on an explicitly transposed
    copy equals 'N' on the original bit for bit, for every configuration."""
    import torch
    mg = _mg()
    for cfg in mg.configs(mode):
        m, n, k = cfg["bm"] + 9, cfg["bn"] + 17, 3 * cfg["bk"] + 1
        p = wl.make_problem("N", "N", m, n, k, 1.0, 0.0, 90 + cfg["id"])
        a = p.A.reshape(k, m).T  # m x k
        b = p.B.reshape(n, k).T  # k x n
        At = np.ascontiguousarray(a).reshape(-1)  # column-major storage of a^T (k x m)
        Bt = np.ascontiguousarray(b).reshape(-1)  # column-major storage of b^T (n x k)
        outs = []
        for (ta, tb, Ah, lda, Bh, ldb) in (("N", "N", p.A, m, p.B, k), ("T", "N", At, k, p.B, k),
                                           ("N", "T", p.A, m, Bt, n), ("T", "T", At, k, Bt, n)):
            A = torch.from_numpy(Ah).cuda()
            B = torch.from_numpy(Bh).cuda()
            C = torch.zeros(m * n, device="cuda")
            mg.sgemm_config(ta, tb, m, n, k, 1.0, A, lda, B, ldb, 0.0, C, m, mode, cfg["id"])
            torch.cuda.synchronize()
            outs.append(C.cpu().numpy())
        for o in outs[1:]:
            assert np.array_equal(o.view(np.uint32), outs[0].view(np.uint32)), cfg["name"]


def test_non_default_stream():
    import torch
    mg = _mg()
    p = wl.make_problem("N", "T", 300, 200, 100, 1.0, 0.0, 8)
    A, B, C = gu.dev_problem(p)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        mg.sgemm("N", "T", p.m, p.n, p.k, 1.0, A, p.lda, B, p.ldb, 0.0, C, p.ldc, stream=s)
    s.synchronize()
    gu.check_full(p, C.cpu().numpy(), "side stream")


def test_concurrent_host_threads_on_own_streams():
    """Four host threads, each on its own stream with its own C, run the
    packed bf16x3 path (4096^3 NT through an explicit packed configuration,
    library scratch per stream) and split-K
    (128x512x8192, partial tiles in that scratch) at the same time, five
    rounds each: every result equals, bit for bit, the same call made alone
    on the default stream (the split-K ones are also checked against the
    oracle) -- no call sees another stream's scratch."""
    import threading
    import torch
    mg = _mg()
    big = wl.make_problem("N", "T", 4096, 4096, 4096, 1.0, 0.5, 8400)
    skinny = wl.make_problem("N", "N", 128, 512, 8192, 1.5, -0.5, 8401)
    jobs = [(big, 1), (big, 1), (skinny, 0), (skinny, 1)]
    dev = {id(p): gu.dev_problem(p) for p in (big, skinny)}
    packed_id = [c["id"] for c in mg.configs(1) if c["packed"]][0]

    def call(p, mode, A, B, C, stream=None):
        # the big problem through an explicit packed configuration (library
        # panels per stream), the skinny one through the default dispatch
        # (split-K, library partial tiles per stream)
        if p is big:
            mg.sgemm_config(p.transa, p.transb, p.m, p.n, p.k, p.alpha, A, p.lda, B, p.ldb,
                            p.beta, C, p.ldc, mode, packed_id, stream=stream)
        else:
            mg.sgemm(p.transa, p.transb, p.m, p.n, p.k, p.alpha, A, p.lda, B, p.ldb, p.beta, C,
                     p.ldc, mode=mode, stream=stream)
    refs = []
    for p, mode in jobs:
        A, B, _ = dev[id(p)]
        C = torch.from_numpy(p.C0.copy()).to(A.device)
        call(p, mode, A, B, C)
        torch.cuda.synchronize()
        refs.append(C.cpu().numpy().view(np.uint32).copy())
    for (p, mode), ref in zip(jobs[2:], refs[2:]):
        gu.check_full(p, ref.view(np.float32), "skinny mode %d" % mode)
    errors = []

    def worker(i):
        try:
            p, mode = jobs[i]
            A, B, _ = dev[id(p)]
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                C0 = torch.from_numpy(p.C0.copy()).to(A.device)
                C = torch.empty_like(C0)
                for _ in range(5):
                    C.copy_(C0)
                    call(p, mode, A, B, C, stream=s)
                    s.synchronize()
                    got = C.cpu().numpy().view(np.uint32)
                    if not np.array_equal(got, refs[i]):
                        errors.append("job %d differs from its single-stream result" % i)
                        return
        except Exception as e:  # reported below
            errors.append("job %d: %r" % (i, e))

    threads = [threading.Thread(target=worker, args=(i,)) for i in range(len(jobs))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors


def test_packed_path_caller_workspace_and_capture():
    """The packed bf16x3 path with a caller-owned workspace: same bits as the
    library-owned one, argument errors for a short or misaligned workspace,
    and capture into a HIP graph (the call allocates nothing)."""
    import torch
    mg = _mg()
    packed = [c for c in mg.configs(1) if c["packed"]]
    assert packed
    p = wl.make_problem("T", "N", 700, 520, 300, 1.5, -0.5, 123, pad=3)
    A, B, C = gu.dev_problem(p)
    need = mg.workspace_size("T", "N", p.m, p.n, p.k, 1)
    assert need > 0 and mg.workspace_size("T", "N", p.m, p.n, p.k, 0) == 0
    ws = torch.empty((need + 3) // 4, dtype=torch.float32, device="cuda")
    ref = gu.run(p, 1, config_id=packed[0]["id"], tensors=(A, B, C)).copy()
    gu.check_full(p, ref, "packed via library workspace")
    mg.load_tuning(None)  # heuristics: a packed config only with a workspace
    try:
        assert mg.config_info(mg.select_config("T", "N", 4096, 4096, 4096, 1))["packed"] == 0
        C.copy_(C.new_tensor(p.C0))
        mg.sgemm_ws("T", "N", p.m, p.n, p.k, p.alpha, A, p.lda, B, p.ldb, p.beta, C, p.ldc, 1,
                    ws, need)
        torch.cuda.synchronize()
        gu.check_full(p, C.cpu().numpy(), "packed via caller workspace")
        with pytest.raises(mg.MisgemmError) as ei:
            mg.sgemm_ws("T", "N", p.m, p.n, p.k, p.alpha, A, p.lda, B, p.ldb, p.beta, C, p.ldc,
                        1, ws, need - 1)
        assert ei.value.status == -16
        with pytest.raises(mg.MisgemmError) as ei:
            mg.sgemm_ws("T", "N", p.m, p.n, p.k, p.alpha, A, p.lda, B, p.ldb, p.beta, C, p.ldc,
                        1, ws.data_ptr() + 4, need)
        assert ei.value.status == -15
        # capture: the caller workspace makes the call allocation-free
        g = torch.cuda.CUDAGraph()
        C.copy_(C.new_tensor(p.C0))
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            mg.sgemm_ws("T", "N", p.m, p.n, p.k, p.alpha, A, p.lda, B, p.ldb, p.beta, C, p.ldc,
                        1, ws, need)
        for rep in range(3):
            C.copy_(C.new_tensor(p.C0))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            gu.check_full(p, C.cpu().numpy(), "graph replay %d" % rep)
    finally:
        if os.path.exists(mg.TUNING_PATH):
            mg.load_tuning(mg.TUNING_PATH)
    mg.release_workspace()
