"""Split-K (each of `splits` workgroups of a C tile computes a K range and
stores a partial tile; a second kernel adds the partials in split order):
results against the
oracle, bit-for-bit reproducibility, exact agreement with the whole-K path
where the arithmetic is exact, graph capture and replay, and independent
scratch per stream."""
import numpy as np
import pytest

from paper_1608_05265_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _mg():
    import paper_1608_05265_amd as mg
    return mg


def _split(p, mode, cfg, splits, tensors, stream=None):
    import torch
    mg = _mg()
    A, B, C = tensors
    mg.sgemm_split(p.transa, p.transb, p.m, p.n, p.k, p.alpha, A, p.lda, B, p.ldb, p.beta, C,
                   p.ldc, mode, config_id=cfg, splits=splits, stream=stream)
    torch.cuda.synchronize()
    return C.cpu().numpy()[:p.C0.size]


def _reset(C, p):
    C.copy_(C.new_tensor(p.C0))


@pytest.mark.parametrize("mode", [0, 1], ids=["fp32", "bf16x3"])
def test_every_split_config_against_oracle(mode):
    """Every configuration with a split-K variant, every transpose pair,
    ragged M/N/K and padded leading dimensions, several split counts
    (including more splits than K blocks, which the library reduces)."""
    mg = _mg()
    cfgs = [c for c in mg.configs(mode) if c["splitk"]]
    assert cfgs
    for ci, c in enumerate(cfgs):
        for ti, (ta, tb) in enumerate([("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")]):
            p = wl.make_problem(ta, tb, 150 + 37 * ti, 97 + 29 * ci, 777, 1.5, -0.5,
                                9000 + 10 * ci + ti, pad=3)
            t = gu.dev_problem(p)
            for splits in (2, 3, 7, 64):
                _reset(t[2], p)
                out = _split(p, mode, c["id"], splits, t)
                gu.check_full(p, out, "%s %s%s splits=%d" % (c["name"], ta, tb, splits))


@pytest.mark.parametrize("mode", [0, 1], ids=["fp32", "bf16x3"])
def test_split_is_reproducible_and_exact_on_integers(mode):
    """Two runs give the same bits whatever order the splits ran in; with small
    integer inputs every sum is exact, so split-K equals the whole-K path
    bit for bit."""
    mg = _mg()
    c = [c for c in mg.configs(mode) if c["splitk"]][0]
    p = wl.make_problem("N", "T", 256, 192, 2048, 1.0, 1.0, 77)
    rng = np.random.default_rng(78)
    p.A[:] = rng.integers(-4, 5, size=p.A.size)
    p.B[:] = rng.integers(-4, 5, size=p.B.size)
    t = gu.dev_problem(p)
    whole = gu.run(p, mode, config_id=c["id"], tensors=t).copy()
    outs = []
    for splits in (4, 4, 16):
        _reset(t[2], p)
        outs.append(_split(p, mode, c["id"], splits, t).copy())
    assert np.array_equal(outs[0].view(np.uint32), outs[1].view(np.uint32))
    for o in outs:
        assert np.array_equal(o.view(np.uint32), whole.view(np.uint32))
    gu.check_full(p, outs[0], "integer split")


@pytest.mark.parametrize("mode", [0, 1], ids=["fp32", "bf16x3"])
def test_automatic_split_on_small_problems(mode):
    """misgemm_sgemm on problems whose tiles leave CUs idle: the 256^3 case
    (K too short to split) and a skinny one with long K (split by the
    heuristics); results stay within the bound and reproducible."""
    mg = _mg()
    for p in (wl.config1(), wl.make_problem("T", "N", 96, 200, 4000, -1.0, 0.5, 31, pad=1)):
        t = gu.dev_problem(p)
        a = gu.run(p, mode, tensors=t).copy()
        gu.check_full(p, a, "auto split %dx%dx%d" % (p.m, p.n, p.k))
        _reset(t[2], p)
        b = gu.run(p, mode, tensors=t).copy()
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    mg.release_workspace()


def test_split_in_graph_replays():
    """A split-K call captured into a HIP graph (its scratch already exists):
    every replay, with eager work between replays, equals the eager result
    bit for bit."""
    import torch
    mg = _mg()
    c = [c for c in mg.configs(0) if c["splitk"]][0]
    p = wl.make_problem("T", "T", 300, 260, 1500, 1.25, 0.75, 55, pad=2)
    A, B, C = gu.dev_problem(p)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        eager = _split(p, 0, c["id"], 5, (A, B, C), stream=s).copy()
    gu.check_full(p, eager, "eager split")
    g = torch.cuda.CUDAGraph()
    _reset(C, p)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        mg.sgemm_split(p.transa, p.transb, p.m, p.n, p.k, p.alpha, A, p.lda, B, p.ldb, p.beta, C,
                       p.ldc, 0, config_id=c["id"], splits=5, stream=s)
    for rep in range(4):
        _reset(C, p)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        out = C.cpu().numpy()[:p.C0.size]
        assert np.array_equal(out.view(np.uint32), eager.view(np.uint32)), "replay %d" % rep
        # unrelated eager work between replays
        x = torch.rand(1 << 20, device="cuda")
        (x * 2).sum().item()
    del g
    mg.release_workspace()


def test_split_capture_without_scratch_is_refused():
    """Forcing split-K on a stream whose scratch does not exist yet, while it
    is capturing, is refused (no allocation during capture); the automatic
    path on the same stream falls back to whole-K tiles and is captured."""
    import torch
    mg = _mg()
    mg.release_workspace()
    c = [c for c in mg.configs(0) if c["splitk"]][0]
    p = wl.make_problem("N", "N", 128, 128, 1024, 1.0, 0.0, 56)
    A, B, C = gu.dev_problem(p)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    status = None
    with torch.cuda.graph(g, stream=s):
        try:
            mg.sgemm_split("N", "N", p.m, p.n, p.k, 1.0, A, p.lda, B, p.ldb, 0.0, C, p.ldc, 0,
                           config_id=c["id"], splits=4, stream=s)
        except mg.MisgemmError as e:
            status = e.status
        mg.sgemm("N", "N", p.m, p.n, p.k, 1.0, A, p.lda, B, p.ldb, 0.0, C, p.ldc, 0, stream=s)
    assert status == 1002
    g.replay()
    torch.cuda.synchronize()
    gu.check_full(p, C.cpu().numpy()[:p.C0.size], "captured fallback")


def test_streams_have_their_own_scratch():
    """Split-K calls in flight on two streams at once use separate partial
    buffers: both results are right."""
    import torch
    mg = _mg()
    c = [c for c in mg.configs(0) if c["splitk"]][0]
    ps = [wl.make_problem("N", "T", 192, 160, 3000, 1.0, 0.0, 60 + i) for i in range(2)]
    ts = [gu.dev_problem(p) for p in ps]
    streams = [torch.cuda.Stream() for _ in ps]
    torch.cuda.synchronize()
    for _ in range(3):
        for p, (A, B, C), s in zip(ps, ts, streams):
            mg.sgemm_split(p.transa, p.transb, p.m, p.n, p.k, 1.0, A, p.lda, B, p.ldb, 0.0, C,
                           p.ldc, 0, config_id=c["id"], splits=6, stream=s)
    torch.cuda.synchronize()
    for p, (A, B, C) in zip(ps, ts):
        gu.check_full(p, C.cpu().numpy()[:p.C0.size], "stream scratch")
    mg.release_workspace()


def test_split_errors():
    mg = _mg()
    p = wl.make_problem("N", "N", 64, 64, 64, 1.0, 0.0, 57)
    A, B, C = gu.dev_problem(p)
    nosplit = [c for c in mg.configs(0) if not c["splitk"] and not c["packed"]][0]
    with pytest.raises(mg.MisgemmError) as ei:
        mg.sgemm_split("N", "N", 64, 64, 64, 1.0, A, 64, B, 64, 0.0, C, 64, 0,
                       config_id=nosplit["id"], splits=2)
    assert ei.value.status == 1001
    # splits = 1 on any configuration is the whole-K path
    mg.sgemm_split("N", "N", 64, 64, 64, 1.0, A, 64, B, 64, 0.0, C, 64, 0,
                   config_id=nosplit["id"], splits=1)
