"""The allocation-free entry point misgemm_sgemm_split_noalloc against the
entry point it is a variant of, misgemm_sgemm_split: the same configuration
and split factor give the same bits, on two calls in a row (the second one
smaller, so it runs on what the first left in the static array), both
forms, within the bound against the oracle; a request beyond the static
array is refused with C untouched; and the call replays correctly from a
captured HIP graph."""
import numpy as np
import pytest

from paper_1608_05265_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

MISGEMM_E_SCRATCH = 1007
STATIC_BYTES = 64 << 20


def _split_config(mg, mode):
    """The split-capable configuration with the smallest tile (the choice of
    both entry points for config_id -1)."""
    c = [c for c in mg.configs(mode) if c["splitk"]]
    return min(c, key=lambda c: c["bm"] * c["bn"])


def _both(mg, torch, p, mode, splits):
    A, B, C = gu.dev_problem(p)
    C2 = torch.from_numpy(p.C0.copy()).to(C.device)
    torch.cuda.synchronize()
    mg.sgemm_split(p.transa, p.transb, p.m, p.n, p.k, p.alpha, A, p.lda, B, p.ldb, p.beta, C,
                   p.ldc, mode, -1, 0, splits)
    mg.sgemm_split_noalloc(p.transa, p.transb, p.m, p.n, p.k, p.alpha, A, p.lda, B, p.ldb,
                           p.beta, C2, p.ldc, mode, -1, 0, splits)
    torch.cuda.synchronize()
    return C.cpu().numpy(), C2.cpu().numpy(), (A, B, C2)


@pytest.mark.parametrize("mode", [0, 1], ids=["fp32", "bf16x3"])
def test_noalloc_matches_split_entry_point(mode):
    import torch
    import paper_1608_05265_amd as mg
    cfg = _split_config(mg, mode)
    first = wl.make_problem("N", "N", 128, 512, 8192, 1.5, -0.5, 7100 + mode)
    second = wl.make_problem("T", "N", 100, 300, 3000, -1.0, 0.5, 7200 + mode, pad=3)
    for p, splits in ((first, 16), (second, 4)):
        tiles = -(-p.m // cfg["bm"]) * -(-p.n // cfg["bn"])
        assert splits * tiles * cfg["bm"] * cfg["bn"] * 4 <= STATIC_BYTES
        ref, got, _ = _both(mg, torch, p, mode, splits)
        assert np.array_equal(ref.view(np.uint32), got.view(np.uint32)), p.label
        gu.check_full(p, got, "noalloc %dx%dx%d mode %d" % (p.m, p.n, p.k, mode))


def test_noalloc_refuses_beyond_the_static_array():
    import torch
    import paper_1608_05265_amd as mg
    cfg = _split_config(mg, 0)
    p = wl.make_problem("N", "N", 4096, 4096, 512, 1.0, 0.0, 7300)
    tiles = -(-p.m // cfg["bm"]) * -(-p.n // cfg["bn"])
    assert 8 * tiles * cfg["bm"] * cfg["bn"] * 4 > STATIC_BYTES
    A, B, C = gu.dev_problem(p)
    before = C.clone()
    with pytest.raises(mg.MisgemmError) as ei:
        mg.sgemm_split_noalloc("N", "N", p.m, p.n, p.k, 1.0, A, p.lda, B, p.ldb, 0.0, C, p.ldc,
                               0, -1, 0, 8)
    assert ei.value.status == MISGEMM_E_SCRATCH
    packed = [c for c in mg.configs(1) if c["packed"]][0]
    with pytest.raises(mg.MisgemmError) as ei:
        mg.sgemm_split_noalloc("N", "N", p.m, p.n, p.k, 1.0, A, p.lda, B, p.ldb, 0.0, C, p.ldc,
                               1, packed["id"], 0, 1)
    assert ei.value.status == -15
    torch.cuda.synchronize()
    assert torch.equal(C.view(torch.int32), before.view(torch.int32))


def test_noalloc_graph_capture_and_replay():
    import torch
    import paper_1608_05265_amd as mg
    p = wl.make_problem("N", "T", 96, 200, 4096, 1.0, 1.0, 7400)
    A, B, C = gu.dev_problem(p)
    ref = torch.from_numpy(p.C0.copy()).to(C.device)
    torch.cuda.synchronize()
    mg.sgemm_split_noalloc("N", "T", p.m, p.n, p.k, 1.0, A, p.lda, B, p.ldb, 1.0, ref, p.ldc,
                           0, -1, 0, 8)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        mg.sgemm_split_noalloc("N", "T", p.m, p.n, p.k, 1.0, A, p.lda, B, p.ldb, 1.0, C, p.ldc,
                               0, -1, 0, 8, stream=s)
    want = ref.cpu().numpy().view(np.uint32)
    for _ in range(3):
        C.copy_(torch.from_numpy(p.C0.copy()).to(C.device))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(C.cpu().numpy().view(np.uint32), want)
