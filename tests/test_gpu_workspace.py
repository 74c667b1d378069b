"""Ownership of the library scratch of misgemm_sgemm (packed bf16x3 panels,
split-K partial tiles): a caller that never captures holds one buffer per
stream, sized for its largest problem; buffers a captured graph may use are
kept until misgemm_release_workspace; an explicitly requested packed
configuration under capture without scratch is an error, not a silent
change of configuration."""
import numpy as np
import pytest

from paper_1608_05265_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _packed_id(mg):
    return [c for c in mg.configs(1) if c["packed"]][0]["id"]


def _run_packed(mg, torch, size, cfg, seed, stream=None):
    p = wl.make_problem("T", "N", size, size, size, 1.0, 0.0, seed)
    A, B, C = gu.dev_problem(p)
    torch.cuda.synchronize()
    mg.sgemm_config("T", "N", size, size, size, 1.0, A, p.lda, B, p.ldb, 0.0, C, p.ldc, 1, cfg,
                    stream=stream)
    torch.cuda.synchronize()
    return p, (A, B, C), mg.workspace_size("T", "N", size, size, size, 1)


def test_growth_without_capture_holds_one_buffer():
    import torch
    import paper_1608_05265_amd as mg
    mg.release_workspace()
    assert mg.workspace_held() == 0
    cfg = _packed_id(mg)
    largest = 0
    for size, seed in ((256, 1), (512, 2), (1024, 3), (300, 4)):
        p, tensors, need = _run_packed(mg, torch, size, cfg, seed)
        gu.check_full(p, tensors[2].cpu().numpy(), "packed %d" % size)
        largest = max(largest, need)
        held = mg.workspace_held()
        # one buffer: at least this problem's need, at most 1.5 x the largest
        # need so far (outgrown buffers were freed, not kept)
        assert need <= held <= int(1.5 * largest), (size, held, need, largest)
    mg.release_workspace()
    assert mg.workspace_held() == 0


def test_capture_keeps_buffers_graphs_use():
    import torch
    import paper_1608_05265_amd as mg
    mg.release_workspace()
    cfg = _packed_id(mg)
    s = torch.cuda.Stream()
    p, (A, B, C), need_small = _run_packed(mg, torch, 512, cfg, 5, stream=s)
    held_small = mg.workspace_held()
    assert held_small >= need_small
    ref = C.cpu().numpy().copy()
    g = torch.cuda.CUDAGraph()
    C.zero_()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        mg.sgemm_config("T", "N", 512, 512, 512, 1.0, A, p.lda, B, p.ldb, 0.0, C, p.ldc, 1, cfg,
                        stream=s)
    # a larger problem on the same stream grows its scratch; the buffer the
    # graph captured is kept for the graph
    _, _, need_big = _run_packed(mg, torch, 1024, cfg, 6, stream=s)
    assert mg.workspace_held() >= held_small + need_big
    for _ in range(3):
        C.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(C.cpu().numpy().view(np.uint32), ref.view(np.uint32))
    del g
    mg.release_workspace()
    assert mg.workspace_held() == 0


def test_explicit_packed_config_under_capture_without_scratch_is_an_error():
    import torch
    import paper_1608_05265_amd as mg
    mg.release_workspace()
    cfg = _packed_id(mg)
    p = wl.make_problem("T", "N", 384, 384, 384, 1.0, 0.0, 7)
    A, B, C = gu.dev_problem(p)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(mg.MisgemmError) as ei:
        with torch.cuda.graph(g, stream=s):
            mg.sgemm_config("T", "N", 384, 384, 384, 1.0, A, p.lda, B, p.ldb, 0.0, C, p.ldc, 1,
                            cfg, stream=s)
    assert ei.value.status == 1002
    torch.cuda.synchronize()
    assert mg.workspace_held() == 0
