"""The batched persistent form: many independent problems in one launch,
every problem checked against the oracle, plus HIP-graph capture and replay."""
import numpy as np
import pytest

import oracle
from paper_1608_05265_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _setup(problems):
    import torch
    dev = [gu.dev_problem(p) for p in problems]
    c0 = [C.clone() for (_, _, C) in dev]
    descs = [(p.transa, p.transb, p.m, p.n, p.k, p.alpha, A, p.lda, B, p.ldb, p.beta, C, p.ldc)
             for p, (A, B, C) in zip(problems, dev)]
    torch.cuda.synchronize()
    return dev, c0, descs


def _check_all(problems, dev, full, label):
    for idx, (p, (_, _, C)) in enumerate(zip(problems, dev)):
        out = C.cpu().numpy()[:p.C0.size]
        if full:
            gu.check_full(p, out, "%s problem %d" % (label, idx))
        else:
            gu.check_sampled(p, out, count=48, seed=idx, label="%s problem %d" % (label, idx))


@pytest.mark.parametrize("mode", [0, 1], ids=["fp32", "bf16x3"])
def test_batch_small_every_batched_config(mode):
    """64 problems of mixed shapes (including ragged, tiny and k = 0 ones),
    run through every configuration that has a persistent variant."""
    import torch
    import paper_1608_05265_amd as mg
    problems = wl.config5(count=60, seed_case=7, lo=1, hi=24, step=7)
    problems.append(wl.make_problem("N", "N", 5, 3, 0, 1.0, 0.5, 11))      # k = 0
    problems.append(wl.make_problem("T", "N", 9, 7, 4, 0.0, -1.0, 12))     # alpha = 0
    problems.append(wl.make_problem("N", "T", 1, 1, 1, 2.0, 0.0, 13))      # 1x1x1
    problems.append(wl.make_problem("T", "T", 33, 65, 17, 1.0, 1.0, 14, pad=3))
    for cfg in mg.configs(mode):
        dev, c0, descs = _setup(problems)
        try:
            plan = mg.Batch(descs, mode=mode, config_id=cfg["id"])
        except mg.MisgemmError as e:
            assert e.status == 1001  # no persistent variant for this config
            continue
        plan.launch()
        torch.cuda.synchronize()
        _check_all(problems, dev, True, cfg["name"])
        plan.destroy()


@pytest.mark.parametrize("mode", [0, 1], ids=["fp32", "bf16x3"])
def test_batch512_graph_replay(mode):
    """The 512-problem batch: one eager launch checked against the oracle on
    sampled entries of every problem, then captured into a HIP graph and
    replayed several times with unrelated eager work in between; every
    replay must equal the eager result bit for bit."""
    import torch
    import paper_1608_05265_amd as mg
    problems = wl.config5()
    dev, c0, descs = _setup(problems)
    plan = mg.Batch(descs, mode=mode)
    info = plan.info()
    assert info["count"] == 512 and info["tiles"] > 0
    # one tile list per XCD, close to even work
    assert info["parts"] == 8 and info["grid"] % 8 == 0
    assert 1.0 <= info["part_imbalance"] < 1.05
    plan.launch()
    torch.cuda.synchronize()
    _check_all(problems, dev, False, "batch512 mode %d" % mode)
    eager = [C.clone() for (_, _, C) in dev]

    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for (_, _, C), c in zip(dev, c0):
            C.copy_(c)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        plan.launch()
    scratch = torch.randn(1 << 20, device="cuda")
    for rep in range(3):
        for (_, _, C), c in zip(dev, c0):
            C.copy_(c)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for idx, ((_, _, C), e) in enumerate(zip(dev, eager)):
            assert torch.equal(C.view(torch.int32), e.view(torch.int32)), (rep, idx)
        scratch.mul_(1.0001).add_(1.0)  # unrelated eager work between replays
        torch.cuda.synchronize()
    plan.destroy()


@pytest.mark.parametrize("mode", [0, 1], ids=["fp32", "bf16x3"])
def test_batch_skewed_work_is_split_over_xcds(mode):
    """One problem carrying most of the work beside small ones: it is cut
    into chunks spread over the XCD lists (not left to one XCD), and every
    problem is still computed right."""
    import torch
    import paper_1608_05265_amd as mg
    problems = [wl.make_problem("N", "T", 1536, 1280, 384, 1.0, 0.5, 21, pad=2)]
    problems += wl.config5(count=24, seed_case=8, lo=1, hi=12, step=5)
    problems.append(wl.make_problem("T", "N", 8, 8, 8, 1.0, 0.0, 22))  # fewer tiles than XCDs
    dev, c0, descs = _setup(problems)
    plan = mg.Batch(descs, mode=mode)
    info = plan.info()
    assert info["parts"] == 8
    assert info["part_imbalance"] < 1.35, info
    plan.launch()
    torch.cuda.synchronize()
    _check_all(problems, dev, False, "skewed mode %d" % mode)
    plan.destroy()

    # a batch with fewer tiles than XCDs runs from one list
    tiny = [wl.make_problem("N", "N", 16, 16, 16, 1.0, 0.0, 23 + i) for i in range(3)]
    dev, c0, descs = _setup(tiny)
    plan = mg.Batch(descs, mode=mode)
    info = plan.info()
    assert info["parts"] == 1 and info["grid"] >= 1
    plan.launch()
    torch.cuda.synchronize()
    _check_all(tiny, dev, True, "tiny mode %d" % mode)
    plan.destroy()


def test_batch_plan_errors():
    import paper_1608_05265_amd as mg
    import torch
    p = wl.make_problem("N", "N", 8, 8, 8, 1.0, 0.0, 1)
    (A, B, C) = gu.dev_problem(p)
    good = ("N", "N", 8, 8, 8, 1.0, A, 8, B, 8, 0.0, C, 8)
    bad = ("N", "N", 8, 8, 8, 1.0, A, 4, B, 8, 0.0, C, 8)  # lda < m
    with pytest.raises(mg.MisgemmError) as ei:
        mg.Batch([good, good, bad], mode=0)
    assert ei.value.status == -8 and ei.value.bad_index == 2
    with pytest.raises(mg.MisgemmError) as ei:
        mg.Batch([good], mode=0, config_id=0)  # 256x256 has no persistent variant
    assert ei.value.status == 1001
    torch.cuda.synchronize()


@pytest.mark.parametrize("mode", [0, 1], ids=["fp32", "bf16x3"])
def test_batch_two_part_rule(mode, tmp_path):
    """A tuning-table rule "batch2 <mode> 256 <large-tile> <small-tile>": the
    default plan puts the problems with m, n >= 256 on the large-tile
    configuration and the rest on the small-tile one, launched concurrently
    (fork/join on the plan's own stream).  Results are checked against the
    oracle on sampled entries, equal bit for bit two explicit single-config
    plans of the same split, and every HIP-graph replay of the launch equals
    the eager result.  The packaged table is restored afterwards."""
    import torch
    import paper_1608_05265_amd as mg
    big_cfg, small_cfg = (("fp32p_128x128x16_w64x64", "fp32_64x64x16_w32x32") if mode == 0
                          else ("x3p_128x128x16_w64x64", "x3_64x64x32_w32x32"))
    names = {c["name"]: c["id"] for c in mg.configs()}
    table = tmp_path / "tuning.txt"
    table.write_text("misgemm-tuning 1\nbatch %d %s\nbatch2 %d 256 %s %s\n"
                     % (mode, small_cfg, mode, big_cfg, small_cfg))
    problems = wl.config5(count=96, seed_case=3)
    big = [i for i, p in enumerate(problems) if p.m >= 256 and p.n >= 256]
    assert 0 < len(big) < len(problems)
    try:
        mg.load_tuning(str(table))
        dev, c0, descs = _setup(problems)
        plan = mg.Batch(descs, mode=mode)
        info = plan.info()
        assert info["config_id"] == names[big_cfg] and info["second_config_id"] == names[small_cfg]
        assert info["count"] == len(problems)
        plan.launch()
        torch.cuda.synchronize()
        _check_all(problems, dev, False, "two-part mode %d" % mode)
        eager = [C.clone() for (_, _, C) in dev]
        # the same split as two explicit single-config plans
        for (_, _, C), c in zip(dev, c0):
            C.copy_(c)
        small = [i for i in range(len(problems)) if i not in set(big)]
        pb = mg.Batch([descs[i] for i in big], mode=mode, config_id=names[big_cfg])
        ps = mg.Batch([descs[i] for i in small], mode=mode, config_id=names[small_cfg])
        pb.launch()
        ps.launch()
        torch.cuda.synchronize()
        for idx, ((_, _, C), e) in enumerate(zip(dev, eager)):
            assert torch.equal(C.view(torch.int32), e.view(torch.int32)), idx
        pb.destroy()
        ps.destroy()
        # captured and replayed
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            plan.launch()
        for rep in range(3):
            for (_, _, C), c in zip(dev, c0):
                C.copy_(c)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            for idx, ((_, _, C), e) in enumerate(zip(dev, eager)):
                assert torch.equal(C.view(torch.int32), e.view(torch.int32)), (rep, idx)
        del g
        plan.destroy()
    finally:
        mg.load_tuning(mg.TUNING_PATH)


def test_packed_batch_matches_single_packed_calls_and_replays():
    """A packed split-form plan (operands split once into plan-owned panels,
    then the persistent tile kernel on them) gives the same bits as the
    same packed configuration called problem by problem, and its graph
    replays (pack launch + tile launch) repeat them after the operands
    change and change back."""
    import torch
    import paper_1608_05265_amd as mg
    problems = wl.config5(count=40, seed_case=8, lo=1, hi=20, step=11)
    problems.append(wl.make_problem("T", "T", 77, 130, 45, 1.5, -0.5, 15, pad=2))
    for cfg in [c for c in mg.configs(1) if c["packed"]]:
        dev, c0, descs = _setup(problems)
        try:
            plan = mg.Batch(descs, mode=1, config_id=cfg["id"])
        except mg.MisgemmError as e:
            assert e.status == 1001  # no persistent variant
            continue
        info = plan.info()
        assert info["panel_bytes"] > 0
        plan.launch()
        torch.cuda.synchronize()
        got = [C.clone() for (_, _, C) in dev]
        _check_all(problems, dev, True, cfg["name"])
        for p, (A, B, C), c, ref in zip(problems, dev, c0, got):
            C.copy_(c)
            mg.sgemm_config(p.transa, p.transb, p.m, p.n, p.k, p.alpha, A, p.lda, B, p.ldb,
                            p.beta, C, p.ldc, 1, cfg["id"])
            torch.cuda.synchronize()
            assert torch.equal(C.view(torch.int32), ref.view(torch.int32)), (cfg["name"], p.label)
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(g, stream=side):
            plan.launch(side)
        A0 = dev[0][0]
        saved = A0.clone()
        for rep in range(3):
            for (_, _, C), c in zip(dev, c0):
                C.copy_(c)
            A0.mul_(2.0 if rep == 1 else 1.0)   # the pack reads the operands at replay
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            for i, ((_, _, C), ref) in enumerate(zip(dev, got)):
                if rep == 1 and i == 0:
                    assert not torch.equal(C.view(torch.int32), ref.view(torch.int32))
                else:
                    assert torch.equal(C.view(torch.int32), ref.view(torch.int32)), (rep, i)
            A0.copy_(saved)
        del g
        plan.destroy()
