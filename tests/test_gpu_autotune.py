"""The autotuner end to end on a few small keys: it times every compiled
configuration (and split factors and tile orders) through the C-ABI,
writes a tuning table, and the library then dispatches by that table --
the chosen configuration is the one selected, results through it match the
oracle, and a batch plan picks the tuned batch configuration (or the
tuned two-part rule).  The packaged
table is restored afterwards."""
import pytest

from paper_1608_05265_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

KEYS = [(0, "N", "T", 300, 200, 500), (1, "T", "N", 256, 192, 320), (0, "N", "N", 96, 64, 4096)]


def test_autotune_table_drives_dispatch(tmp_path):
    import paper_1608_05265_amd as mg
    from paper_1608_05265_amd import autotune
    try:
        mg.load_tuning(None)  # tune from the built-in defaults
        rows = autotune.tune_gemm(KEYS, reps=2, warmup=1, log=lambda s: None)
        batch = autotune.tune_batch(wl.config5(count=8), reps=2, warmup=1, log=lambda s: None)
        path = tmp_path / "tuning.txt"
        autotune.write_table(str(path), rows, batch)
        mg.load_tuning(str(path))
        names = {c["name"]: c["id"] for c in mg.configs()}
        packed = {c["name"] for c in mg.configs() if c["packed"]}
        for mode, ta, tb, m, n, k in KEYS:
            mine = [r for r in rows if (r["mode"], r["ta"], r["tb"], r["m"], r["n"], r["k"]) ==
                    (mode, ta, tb, m, n, k)]
            assert mine and all(r["config"] in names and r["tflops"] > 0 for r in mine)
            # the fastest first; a packed winner is followed by the fastest
            # non-packed entry, which is what misgemm_sgemm dispatches to
            assert len(mine) == (2 if mine[0]["config"] in packed else 1)
            row = [r for r in mine if r["config"] not in packed][0]
            assert mg.select_config(ta, tb, m, n, k, mode) == names[row["config"]], row
            p = wl.make_problem(ta, tb, m, n, k, 1.25, -0.5, 9700 + m, pad=2)
            gu.check_full(p, gu.run(p, mode), "tuned %s%s %dx%dx%d mode %d" % (ta, tb, m, n, k,
                                                                                mode))
        probs = wl.config5(count=8)
        tensors = [gu.dev_problem(p) for p in probs]
        for mode in (0, 1):
            plan = mg.Batch([(p.transa, p.transb, p.m, p.n, p.k, p.alpha, A, p.lda, B, p.ldb,
                              p.beta, C, p.ldc) for p, (A, B, C) in zip(probs, tensors)], mode)
            info = plan.info()
            rule = batch[mode].get("rule")
            if rule is None:
                assert info["config_id"] == names[batch[mode]["config"]]
                assert info["second_config_id"] == -1
            else:
                big = [p for p in probs if p.m >= rule["threshold"] and p.n >= rule["threshold"]]
                if big and len(big) < len(probs):
                    assert info["config_id"] == names[rule["big"]]
                    assert info["second_config_id"] == names[rule["small"]]
                else:
                    assert info["config_id"] == names[rule["big"] if big else rule["small"]]
            plan.destroy()
    finally:
        mg.load_tuning(mg.TUNING_PATH)
