"""Autotuner: pick the kernel configuration and tile order per problem shape.

    python -m paper_1608_05265_amd.autotune --out paper_1608_05265_amd/tuning_mi355x.txt

For every tuning key (mode, transposes, m, n, k) every compiled
configuration of that mode is timed through the C-ABI
(misgemm_sgemm_config, HIP events on the launching stream, median of
several repetitions after warm-up) -- configurations with a split-K variant
also with several split factors (misgemm_sgemm_split) when their tiles
alone leave CUs idle -- then the best one is timed again over a few tile
orders (group_m); the winner goes into the tuning table that the
library reads (include/misgemm.h, misgemm_load_tuning).  Batched plans are
tuned the same way over the configurations with a persistent variant, on
the batch workload, and also as two concurrent parts (problems with m and
n at or above a threshold on a large-tile configuration, the others on a
small-tile one) when that is faster.  The paper fixes its block sizes at compile time; here
the search replaces that choice, per shape.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

GROUP_MS = [1, 4, 8, 16]
SPLITS = [2, 4, 8, 16]


def _time(fn, reps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    times = []
    for _ in range(reps):
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record(stream)
        fn()
        e.record(stream)
        times.append((s, e))
    torch.cuda.synchronize()
    return statistics.median(s.elapsed_time(e) for s, e in times)


def default_keys():
    """Shapes of the workloads (square sweep, rank-k updates, the 256^3 case)
    plus a grid of sizes between them, every transpose pair."""
    keys = []
    pairs = [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")]
    for mode in (0, 1):
        for ta, tb in pairs:
            for s in (256, 384, 512, 1024, 2048, 4096, 8192):
                keys.append((mode, ta, tb, s, s, s))
        for k in (128, 256, 512):
            keys.append((mode, "N", "N", 16384, 16384, k))
        # skinny outputs with long K (the split-K regime)
        for (m, n, k) in ((128, 512, 8192), (512, 512, 16384)):
            keys.append((mode, "N", "N", m, n, k))
    return keys


# Leading dimensions of the timed operands: the stored rows plus LD_PAD (the
# benchmark sweep's layout), so that a power-of-two ld's cache-set and
# memory-channel aliasing, which few callers have, does not decide the choice.
LD_PAD = 16


def tune_gemm(keys, reps=5, warmup=2, log=print):
    import torch
    import paper_1608_05265_amd as mg
    dev = torch.device("cuda:0")
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    results = []

    def call(mode, ta, tb, m, n, k, A, lda, B, ldb, C, cid, gm, sp):
        ldc = m + LD_PAD
        if sp == 1:
            mg.sgemm_config(ta, tb, m, n, k, 1.0, A, lda, B, ldb, 0.5, C, ldc, mode, cid, gm)
        else:
            mg.sgemm_split(ta, tb, m, n, k, 1.0, A, lda, B, ldb, 0.5, C, ldc, mode, cid, gm, sp)

    for (mode, ta, tb, m, n, k) in keys:
        ar, ac = (k, m) if ta == "T" else (m, k)
        br, bc = (n, k) if tb == "T" else (k, n)
        ar, br = ar + LD_PAD, br + LD_PAD  # leading dimensions
        A = torch.rand(ar * ac, device=dev) * 2 - 1
        B = torch.rand(br * bc, device=dev) * 2 - 1
        C = torch.rand((m + LD_PAD) * n, device=dev)
        flops = 2.0 * m * n * k
        small = flops < 2e10
        r, w = (reps * 4, warmup * 2) if small else (reps, warmup)
        timings = {}
        ids = {}
        for cfg in mg.configs(mode):
            ids[cfg["name"]] = cfg["id"]
            tiles = -(-m // cfg["bm"]) * -(-n // cfg["bn"])
            splits = [1] + (SPLITS if cfg["splitk"] and tiles < 2 * cus else [])
            for sp in splits:
                def fn(cid=cfg["id"], sp=sp):
                    call(mode, ta, tb, m, n, k, A, ar, B, br, C, cid, 0, sp)
                timings[(cfg["name"], sp)] = _time(fn, r, w)
        packed = {c["name"] for c in mg.configs(mode) if c["packed"]}
        # the fastest entry, and, when that one is packed (it needs a workspace,
        # which only misgemm_sgemm_ws is given), also the fastest non-packed one
        picks = [min(timings, key=timings.get)]
        if picks[0][0] in packed:
            picks.append(min((key for key in timings if key[0] not in packed),
                             key=timings.get))
        for best, best_sp in picks:
            orders = {}
            for gm in GROUP_MS:
                def fn(gm=gm, best=best, best_sp=best_sp):
                    call(mode, ta, tb, m, n, k, A, ar, B, br, C, ids[best], gm, best_sp)
                orders[gm] = _time(fn, r, w)
            best_gm = min(orders, key=orders.get)
            row = {"mode": mode, "ta": ta, "tb": tb, "m": m, "n": n, "k": k, "config": best,
                   "group_m": best_gm, "splits": best_sp, "ms": orders[best_gm],
                   "tflops": flops / (orders[best_gm] * 1e-3) / 1e12,
                   "all_ms": {"%s/s%d" % key: v for key, v in timings.items()},
                   "group_m_ms": orders}
            log("mode %d %s%s %6d %6d %6d -> %-26s gm=%-2d splits=%-2d %8.3f ms %7.1f TF/s"
                % (mode, ta, tb, m, n, k, best, best_gm, best_sp, row["ms"], row["tflops"]))
            results.append(row)
        del A, B, C
        torch.cuda.empty_cache()
    return results


def tune_batch(problems, reps=5, warmup=2, log=print):
    import torch
    import paper_1608_05265_amd as mg
    dev = torch.device("cuda:0")
    tensors = []
    descs = []
    for p in problems:
        A = torch.from_numpy(p.A).to(dev)
        B = torch.from_numpy(p.B).to(dev)
        C = torch.from_numpy(p.C0).to(dev)
        tensors.append((A, B, C))
        descs.append((p.transa, p.transb, p.m, p.n, p.k, p.alpha, A, p.lda, B, p.ldb, p.beta, C,
                      p.ldc))
    flops = sum(p.flops() for p in problems)
    out = {}
    for mode in (0, 1):
        timings = {}
        for cfg in mg.configs(mode):
            try:
                plan = mg.Batch(descs, mode=mode, config_id=cfg["id"])
            except mg.MisgemmError:
                continue  # no persistent variant
            timings[cfg["name"]] = _time(plan.launch, reps, warmup)
            plan.destroy()
        best = min(timings, key=timings.get)
        out[mode] = {"config": best, "ms": timings[best],
                     "tflops": flops / (timings[best] * 1e-3) / 1e12, "all_ms": timings}
        log("batch mode %d -> %s %.3f ms %.1f TF/s" % (mode, best, timings[best],
                                                       out[mode]["tflops"]))
        # two-part rules: problems with m, n >= T on a large-tile config,
        # the rest on a small-tile one, launched concurrently (fork/join on a
        # second stream, as the library launches a two-part plan)
        rules = {}
        side = torch.cuda.Stream()
        main = torch.cuda.current_stream()
        bigs = [c for c in mg.configs(mode) if c["bm"] >= 128 and c["bn"] >= 128]
        smalls = [c for c in mg.configs(mode) if c["bm"] <= 64 and c["bn"] <= 64]
        for thr in (192, 256, 384):
            ib = [i for i, p in enumerate(problems) if p.m >= thr and p.n >= thr]
            isml = [i for i, p in enumerate(problems) if not (p.m >= thr and p.n >= thr)]
            if not ib or not isml:
                continue
            for cb in bigs:
                for cs in smalls:
                    try:
                        pb = mg.Batch([descs[i] for i in ib], mode=mode, config_id=cb["id"])
                        ps = mg.Batch([descs[i] for i in isml], mode=mode, config_id=cs["id"])
                    except mg.MisgemmError:
                        continue

                    def launch(pb=pb, ps=ps):
                        fork = torch.cuda.Event()
                        fork.record(main)
                        side.wait_event(fork)
                        pb.launch(main)
                        ps.launch(side)
                        join = torch.cuda.Event()
                        join.record(side)
                        main.wait_event(join)
                    rules[(thr, cb["name"], cs["name"])] = _time(launch, reps, warmup)
                    pb.destroy()
                    ps.destroy()
        if rules:
            key = min(rules, key=rules.get)
            log("batch mode %d: best two-part option m,n >= %d on %s, others on %s: %.3f ms "
                "(one part: %.3f ms)" % (mode, key[0], key[1], key[2], rules[key],
                                         timings[best]))
            if rules[key] < 0.99 * timings[best]:
                out[mode]["rule"] = {"threshold": key[0], "big": key[1], "small": key[2],
                                     "ms": rules[key],
                                     "tflops": flops / (rules[key] * 1e-3) / 1e12}
                log("batch mode %d -> two parts: m,n >= %d on %s, others on %s: %.3f ms "
                    "%.1f TF/s" % (mode, key[0], key[1], key[2], rules[key],
                                   out[mode]["rule"]["tflops"]))
    return out


def write_table(path, gemm_rows, batch):
    with open(path, "w") as f:
        f.write("misgemm-tuning 1\n")
        f.write("# written by paper_1608_05265_amd.autotune on %s\n" % time.strftime("%Y-%m-%d"))
        f.write("# mode transa transb m n k config group_m splits   (best TFLOP/s)\n")
        for r in gemm_rows:
            f.write("%d %s %s %d %d %d %s %d %d\n" % (r["mode"], r["ta"], r["tb"], r["m"], r["n"],
                                                      r["k"], r["config"], r["group_m"],
                                                      r.get("splits", 1)))
            f.write("#   %.1f TFLOP/s\n" % r["tflops"])
        write_batch_lines(f, batch)


def write_batch_lines(f, batch):
    for mode, b in sorted(batch.items()):
        f.write("batch %d %s\n" % (mode, b["config"]))
        f.write("#   %.1f TFLOP/s on a 512-problem batch of the benchmark's distribution "
                "(other seeds)\n" % b["tflops"])
        if "rule" in b:
            r = b["rule"]
            f.write("batch2 %d %d %s %s\n" % (mode, r["threshold"], r["big"], r["small"]))
            f.write("#   %.1f TFLOP/s on that batch, two concurrent parts\n" % r["tflops"])


def merge_table(base_path, out_path, gemm_rows, batch=None):
    """Write base_path to out_path with the entries (and their comment
    lines) of every key in gemm_rows replaced by the new rows, placed where
    the key's first old entry was (new keys go after the last entry); with
    `batch` (tune_batch's result), the batch and batch2 lines of its modes
    are replaced by the new ones, at the end."""
    new = {}
    for r in gemm_rows:
        new.setdefault((r["mode"], r["ta"], r["tb"], r["m"], r["n"], r["k"]), []).append(r)

    def fmt(r):
        return ["%d %s %s %d %d %d %s %d %d\n" % (r["mode"], r["ta"], r["tb"], r["m"], r["n"],
                                                r["k"], r["config"], r["group_m"],
                                                r.get("splits", 1)),
                "#   %.1f TFLOP/s\n" % r["tflops"]]
    out, done, skipping, last_entry = [], set(), False, 0
    with open(base_path) as f:
        lines = f.readlines()
    for line in lines:
        parts = line.split()
        if line.startswith("#") and skipping:
            continue
        skipping = False
        if batch and len(parts) >= 3 and parts[0] in ("batch", "batch2") and \
                int(parts[1]) in batch:
            skipping = True
            continue
        if len(parts) == 9 and parts[0] in ("0", "1"):
            key = (int(parts[0]), parts[1], parts[2], int(parts[3]), int(parts[4]), int(parts[5]))
            if key in new:
                skipping = True
                if key not in done:
                    done.add(key)
                    for r in new[key]:
                        out.extend(fmt(r))
                    last_entry = len(out)
                continue
            out.append(line)
            last_entry = len(out)
            continue
        out.append(line)
    rest = [ln for key, rows in new.items() if key not in done for r in rows for ln in fmt(r)]
    out[last_entry:last_entry] = rest
    with open(out_path, "w") as f:
        f.writelines(out)
        if batch:
            write_batch_lines(f, batch)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                   "tuning_mi355x.txt"))
    ap.add_argument("--json", default=None, help="also dump every timing here")
    ap.add_argument("--quick", action="store_true", help="fewer keys (smoke test of the tuner)")
    ap.add_argument("--sizes", default=None,
                    help="comma list: tune only the square keys of these sizes and merge the "
                         "rows into the table named by --merge (no batch tuning)")
    ap.add_argument("--rankk", action="store_true",
                    help="with --merge: also tune the 16384^2 x K rank-k keys")
    ap.add_argument("--batch", action="store_true",
                    help="with --merge: also retune the batch lines")
    ap.add_argument("--merge", default=None, help="table to merge --sizes rows into")
    args = ap.parse_args(argv)
    os.environ["MISGEMM_TUNING"] = "none"  # tune from the built-in defaults
    from paper_1608_05265_amd import workloads as wl
    keys = default_keys()
    if args.sizes or args.rankk or args.batch:
        if not args.merge:
            ap.error("--sizes, --rankk and --batch need --merge")
        sizes = {int(v) for v in args.sizes.split(",")} if args.sizes else set()
        keys = [k for k in keys if (k[3] == k[4] == k[5] and k[3] in sizes) or
                (args.rankk and k[3] == k[4] == 16384 and k[5] in wl.RANKK_KS)]
        rows = tune_gemm(keys, log=lambda s: print(s, flush=True)) if keys else []
        batch = None
        if args.batch:
            batch = tune_batch(wl.config5(count=512, seed_case=1),
                               log=lambda s: print(s, flush=True))
        merge_table(args.merge, args.out, rows, batch)
        print("wrote", args.out)
        return 0
    if args.quick:
        keys = [k for k in keys if k[3] <= 1024 and k[5] <= 1024][:6]
    rows = tune_gemm(keys, log=lambda s: print(s, flush=True))
    # a batch drawn like the benchmark's but from other seeds, so that the
    # batch configuration is not chosen on the very problems it is measured on
    problems = wl.config5(count=64 if args.quick else 512, seed_case=1)
    batch = tune_batch(problems, log=lambda s: print(s, flush=True))
    write_table(args.out, rows, batch)
    if args.json:
        with open(args.json, "w") as f:
            json.dump({"gemm": rows, "batch": {str(k): v for k, v in batch.items()}}, f)
    print("wrote", args.out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
