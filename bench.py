#!/usr/bin/env python3
"""Benchmark of the sgemm hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload square|c1|rankk|wide|skinny|batch|...]

One step is one pass of the workload's GEMMs over seeded synthetic inputs
that are already resident in HBM.  The default workload is the square sweep
M = N = K in {1024, 2048, 4096, 8192} over the four transpose pairs
(alpha = 1.5, beta = -0.5, every leading dimension padded by 16): sixteen
sgemm calls per step, run first in native FP32-MFMA form (the line's
`value`) and then in bf16x3 form (the `bf16x3` object).  TFLOP/s counts
2*M*N*K per call.

Printed: one JSON line with the metric, the roofline of the dominant kernel
(timed with HIP events on the stream it runs on), and the CPU oracle timed on
a bounded sample of the same inputs, which also measures the error of the
GPU results on that sample against the acceptance bound.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SGEMM TFLOP/s and % of MFMA peak, native FP32 vs bf16x3 at stated error"
PEAK_FP32 = 157.3      # TFLOP/s, MI355X dense FP32 matrix (= FP32 vector)
PEAK_BF16 = 2516.6     # TFLOP/s, MI355X dense BF16 matrix
PEAK_HBM = 8000.0      # GB/s
PEAK_FP64 = 78.6       # TFLOP/s, MI355X dense FP64 matrix
# equal measured error: the split form's max and mean normalized error at
# most this factor above the native form's on the same inputs
EQUAL_ERROR_RATIO = 1.5


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="square",
                    choices=["square", "c1", "rankk", "wide", "skinny", "batch", "dominant", "peak",
                             "dgemm", "host", "lu"],
                    help="dominant: only the 8192^3 NN problem of the square sweep in both "
                         "forms plus a 1 GiB device copy, for counter collection")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (used under the profiler)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-form measurement in the default run")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the wide-range, rank-k, copy-bandwidth and 256^3 objects of the "
                         "default run")
    ap.add_argument("--no-clock", action="store_true",
                    help="skip the clock/power sampling runs (used under the profiler)")
    ap.add_argument("--no-peak", action="store_true",
                    help="skip the matrix-core rate probe in the default run")
    ap.add_argument("--problem", default="",
                    help="comma-separated problem labels: run only these problems of the "
                         "workload (e.g. rankk128_16384x16384), for per-problem profiles")
    return ap.parse_args()


def make_problems(workload, only=""):
    probs, desc = _workload_problems(workload)
    if only:
        keep = set(only.split(","))
        probs = [p for p in probs if p.label in keep]
        if not probs:
            raise SystemExit("no problem of workload %s is labelled %s" % (workload, only))
        desc += " (only %s)" % only
    return probs, desc


def _workload_problems(workload):
    from paper_1608_05265_amd import workloads as wl
    if workload == "square":
        return [wl.config2(s, ta, tb) for s in wl.SQUARE_SIZES for ta, tb in wl.TRANS_PAIRS], \
            "square sweep M=N=K in {1024,2048,4096,8192} x {NN,NT,TN,TT}, alpha=1.5, " \
            "beta=-0.5, ld=rows+16, uniform[-1,1]"
    if workload == "c1":
        return [wl.config1()], "single sgemm 256^3 NN, alpha=1, beta=0, uniform[-1,1]"
    if workload == "rankk":
        return [wl.config3(k) for k in wl.RANKK_KS], \
            "rank-k update M=N=16384, K in {128,256,512}, NN, alpha=-1, beta=1, normal(0,1)"
    if workload == "wide":
        return [wl.config4()], "8192^3 NN, alpha=1, beta=0, entries random sign x 2^U[-8,8]"
    if workload == "skinny":
        return [wl.config7(*s) for s in wl.SKINNY_SHAPES], \
            "split-K regime (few output tiles, long K): 512^3, 128x512x8192, " \
            "512x512x16384, NN, alpha=1.5, beta=-0.5, uniform[-1,1]"
    raise ValueError(workload)


class ClockSampler:
    """Samples the GPU's graphics clock (MHz, mean over the XCDs) and socket
    power (W) from the SMU metrics table through amdsmi on a host thread
    every `period` seconds, and the share of the interval spent at the
    package power limit (PPT residency).  Fields stay None where amdsmi is
    missing or refuses."""

    def __init__(self, period=0.05, skip=0.5):
        self.period = period
        self.skip = skip
        self.clk = []
        self.power = []
        self.first = None
        self.last = None
        self.error = None
        self._stop = None
        self._thread = None
        self._h = None
        self._amdsmi = None

    @staticmethod
    def _num(v):
        return float(v) if isinstance(v, (int, float)) and 0 < v < 1e15 else None

    def _read(self, keep):
        try:
            m = self._amdsmi.amdsmi_get_gpu_metrics_info(self._h)
        except Exception as e:  # noqa: BLE001 - report, do not fail the bench
            self.error = "metrics: %s" % type(e).__name__
            return
        clks = [self._num(c) for c in (m.get("current_gfxclks") or [])]
        clks = [c for c in clks if c is not None and c < 10000]
        pw = self._num(m.get("current_socket_power"))
        acc = (self._num(m.get("accumulation_counter")), self._num(m.get("ppt_residency_acc")))
        if keep:
            if clks:
                self.clk.append(sum(clks) / len(clks))
            if pw is not None:
                self.power.append(pw)
            if self.first is None:
                self.first = acc
            self.last = acc

    def _loop(self):
        import time as _t
        t0 = _t.perf_counter()
        while not self._stop.wait(self.period):
            self._read(_t.perf_counter() - t0 >= self.skip)

    def __enter__(self):
        import threading
        try:
            import amdsmi
            amdsmi.amdsmi_init()
            self._h = amdsmi.amdsmi_get_processor_handles()[0]
            self._amdsmi = amdsmi
        except Exception as e:  # noqa: BLE001
            self.error = "amdsmi unavailable: %s" % type(e).__name__
            return self
        self._stop = threading.Event()
        self._thread = threading.Thread(target=self._loop, daemon=True)
        self._thread.start()
        return self

    def __exit__(self, *exc):
        if self._thread is not None:
            self._stop.set()
            self._thread.join()
            try:
                self._amdsmi.amdsmi_shut_down()
            except Exception:  # noqa: BLE001
                pass
        return False

    def summary(self):
        def stats(v):
            if not v:
                return None
            v = sorted(v)
            return {"median": round(v[len(v) // 2], 1), "min": round(v[0], 1),
                    "max": round(v[-1], 1), "samples": len(v)}
        out = {"sclk_mhz": stats(self.clk), "socket_power_w": stats(self.power),
               "ppt_residency": None}
        if self.first and self.last and None not in self.first + self.last:
            d_acc = self.last[0] - self.first[0]
            if d_acc > 0:
                out["ppt_residency"] = round((self.last[1] - self.first[1]) / d_acc, 3)
        if self.error:
            out["note"] = self.error
        return out


def clock_probe(torch, fn, seconds=2.5):
    """Run `fn` (which enqueues GPU work) back to back for about `seconds`
    while sampling clock and power; the first half second is not sampled so
    that the readings describe the loaded steady state."""
    with ClockSampler() as clock:
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < seconds:
            fn()
            n += 1
            if n % 4 == 0:
                torch.cuda.synchronize()
        torch.cuda.synchronize()
    return clock.summary()


PROBE_FLOP = {0: 32 * 32 * 2 * 2, 1: 32 * 32 * 16 * 2, 2: 16 * 16 * 4 * 2}
# per MFMA: 32x32x2 f32, 32x32x16 bf16, 16x16x4 f64


PROBE_KINDS = {"fp32": (0, "float32", 8000), "bf16": (1, "bfloat16", 16000),
               "fp64": (2, "float64", 4000)}


def measure_peaks(torch, seconds=2.5, kinds=("fp32", "bf16"), datas=("random", "zero")):
    """Sustained matrix-core rate of this GPU (the probe library: four
    independent accumulators per wave, two waves per SIMD, back-to-back
    MFMAs), with random and with zero operands, each after `seconds` of
    back-to-back launches so that clock and power have settled; the clock,
    power and PPT residency of that interval come with each rate."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1608_05265_amd", "libmisgemm_probe.so"))
    lib.probe_mfma_launch.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    lib.probe_mfma_launch.restype = ctypes.c_int
    dev = torch.device("cuda:0")
    blocks = torch.cuda.get_device_properties(0).multi_processor_count * 2
    out = torch.empty(blocks * 256, device=dev)
    gen = torch.Generator().manual_seed(1608)
    stream = torch.cuda.current_stream()
    res = {}
    for name in kinds:
        kind, dtname, iters = PROBE_KINDS[name]
        dt = getattr(torch, dtname)
        for data in datas:
            ops = ((torch.rand(4096, generator=gen, dtype=torch.float64) * 2 - 1).to(dt)
                   if data == "random" else torch.zeros(4096, dtype=dt)).to(dev)

            def launch():
                rc = lib.probe_mfma_launch(kind, ops.data_ptr(), out.data_ptr(), iters, blocks,
                                           stream.cuda_stream)
                if rc != 0:
                    raise RuntimeError("probe launch failed: %d" % rc)
            launch()
            torch.cuda.synchronize()
            clock = clock_probe(torch, launch, seconds=seconds)
            evs = []
            for _ in range(15):
                s_ = torch.cuda.Event(enable_timing=True)
                e_ = torch.cuda.Event(enable_timing=True)
                s_.record(stream)
                launch()
                e_.record(stream)
                evs.append((s_, e_))
            torch.cuda.synchronize()
            ms = sorted(a.elapsed_time(b) for a, b in evs)[7]
            flops = blocks * 4 * iters * 4 * PROBE_FLOP[kind]
            res["%s_%s" % (name, data)] = {"tflops": round(flops / (ms * 1e-3) / 1e12, 1),
                                           "clock": clock}
    return res


class Resident:
    """A problem's operands on the device, C restorable to C0.  FP32 calls go
    through misgemm_sgemm; split-form calls through misgemm_sgemm_ws with a
    workspace this program owns (allocated before any timing, shared by the
    problems, which run one after another on one stream), so that the
    tuning table's packed configurations can serve them -- unless `ws` is
    False: then through misgemm_sgemm too, for shapes whose tuned entry is a
    split-K configuration (misgemm_sgemm_ws never splits K; misgemm_sgemm
    keeps the partial tiles in the library's scratch)."""

    workspace = None

    def __init__(self, p, dev, ws=True):
        import torch
        import paper_1608_05265_amd as mg
        self.p = p
        self.ws = ws
        self.A = torch.from_numpy(p.A).to(dev)
        self.B = torch.from_numpy(p.B).to(dev)
        self.C0 = torch.from_numpy(p.C0).to(dev)
        self.C = self.C0.clone()
        need = mg.workspace_size(p.transa, p.transb, p.m, p.n, p.k, mg.BF16X3)
        ws = Resident.workspace
        if ws is None or ws.numel() * 4 < need:
            Resident.workspace = None
            torch.cuda.empty_cache()
            Resident.workspace = torch.empty((need + 3) // 4, dtype=torch.float32, device=dev)

    def call(self, mg, mode):
        p = self.p
        if mode == mg.BF16X3 and self.ws:
            ws = Resident.workspace
            mg.sgemm_ws(p.transa, p.transb, p.m, p.n, p.k, p.alpha, self.A, p.lda, self.B,
                        p.ldb, p.beta, self.C, p.ldc, mode, ws, ws.numel() * 4)
        else:
            mg.sgemm(p.transa, p.transb, p.m, p.n, p.k, p.alpha, self.A, p.lda, self.B, p.ldb,
                     p.beta, self.C, p.ldc, mode=mode)

    def reset(self):
        self.C.copy_(self.C0)


def time_steps(torch, res, mg, mode, steps, warmup, dominant):
    """Run warmup passes, then about 0.3 s more of them to bring the GPU to
    its working clock (when warmup > 0), then `steps` timed passes; returns
    (total seconds, dominant-kernel launch durations in ms).  The dominant
    kernel is timed with events on the stream the library launches on
    (torch's current stream), on every step, or every 8th when the workload
    is a single problem."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        for r in res:
            r.call(mg, mode)
    torch.cuda.synchronize()
    if warmup > 0:
        warm(torch, lambda: [r.call(mg, mode) for r in res], seconds=0.3)
    ev = []
    # a one-problem workload (the 256^3 case) would time the event records
    # along with each microsecond-scale call: sample every 8th step there
    every = 1 if len(res) > 1 else 8
    t0 = time.perf_counter()
    for step in range(steps):
        for i, r in enumerate(res):
            if i in dominant and step % every == 0:
                s = torch.cuda.Event(enable_timing=True)
                e = torch.cuda.Event(enable_timing=True)
                s.record(stream)
                r.call(mg, mode)
                e.record(stream)
                ev.append((s, e))
            else:
                r.call(mg, mode)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    durs = [s.elapsed_time(e) for s, e in ev]
    return total, durs


def latency(torch, r, mg, mode, calls=1000):
    """Per-call latency of one small problem: `calls` calls each bracketed
    by events on the launching stream (median and minimum of the event
    times), then `calls` calls back to back (host wall time per call)."""
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(calls)]
    for s, e in evs:
        s.record(stream)
        r.call(mg, mode)
        e.record(stream)
    torch.cuda.synchronize()
    d = sorted(s.elapsed_time(e) * 1e3 for s, e in evs)
    t0 = time.perf_counter()
    for _ in range(calls):
        r.call(mg, mode)
    torch.cuda.synchronize()
    b2b = (time.perf_counter() - t0) / calls * 1e6
    return {"median_us": round(d[calls // 2], 3), "min_us": round(d[0], 3),
            "back_to_back_us": round(b2b, 3), "calls": calls}


def cpu_model():
    """The host CPU's model name (as lscpu prints it), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline_leg(res, mg, torch, workload):
    """The FP64 oracle timed on a bounded sample of the same inputs, on the
    host's cores; the same sample gives the error of the GPU results."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    out = {"kind": "oracle", "cores": cores, "unit": "TFLOP/s", "cpu_model": cpu_model()}
    # the full oracle on every problem of the largest size it finishes in
    # about 10-30 s of CPU work (the four 4096^3 problems of the sweep)
    sizes = sorted(set(r.p.m * r.p.n * r.p.k for r in res))
    fit = [s_ for s_ in sizes if s_ <= 4096 ** 3]
    pick_size = fit[-1] if fit else sizes[0]
    picks = [r for r in res if r.p.m * r.p.n * r.p.k == pick_size]
    errors = {}
    total_dt = 0.0
    total_flops = 0.0
    for pick in picks:
        p = pick.p
        for mode, name in ((mg.FP32, "fp32"), (mg.BF16X3, "bf16x3")):
            pick.reset()
            pick.call(mg, mode)
            torch.cuda.synchronize()
            gpu = pick.C.cpu().numpy()
            if name == "fp32":
                t0 = time.perf_counter()
                cref, den = oracle.sgemm_f64(p.transa, p.transb, p.m, p.n, p.k, p.alpha, p.A,
                                             p.lda, p.B, p.ldb, p.beta, p.C0, p.ldc,
                                             nthreads=cores)
                total_dt += time.perf_counter() - t0
                total_flops += 2.0 * p.m * p.n * p.k
            got = gpu.reshape(p.n, p.ldc).T[:p.m, :]
            ok, mx, mean, ratio = oracle.check(got, cref, den, p.k)
            e = errors.setdefault(name, {"problems": [], "max_norm_err": 0.0, "mean_norm_err": 0.0,
                                         "max_over_bound": 0.0, "within_bound": True})
            e["problems"].append(p.label)
            e["max_norm_err"] = max(e["max_norm_err"], mx)
            e["mean_norm_err"] += mean / len(picks)
            e["max_over_bound"] = max(e["max_over_bound"], ratio)
            e["within_bound"] = e["within_bound"] and bool(ok)
    out["value"] = total_flops / total_dt / 1e12
    out["seconds"] = total_dt
    if workload == "c1":
        # the paper's host reference ran on one core: the same oracle on one thread
        p = picks[0].p
        t0 = time.perf_counter()
        oracle.sgemm_f64(p.transa, p.transb, p.m, p.n, p.k, p.alpha, p.A, p.lda, p.B, p.ldb,
                         p.beta, p.C0, p.ldc, nthreads=1)
        dt1 = time.perf_counter() - t0
        out["single_thread"] = {"value": 2.0 * p.m * p.n * p.k / dt1 / 1e12, "cores": 1,
                                "seconds": dt1}
    out["sample"] = ("full FP64 oracle (C and |A||B|) of the %d problems %s of the workload, "
                     "the same inputs as the GPU run; rate = sum 2MNK / time"
                     % (len(picks), ",".join(r.p.label for r in picks)))
    # sampled entries of every other problem, both forms
    for r in res:
        if r in picks:
            continue
        q = r.p
        rng = np.random.default_rng(17)
        rows = rng.integers(0, q.m, 512)
        cols = rng.integers(0, q.n, 512)
        cref_s, den_s = oracle.sgemm_f64_entries(q.transa, q.transb, q.m, q.n, q.k, q.alpha, q.A,
                                                 q.lda, q.B, q.ldb, q.beta, q.C0, q.ldc, rows,
                                                 cols, nthreads=cores)
        for mode, name in ((mg.FP32, "fp32"), (mg.BF16X3, "bf16x3")):
            r.reset()
            r.call(mg, mode)
            torch.cuda.synchronize()
            got = r.C.cpu().numpy()[rows + cols * q.ldc]
            ok, mx, mean, ratio = oracle.check(got, cref_s, den_s, q.k)
            e = errors.setdefault(name + "_sampled", {"max_over_bound": 0.0, "within_bound": True,
                                                     "entries_per_problem": 512})
            e["max_over_bound"] = max(e["max_over_bound"], ratio)
            e["within_bound"] = e["within_bound"] and bool(ok)
    return out, errors


def batch_measure(torch, mg, problems, mode, steps, warmup, no_clock=False):
    """Plan the batch, capture one persistent launch in a HIP graph, replay
    it warmup + steps times; the replays of the timed region are bracketed
    by events on the replay stream."""
    dev = torch.device("cuda:0")
    res = [Resident(p, dev) for p in problems]
    descs = [(r.p.transa, r.p.transb, r.p.m, r.p.n, r.p.k, r.p.alpha, r.A, r.p.lda, r.B, r.p.ldb,
              r.p.beta, r.C, r.p.ldc) for r in res]
    plan = mg.Batch(descs, mode=mode)
    info = plan.info()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        plan.launch()
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    if warmup > 0:
        warm(torch, g.replay, seconds=0.3)
    stream = torch.cuda.current_stream()
    evs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record(stream)
        g.replay()
        e.record(stream)
        evs.append((s, e))
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    durs = [s.elapsed_time(e) for s, e in evs]
    info["clock"] = None if no_clock else clock_probe(torch, g.replay, seconds=1.5)
    return res, plan, info, total, durs


def batch_errors(torch, mg, res, plan, cores):
    """Fresh eager launch, then sampled entries of every problem against the
    oracle (this is part of the CPU-baseline leg)."""
    import oracle
    for r in res:
        r.reset()
    plan.launch()
    torch.cuda.synchronize()
    worst = 0.0
    ok_all = True
    t0 = time.perf_counter()
    flops = 0.0
    for idx, r in enumerate(res):
        q = r.p
        rng = np.random.default_rng(idx)
        rows = rng.integers(0, q.m, 32)
        cols = rng.integers(0, q.n, 32)
        cref, den = oracle.sgemm_f64_entries(q.transa, q.transb, q.m, q.n, q.k, q.alpha, q.A,
                                             q.lda, q.B, q.ldb, q.beta, q.C0, q.ldc, rows, cols,
                                             nthreads=cores)
        flops += 2.0 * 32 * q.k
        got = r.C.cpu().numpy()[rows + cols * q.ldc]
        ok, mx, mean, ratio = oracle.check(got, cref, den, q.k)
        worst = max(worst, ratio)
        ok_all = ok_all and bool(ok)
    dt = time.perf_counter() - t0
    return {"max_over_bound": worst, "within_bound": ok_all, "entries_per_problem": 32}, flops, dt


def batch_line(args, torch, mg):
    from paper_1608_05265_amd import workloads as wl
    problems = wl.config5()
    flops = sum(p.flops() for p in problems)
    out = {}
    cores = len(os.sched_getaffinity(0))
    for mode, name in ((mg.FP32, "fp32"), (mg.BF16X3, "bf16x3")):
        res, plan, info, total, durs = batch_measure(torch, mg, problems, mode, args.steps,
                                                     args.warmup, args.no_clock)
        cfg = mg.config_info(info["config_id"])
        avg = float(np.mean(durs))
        out[name] = {"tflops": flops * args.steps / total / 1e12,
                     "ms_per_step": total / args.steps * 1e3,
                     "launch_avg_ms": avg,
                     "launch_tflops": flops / (avg * 1e-3) / 1e12,
                     "config": cfg["name"], "tiles": info["tiles"], "grid": info["grid"],
                     "second_config": (mg.config_info(info["second_config_id"])["name"]
                                       if info.get("second_config_id", -1) >= 0 else None),
                     "tile_efficiency": info["flops"] / info["tile_flops"],
                     "clock": info["clock"]}
        if not args.no_cpu_baseline:
            err, oflops, odt = batch_errors(torch, mg, res, plan, cores)
            out[name]["error"] = err
            out[name]["oracle_flops"] = oflops
            out[name]["oracle_seconds"] = odt
        plan.destroy()
        del res
        torch.cuda.empty_cache()
    f32 = out["fp32"]
    algo_bytes = sum(4.0 * (p.m * p.k + p.k * p.n + p.m * p.n * (1 + (p.beta != 0.0)))
                     for p in problems)
    line = {
        "metric": METRIC,
        "value": round(f32["tflops"], 3),
        "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(f32["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch of 512 independent GEMMs, M,N,K = 16*U{2..64}, "
                               "NN/NT/TN, alpha=1, beta in {0,1}, one persistent launch "
                               "replayed from a HIP graph", "flops_per_step": flops},
        "pct_of_fp32_peak": round(100.0 * f32["tflops"] / PEAK_FP32, 2),
        "bf16x3": {"value": round(out["bf16x3"]["tflops"], 3),
                   "pct_of_bf16_mfma_peak": round(100.0 * 6 * out["bf16x3"]["tflops"] / PEAK_BF16, 2),
                   "roofline": {
                       "bound": "mfma",
                       "kernel": "persistent batch kernel (%s%s)" % (
                           out["bf16x3"]["config"],
                           " + " + out["bf16x3"]["second_config"]
                           if out["bf16x3"]["second_config"] else ""),
                       "achieved": round(6 * out["bf16x3"]["launch_tflops"], 3),
                       "peak": PEAK_BF16,
                       "unit": "TFLOP/s of BF16 MFMA work (6 x the FP32-equivalent rate)",
                       "frac": round(6 * out["bf16x3"]["launch_tflops"] / PEAK_BF16, 4),
                       "avg_launch_ms": round(out["bf16x3"]["launch_avg_ms"], 4),
                       "flops_per_launch": 6 * flops,
                       "traffic": measured_traffic("batch_bf16x3", BATCH_TRAFFIC_FILE),
                       "traffic_requests": measured_bytes("batch_bf16x3", BATCH_TRAFFIC_FILE),
                       "algorithmic_bytes_per_launch": algo_bytes}},
        "roofline": {"bound": "mfma",
                     "kernel": "persistent batch kernel (%s%s)" % (
                         f32["config"], " + " + f32["second_config"] if f32["second_config"]
                         else ""),
                     "achieved": round(f32["launch_tflops"], 3), "peak": PEAK_FP32,
                     "unit": "TFLOP/s", "frac": round(f32["launch_tflops"] / PEAK_FP32, 4),
                     "avg_launch_ms": round(f32["launch_avg_ms"], 4),
                     "flops_per_launch": flops,
                     # per launch: both parts of a two-part plan
                     "traffic": measured_traffic("batch_fp32", BATCH_TRAFFIC_FILE),
                     "traffic_requests": measured_bytes("batch_fp32", BATCH_TRAFFIC_FILE),
                     "algorithmic_bytes_per_launch": algo_bytes},
        "detail": out,
    }
    if "oracle_seconds" in f32:
        line["cpu_baseline"] = {"cpu_model": cpu_model(),
                                "value": f32["oracle_flops"] / f32["oracle_seconds"] / 1e12,
                                "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
                                "sample": "32 entries of every one of the 512 problems (one dot "
                                          "product of length K each, with |A||B|); rate = "
                                          "2K per entry / time"}
    return line


def dgemm_line(args, torch, mg):
    """Double precision (the paper's dgemm, Section IV-B): M = N = K in
    {2048, 4096, 8192}, NN, alpha = 1.5, beta = -0.5, ld + 16, in both forms
    (FP64 matrix cores: the line's value; FP32 compute, the paper's "false
    dgemm": the fp32_compute object); errors and the CPU baseline from the
    binary128 oracle on sampled entries."""
    from paper_1608_05265_amd import workloads as wl
    dev = torch.device("cuda:0")
    probs = [wl.config6(sz) for sz in wl.DGEMM_SIZES]
    tens = [(torch.from_numpy(p.A).to(dev), torch.from_numpy(p.B).to(dev),
             torch.from_numpy(p.C0).to(dev)) for p in probs]
    flops_step = sum(2.0 * p.m * p.n * p.k for p in probs)
    stream = torch.cuda.current_stream()

    def call(i, dmode):
        p = probs[i]
        A, B, C = tens[i]
        mg.dgemm(p.transa, p.transb, p.m, p.n, p.k, p.alpha, A, p.lda, B, p.ldb, p.beta, C,
                 p.ldc, dmode)

    out = {}
    for dmode, name in ((mg.D_FP64, "fp64"), (mg.D_FP32, "fp32_compute")):
        for _ in range(args.warmup):
            for i in range(len(probs)):
                call(i, dmode)
        torch.cuda.synchronize()
        evs = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for i in range(len(probs)):
                if i == len(probs) - 1:
                    s_ = torch.cuda.Event(enable_timing=True)
                    e_ = torch.cuda.Event(enable_timing=True)
                    s_.record(stream)
                    call(i, dmode)
                    e_.record(stream)
                    evs.append((s_, e_))
                else:
                    call(i, dmode)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        dom = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        pd = probs[-1]
        out[name] = {"tflops": flops_step * args.steps / total / 1e12,
                     "ms_per_step": total / args.steps * 1e3, "dominant_avg_ms": dom,
                     "dominant_tflops": 2.0 * pd.m * pd.n * pd.k / (dom * 1e-3) / 1e12,
                     "clock": clock_probe(torch, lambda: call(len(probs) - 1, dmode))}
    f64 = out["fp64"]
    pd = probs[-1]
    line = {
        "metric": METRIC, "value": round(f64["tflops"], 3), "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(f64["ms_per_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "dgemm M=N=K in {2048,4096,8192}, NN, alpha=1.5, beta=-0.5, "
                               "ld=rows+16, uniform[-1,1], FP64 storage",
                   "flops_per_step": flops_step},
        "pct_of_fp64_peak": round(100.0 * f64["tflops"] / PEAK_FP64, 2),
        "fp32_compute": {"value": round(out["fp32_compute"]["tflops"], 3),
                         "pct_of_fp32_peak": round(100.0 * out["fp32_compute"]["tflops"] /
                                                   PEAK_FP32, 2),
                         "dominant_tflops": round(out["fp32_compute"]["dominant_tflops"], 2)},
        "roofline": {"bound": "mfma", "kernel": "FP64 MFMA tile kernel, %dx%dx%d NN"
                                                % (pd.m, pd.n, pd.k),
                     "achieved": round(f64["dominant_tflops"], 3), "peak": PEAK_FP64,
                     "unit": "TFLOP/s", "frac": round(f64["dominant_tflops"] / PEAK_FP64, 4),
                     "avg_launch_ms": round(f64["dominant_avg_ms"], 4),
                     "flops_per_launch": 2.0 * pd.m * pd.n * pd.k, "traffic": None},
        "clock": {k: v["clock"] for k, v in out.items()},
    }
    if not args.no_peak:
        peak = measure_peaks(torch, kinds=("fp64",), datas=("random",))["fp64_random"]
        line["roofline"]["measured_peak"] = peak["tflops"]
        line["roofline"]["frac_of_measured_peak"] = round(f64["dominant_tflops"] /
                                                          peak["tflops"], 4)
        line["measured_peak"] = {"fp64_random": peak}
    if not args.no_cpu_baseline:
        import oracle
        cores = len(os.sched_getaffinity(0))
        errs = {}
        t_or = 0.0
        fl_or = 0.0
        for i, p in enumerate(probs):
            rng = np.random.default_rng(31 + i)
            rows = rng.integers(0, p.m, 1024)
            cols = rng.integers(0, p.n, 1024)
            t0 = time.perf_counter()
            cref, den = oracle.dgemm_f128_entries(p.transa, p.transb, p.m, p.n, p.k, p.alpha,
                                                  p.A, p.lda, p.B, p.ldb, p.beta, p.C0, p.ldc,
                                                  rows, cols, nthreads=cores)
            t_or += time.perf_counter() - t0
            fl_or += 2.0 * p.k * rows.size
            for dmode, name, tol_fn in ((mg.D_FP64, "fp64", oracle.tol_d),
                                        (mg.D_FP32, "fp32_compute", oracle.tol_false_d)):
                A, B, C = tens[i]
                C.copy_(torch.from_numpy(p.C0).to(dev))
                call(i, dmode)
                torch.cuda.synchronize()
                got = C.cpu().numpy()[rows + cols * p.ldc]
                ok, mx, mean, ratio = oracle.check(got, cref, den, p.k, tol_fn)
                e = errs.setdefault(name, {"max_norm_err": 0.0, "max_over_bound": 0.0,
                                           "within_bound": True, "entries_per_problem": 1024})
                e["max_norm_err"] = max(e["max_norm_err"], mx)
                e["max_over_bound"] = max(e["max_over_bound"], ratio)
                e["within_bound"] = e["within_bound"] and bool(ok)
        line["error"] = errs
        line["cpu_baseline"] = {"cpu_model": cpu_model(),
                                "value": fl_or / t_or / 1e12, "unit": "TFLOP/s", "cores": cores,
                                "kind": "oracle",
                                "sample": "binary128 oracle on 1024 sampled entries of each "
                                          "problem (one length-K dot product with |A||B| per "
                                          "entry); rate = 2K per entry / time"}
    return line


def host_line(args, torch, mg):
    """Host-pointer sgemm (the Fortran-style drop-in): square NN problems at
    4096^3 and 8192^3 with padded leading dimensions (C then moves column by
    column) and 8192^3 with tight ones, operands and result in host memory;
    the rate includes every PCIe transfer (A, B and C0 in, C out) and is
    compared with the device-resident rate of the same call."""
    from paper_1608_05265_amd import workloads as wl
    rows = []
    for size, pad in ((4096, 16), (8192, 16), (8192, 0)):
        p = wl.make_problem("N", "N", size, size, size, 1.5, -0.5, wl.seed_for(2, 100 + size),
                            pad=pad, label="host%d_pad%d" % (size, pad))
        C = p.C0.copy()
        call = lambda: mg.sgemm_host("N", "N", p.m, p.n, p.k, p.alpha, p.A, p.lda, p.B, p.ldb,
                                     p.beta, C, p.ldc)
        for _ in range(args.warmup):
            call()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            call()
        dt = (time.perf_counter() - t0) / args.steps
        moved = 4.0 * (p.lda * p.k + p.ldb * p.n + 2 * p.m * p.n)
        r = Resident(p, torch.device("cuda:0"))
        torch.cuda.synchronize()
        s_ = torch.cuda.Event(enable_timing=True)
        e_ = torch.cuda.Event(enable_timing=True)
        r.call(mg, mg.FP32)
        s_.record()
        for _ in range(args.steps):
            r.call(mg, mg.FP32)
        e_.record()
        torch.cuda.synchronize()
        dev_ms = s_.elapsed_time(e_) / args.steps
        rows.append({"size": size, "ld_pad": pad, "host_tflops": round(p.flops() / dt / 1e12, 2),
                     "host_ms": round(dt * 1e3, 3), "pcie_bytes": moved,
                     "effective_gb_s": round(moved / dt / 1e9, 1),
                     "device_tflops": round(p.flops() / (dev_ms * 1e-3) / 1e12, 2)})
        del r
    return {"workload": "host-pointer sgemm (square sweep problems, NN, FP32), PCIe-inclusive",
            "rows": rows}


def hpl_residual(a, x, b, eps):
    """HPL's check of a solve (the formula of the paper's Table VII footnote):
    ||A x - b||_inf / (eps (||A||_inf ||x||_inf + ||b||_inf) N), in FP64."""
    a64 = np.asarray(a, dtype=np.float64)
    x64 = np.asarray(x, dtype=np.float64).reshape(-1)
    b64 = np.asarray(b, dtype=np.float64).reshape(-1)
    r = np.max(np.abs(a64 @ x64 - b64))
    norm_a = np.max(np.sum(np.abs(a64), axis=1))
    return float(r / (eps * (norm_a * np.max(np.abs(x64)) + np.max(np.abs(b64))) * a64.shape[0]))


def lu_line(args, torch, mg):
    """The Linpack workload of the paper (Section IV-C): LU with partial
    pivoting of an N x N uniform[-1,1] matrix and the solve of A x = b, at
    the paper's N = 4608 and at N = 16384, trailing updates in both sgemm
    forms; GFLOP/s by the HPL count (2/3 N^3 + 3/2 N^2) / t, and the scaled
    residual of Table VII's footnote (with FP32's eps, and with the 2^-53 the paper's
    double-precision HPL used)."""
    dev = torch.device("cuda:0")
    rows = []
    for n in (4608, 16384):
        rng = np.random.default_rng(4608 + n)
        a = rng.uniform(-1, 1, (n, n)).astype(np.float32)
        b = rng.uniform(-1, 1, n).astype(np.float32)
        a_cm = torch.from_numpy(np.ascontiguousarray(a.T).reshape(-1)).to(dev)
        for mode, name in ((mg.FP32, "fp32"), (mg.BF16X3, "bf16x3")):
            times = []
            for rep_ in range(args.warmup + max(1, min(args.steps, 3))):
                A = a_cm.clone()
                ipiv = torch.empty(n, dtype=torch.int64, device=dev)
                info = torch.empty(1, dtype=torch.int32, device=dev)
                B = torch.from_numpy(b.copy()).to(dev)
                torch.cuda.synchronize()
                s_ = torch.cuda.Event(enable_timing=True)
                m_ = torch.cuda.Event(enable_timing=True)
                e_ = torch.cuda.Event(enable_timing=True)
                s_.record()
                mg.sgetrf(n, A, n, ipiv, info, mode)
                m_.record()
                mg.sgetrs(n, 1, A, n, ipiv, B, n, mode)
                e_.record()
                torch.cuda.synchronize()
                if rep_ >= args.warmup:
                    times.append((s_.elapsed_time(m_), m_.elapsed_time(e_)))
            t_f = min(t[0] for t in times) * 1e-3
            t_s = min(t[1] for t in times) * 1e-3
            x = B.cpu().numpy().astype(np.float64)
            hpl_flops = 2.0 / 3.0 * n ** 3 + 1.5 * n ** 2
            rows.append({"n": n, "form": name, "info": int(info.item()),
                         "getrf_ms": round(t_f * 1e3, 3), "getrs_ms": round(t_s * 1e3, 3),
                         "gflops": round(hpl_flops / (t_f + t_s) / 1e9, 1),
                         "scaled_residual_eps32": hpl_residual(a, x, b, 2.0 ** -24),
                         "scaled_residual_eps64": hpl_residual(a, x, b, 2.0 ** -53)})
            del A, B
        del a_cm
    line = {"workload": "LU with partial pivoting + solve (HPL-style), uniform[-1,1]",
            "rows": rows,
            "paper": "Parallella, N=4608, NB=768: 0.495 GFLOP/s, scaled residual 2.11e10 "
                     "(eps 2^-53), Table VII"}
    if not args.no_cpu_baseline:
        import oracle
        cores = len(os.sched_getaffinity(0))
        n = 2048
        a = np.random.default_rng(7).uniform(-1, 1, (n, n)).astype(np.float32)
        t0 = time.perf_counter()
        oracle.getrf_f64(n, np.ascontiguousarray(a.T).reshape(-1), n, nthreads=cores)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"cpu_model": cpu_model(),
                                "value": (2.0 / 3.0 * n ** 3) / dt / 1e9, "unit": "GFLOP/s",
                                "cores": cores, "kind": "oracle",
                                "sample": "FP64 textbook LU of one 2048 x 2048 matrix"}
    return line


COPY_BYTES = 1 << 30
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sgemm_dominant8192_hbm_counters.txt")
BATCH_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "batch512_kernel_trace.txt")
# what decides the sgemm kernels and which of them runs: their sources and
# the packaged tuning table
KERNEL_SOURCES = ["gemm_tile.hpp", "gemm_rtile.hpp", "packed_x3.hpp", "registry.hpp", "aux_kernels.hip",
                  "sgemm_f32.hip", "sgemm_x3.hip", "sgemm_x3k.hip"]
# host code that decides what the kernels touch and in which order (tile
# choice, tile order, the batch plan's tile lists), hashed with the kernels
SCHEDULE_SOURCES = ["api.cpp"]
TUNING_TABLE = os.path.join(ROOT, "paper_1608_05265_amd", "tuning_mi355x.txt")


def kernel_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES + SCHEDULE_SOURCES:
        with open(os.path.join(ROOT, "paper_1608_05265_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    with open(TUNING_TABLE, "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(form: str, path: str = ""):
    """HBM bytes per launch of a kernel from a committed counter summary
    (FETCH_SIZE and WRITE_SIZE runs, calibrated on a copy kernel; the
    dominant-kernel summary unless `path` names another), or None when the
    kernel sources, the host code that schedules their tiles or the tuning
    table changed since the counters were taken."""
    try:
        with open(path or TRAFFIC_FILE) as f:
            for line in f:
                parts = line.split()
                if len(parts) == 4 and parts[0] == "traffic_bytes_per_launch" and \
                        parts[1] == form:
                    return float(parts[3]) if parts[2] == kernel_sources_hash() else None
    except OSError:
        return None
    return None


def measured_bytes(form: str, path: str = ""):
    """The L2-to-memory request bytes per launch of a kernel from a committed
    counter summary (TCC_EA0 read requests by size, 128/64/32 bytes, and
    write requests, each with the part addressed to the memory controller:
    Infinity Cache and HBM), or None when the kernel sources, their host
    scheduling code or the tuning table changed since the counters were
    taken."""
    try:
        with open(path or TRAFFIC_FILE) as f:
            for line in f:
                parts = line.split()
                if len(parts) == 7 and parts[0] == "ea_bytes_per_launch" and parts[1] == form:
                    if parts[2] != kernel_sources_hash():
                        return None
                    rd, rd_dram, wr, wr_dram = (float(v) for v in parts[3:])
                    return {"read": rd, "read_to_memory": rd_dram, "write": wr,
                            "write_to_memory": wr_dram, "total": rd + wr,
                            "unit": "bytes per launch leaving the L2 (TCC_EA0 requests x size)"}
    except OSError:
        return None
    return None


def dominant_only(args, torch, mg):
    """The dominant problem alone, for rocprofv3 runs: `steps` calls of the
    8192^3 NN sgemm in each form, then `steps` device-to-device copies of
    COPY_BYTES (a plain copy kernel of known traffic, to calibrate the HBM
    byte counters)."""
    from paper_1608_05265_amd import workloads as wl
    r = Resident(wl.config2(8192, "N", "N"), torch.device("cuda:0"))
    for mode in (mg.FP32, mg.BF16X3):
        for _ in range(args.steps):
            r.call(mg, mode)
    src = torch.empty(COPY_BYTES // 4, device="cuda:0")
    src.fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"workload": "dominant", "steps": args.steps, "copy_bytes": COPY_BYTES}))


def event_median_ms(torch, fn, reps):
    """Median and minimum of `reps` calls of fn, each bracketed by HIP events
    on torch's current stream (the stream the library launches on)."""
    stream = torch.cuda.current_stream()
    evs = []
    for _ in range(reps):
        s_ = torch.cuda.Event(enable_timing=True)
        e_ = torch.cuda.Event(enable_timing=True)
        s_.record(stream)
        fn()
        e_.record(stream)
        evs.append((s_, e_))
    torch.cuda.synchronize()
    d = sorted(a.elapsed_time(b) for a, b in evs)
    return d[len(d) // 2], d[0]


def warm(torch, fn, seconds=0.5):
    """Run fn back to back for about `seconds`, so that a GPU that idled while
    the host drew the next inputs is back at its working clock before the
    timed calls (a cold GPU ran the first calls up to 15 % slower)."""
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds:
        fn()
        n += 1
        if n % 8 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()


def copy_bandwidth(torch, nbytes=COPY_BYTES, reps=20):
    """Achievable HBM bandwidth on this GPU: a device-to-device copy of
    `nbytes` (4x the 256 MB Infinity Cache), read + write bytes over the
    median event-timed copy."""
    src = torch.empty(nbytes // 4, device="cuda:0")
    src.fill_(1.0)
    dst = torch.empty_like(src)
    warm(torch, lambda: dst.copy_(src))
    med, best = event_median_ms(torch, lambda: dst.copy_(src), reps)
    del src, dst
    torch.cuda.empty_cache()
    return {"gbs": round(2.0 * nbytes / (med * 1e-3) / 1e9, 1),
            "gbs_best": round(2.0 * nbytes / (best * 1e-3) / 1e9, 1),
            "bytes_per_copy": 2 * nbytes, "spec_gbs": PEAK_HBM,
            "how": "device-to-device copy of 1 GiB (read + write), median of %d event-timed "
                   "copies" % reps}


def sampled_error(mg, torch, r, mode, count, seed, cores):
    """Run r once in `mode` from a pristine C0 and compare `count` random
    entries with the FP64 oracle: (max, mean normalized error, max/bound,
    within bound)."""
    import oracle
    q = r.p
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, q.m, count)
    cols = rng.integers(0, q.n, count)
    cref, den = oracle.sgemm_f64_entries(q.transa, q.transb, q.m, q.n, q.k, q.alpha, q.A, q.lda,
                                         q.B, q.ldb, q.beta, q.C0, q.ldc, rows, cols,
                                         nthreads=cores)
    r.reset()
    r.call(mg, mode)
    torch.cuda.synchronize()
    got = r.C.cpu().numpy()[rows + cols * q.ldc]
    ok, mx, mean, ratio = oracle.check(got, cref, den, q.k)
    return float(mx), float(mean), float(ratio), bool(ok)


def wide_object(args, torch, mg, cores):
    """The precision form's workload: 8192^3 NN, entries random sign x 2^U[-8,8],
    alpha = 1, beta = 0, both forms on the same inputs: rate, share of each
    form's matrix-core peak, and the normalized error of 2048 entries checked
    against the FP64 oracle, with the split form's error over the native one
    (equal error: both ratios at most EQUAL_ERROR_RATIO)."""
    from paper_1608_05265_amd import workloads as wl
    r = Resident(wl.config4(), torch.device("cuda:0"))
    p = r.p
    flops = 2.0 * p.m * p.n * p.k
    out = {"workload": "8192^3 NN, alpha=1, beta=0, entries random sign x 2^U[-8,8] "
                       "(continuous U), both forms on the same inputs"}
    for mode, name in ((mg.FP32, "fp32"), (mg.BF16X3, "bf16x3")):
        warm(torch, lambda: r.call(mg, mode))
        med, best = event_median_ms(torch, lambda: r.call(mg, mode), max(args.steps, 10))
        tf = flops / (med * 1e-3) / 1e12
        o = {"tflops": round(tf, 3), "ms": round(med, 4), "ms_min": round(best, 4)}
        if name == "fp32":
            o["pct_of_fp32_mfma_peak"] = round(100.0 * tf / PEAK_FP32, 2)
        else:
            o["pct_of_bf16_mfma_peak"] = round(100.0 * 6 * tf / PEAK_BF16, 2)
        if not args.no_cpu_baseline:
            mx, mean, ratio, ok = sampled_error(mg, torch, r, mode, 2048, 44, cores)
            o["error"] = {"max_norm_err": mx, "mean_norm_err": mean, "max_over_bound": ratio,
                          "within_bound": ok, "entries": 2048}
        out[name] = o
    if not args.no_cpu_baseline:
        e0, e1 = out["fp32"]["error"], out["bf16x3"]["error"]
        rmax = e1["max_norm_err"] / e0["max_norm_err"]
        rmean = e1["mean_norm_err"] / e0["mean_norm_err"]
        out["bf16x3_over_fp32_error"] = {"max": round(rmax, 4), "mean": round(rmean, 4)}
        out["equal_error"] = bool(rmax <= EQUAL_ERROR_RATIO and rmean <= EQUAL_ERROR_RATIO)
        out["equal_error_rule"] = "split-form max and mean normalized error each at most %.1f x " \
                                  "the native form's on the same 2048 entries" % EQUAL_ERROR_RATIO
    del r
    torch.cuda.empty_cache()
    return out


def rankk_object(args, torch, mg, copy_gbs, cores):
    """The Linpack-style trailing update, 16384^2 x K for K in {128, 256, 512},
    alpha = -1, beta = 1, normal(0,1), both forms: rate, algorithmic HBM
    GB/s, and the time against the larger of its two floors (matrix cores
    at spec peak, algorithmic bytes at the measured copy bandwidth)."""
    from paper_1608_05265_amd import workloads as wl
    rows = []
    for k in wl.RANKK_KS:
        r = Resident(wl.config3(k), torch.device("cuda:0"))
        p = r.p
        flops = 2.0 * p.m * p.n * p.k
        nbytes = float(p.bytes())
        row = {"k": k, "algorithmic_bytes": nbytes, "flops": flops}
        for mode, name, peak, mult in ((mg.FP32, "fp32", PEAK_FP32, 1),
                                       (mg.BF16X3, "bf16x3", PEAK_BF16, 6)):
            warm(torch, lambda: r.call(mg, mode))
            med, _ = event_median_ms(torch, lambda: r.call(mg, mode), max(args.steps, 10))
            mfma_floor = mult * flops / (peak * 1e12) * 1e3
            hbm_floor = nbytes / (copy_gbs * 1e9) * 1e3
            o = {"tflops": round(flops / (med * 1e-3) / 1e12, 3), "ms": round(med, 4),
                 "gbs": round(nbytes / (med * 1e-3) / 1e9, 1),
                 "mfma_floor_ms": round(mfma_floor, 4), "hbm_floor_ms": round(hbm_floor, 4),
                 "bound": "mfma" if mfma_floor >= hbm_floor else "hbm",
                 "frac_of_floor": round(max(mfma_floor, hbm_floor) / med, 4)}
            if not args.no_cpu_baseline:
                mx, mean, ratio, ok = sampled_error(mg, torch, r, mode, 512, 45 + k, cores)
                o["error"] = {"max_over_bound": ratio, "within_bound": ok, "entries": 512}
            row[name] = o
        rows.append(row)
        del r
        torch.cuda.empty_cache()
    return {"workload": "16384^2 x K, K in {128,256,512}, NN, alpha=-1, beta=1, normal(0,1) "
                        "(Linpack-style trailing update)",
            "hbm_roof_gbs": copy_gbs, "hbm_roof": "measured copy bandwidth", "rows": rows}


def c1_object(args, torch, mg):
    """The 256^3 single call (NN, alpha = 1, beta = 0): per-call latency in
    both forms (1000 event-timed calls: median and minimum; 1000 calls back
    to back: host wall time per call) and the rate at the median."""
    from paper_1608_05265_amd import workloads as wl
    r = Resident(wl.config1(), torch.device("cuda:0"))
    flops = 2.0 * r.p.m * r.p.n * r.p.k
    out = {"workload": "256^3 NN, alpha=1, beta=0, uniform[-1,1]"}
    for mode, name in ((mg.FP32, "fp32"), (mg.BF16X3, "bf16x3")):
        warm(torch, lambda: r.call(mg, mode))
        lat = latency(torch, r, mg, mode)
        lat["tflops_at_median"] = round(flops / (lat["median_us"] * 1e-6) / 1e12, 3)
        lat["config"] = mg.config_info(mg.select_config("N", "N", 256, 256, 256, mode))["name"]
        out[name] = lat
    del r
    torch.cuda.empty_cache()
    return out


def progress(msg):
    """A stage of the run, on stderr (stdout carries only the JSON line)."""
    print("bench: %s (%.0f s)" % (msg, time.perf_counter() - _T0), file=sys.stderr, flush=True)


_T0 = time.perf_counter()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1608_05265_amd as mg
    dev = torch.device("cuda:0")
    if args.workload == "batch":
        line = batch_line(args, torch, mg)
        print(json.dumps(line))
        return
    if args.workload == "dominant":
        dominant_only(args, torch, mg)
        return
    if args.workload == "lu":
        print(json.dumps(lu_line(args, torch, mg)))
        return
    if args.workload == "host":
        print(json.dumps(host_line(args, torch, mg)))
        return
    if args.workload == "dgemm":
        print(json.dumps(dgemm_line(args, torch, mg)))
        return
    if args.workload == "peak":
        print(json.dumps({"workload": "peak", "spec_tflops": {"fp32": PEAK_FP32,
                                                             "bf16": PEAK_BF16},
                          "measured": measure_peaks(torch)}))
        return
    problems, desc = make_problems(args.workload, args.problem)
    # the split-K regime's tuned entries are split-K configurations in both
    # forms, which misgemm_sgemm runs (misgemm_sgemm_ws never splits K)
    split_regime = args.workload == "skinny"
    res = [Resident(p, dev, ws=not split_regime) for p in problems]
    torch.cuda.synchronize()
    flops_step = sum(2.0 * r.p.m * r.p.n * r.p.k for r in res)
    big = max(r.p.m * r.p.n * r.p.k for r in res)
    dominant = [i for i, r in enumerate(res) if r.p.m * r.p.n * r.p.k == big]

    progress("inputs of %d problems resident" % len(res))
    result = {}
    for mode, name in ((mg.FP32, "fp32"), (mg.BF16X3, "bf16x3")):
        total, durs = time_steps(torch, res, mg, mode, args.steps, args.warmup, dominant)
        dp = res[dominant[0]].p
        per_launch = 2.0 * dp.m * dp.n * dp.k
        avg_ms = float(np.mean(durs))
        result[name] = {"seconds": total, "tflops": flops_step * args.steps / total / 1e12,
                        "ms_per_step": total / args.steps * 1e3,
                        "dominant_avg_ms": avg_ms,
                        "dominant_tflops": per_launch / (avg_ms * 1e-3) / 1e12,
                        "dominant": "%dx%dx%d (%s)" % (dp.m, dp.n, dp.k,
                                                       ",".join(res[i].p.transa + res[i].p.transb
                                                                for i in dominant)),
                        "clock": None if args.no_clock else
                        clock_probe(torch, lambda: res[dominant[0]].call(mg, mode))}
    progress("timed steps done")
    # per-problem rates (one extra timed pass each, after the timed region)
    per_problem = []
    for r in res:
        row = {"problem": r.p.label}
        for mode, name in ((mg.FP32, "fp32"), (mg.BF16X3, "bf16x3")):
            s = torch.cuda.Event(enable_timing=True)
            e = torch.cuda.Event(enable_timing=True)
            r.call(mg, mode)
            s.record()
            reps = 5
            for _ in range(reps):
                r.call(mg, mode)
            e.record()
            torch.cuda.synchronize()
            ms = s.elapsed_time(e) / reps
            row[name + "_tflops"] = round(2.0 * r.p.m * r.p.n * r.p.k / ms / 1e9, 2)
        if args.workload == "c1":
            for mode, name in ((mg.FP32, "fp32"), (mg.BF16X3, "bf16x3")):
                row[name + "_latency"] = latency(torch, r, mg, mode)
        per_problem.append(row)

    f32 = result["fp32"]
    x3 = result["bf16x3"]
    dp = res[dominant[0]].p
    line = {
        "metric": METRIC,
        "value": round(f32["tflops"], 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f32["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "gemms_per_step": len(res),
                   "flops_per_step": flops_step,
                   "forms": "fp32 (value, misgemm_sgemm), bf16x3 (bf16x3 object, " +
                            ("misgemm_sgemm, split-K partials in the library scratch)"
                             if split_regime else
                             "misgemm_sgemm_ws with a caller-owned workspace)")},
        "pct_of_fp32_peak": round(100.0 * f32["tflops"] / PEAK_FP32, 2),
        "bf16x3": {"value": round(x3["tflops"], 3), "unit": "TFLOP/s (FP32-equivalent, 2MNK)",
                   "ms_per_step": round(x3["ms_per_step"], 4),
                   "pct_of_bf16_mfma_peak": round(100.0 * 6 * x3["tflops"] / PEAK_BF16, 2),
                   "dominant_tflops": round(x3["dominant_tflops"], 2)},
        "roofline": {
            "bound": "mfma",
            "kernel": "sgemm fp32 tile kernel, %s" % f32["dominant"],
            "achieved": round(f32["dominant_tflops"], 3),
            "peak": PEAK_FP32,
            "unit": "TFLOP/s",
            "frac": round(f32["dominant_tflops"] / PEAK_FP32, 4),
            "avg_launch_ms": round(f32["dominant_avg_ms"], 4),
            "flops_per_launch": 2.0 * dp.m * dp.n * dp.k,
            "traffic": measured_traffic("fp32") if (dp.m, dp.n, dp.k) == (8192, 8192, 8192)
            else None,
            "traffic_unit": "bytes per launch beyond the L2, to the memory controller (Infinity "
                            "Cache and HBM behind it; rocprofv3 FETCH_SIZE and WRITE_SIZE, each "
                            "scaled by its reading for a copy of known size)",
            "traffic_requests": measured_bytes("fp32")
            if (dp.m, dp.n, dp.k) == (8192, 8192, 8192) else None,
            "algorithmic_bytes_per_launch": 4.0 * (dp.m * dp.k + dp.k * dp.n + 2 * dp.m * dp.n),
        },
        "per_problem": per_problem,
        "clock": {"fp32": f32["clock"], "bf16x3": x3["clock"]},
    }
    # the split form's dominant kernel against the BF16 matrix cores it runs on
    # (six BF16 products per FP32-equivalent flop)
    line["bf16x3"]["roofline"] = {
        "bound": "mfma",
        "kernel": "sgemm bf16x3 tile kernel, %s" % x3["dominant"],
        "achieved": round(6 * x3["dominant_tflops"], 3),
        "peak": PEAK_BF16,
        "unit": "TFLOP/s of BF16 MFMA work (6 x the FP32-equivalent rate)",
        "frac": round(6 * x3["dominant_tflops"] / PEAK_BF16, 4),
        "avg_launch_ms": round(x3["dominant_avg_ms"], 4),
        "flops_per_launch": 6 * 2.0 * dp.m * dp.n * dp.k,
        "traffic": measured_traffic("bf16x3") if (dp.m, dp.n, dp.k) == (8192, 8192, 8192)
        else None,
        "traffic_requests": measured_bytes("bf16x3")
        if (dp.m, dp.n, dp.k) == (8192, 8192, 8192) else None,
        "algorithmic_bytes_per_launch": 4.0 * (dp.m * dp.k + dp.k * dp.n + 2 * dp.m * dp.n),
    }
    progress("per-problem rates done")
    if not args.no_cpu_baseline:
        cpu, errors = cpu_baseline_leg(res, mg, torch, args.workload)
        progress("oracle leg done")
        line["cpu_baseline"] = cpu
        line["error"] = errors
    if args.workload == "square" and not args.no_peak:
        peaks = measure_peaks(torch)
        progress("matrix-core peaks measured")
        line["measured_peak"] = peaks
        fp = peaks["fp32_random"]["tflops"]
        line["roofline"]["measured_peak"] = fp
        line["roofline"]["frac_of_measured_peak"] = round(f32["dominant_tflops"] / fp, 4)
        line["bf16x3"]["pct_of_measured_bf16_peak"] = round(
            100.0 * 6 * x3["tflops"] / peaks["bf16_random"]["tflops"], 2)
        bp = peaks["bf16_random"]["tflops"]
        line["bf16x3"]["roofline"]["measured_peak"] = bp
        line["bf16x3"]["roofline"]["frac_of_measured_peak"] = round(
            6 * x3["dominant_tflops"] / bp, 4)
    if args.workload == "square" and not args.no_extra:
        del res
        torch.cuda.empty_cache()
        res = []
        cores = len(os.sched_getaffinity(0))
        line["wide8192"] = wide_object(args, torch, mg, cores)
        progress("wide-range workload done")
        copy = copy_bandwidth(torch)
        line["hbm_copy"] = copy
        line["rankk"] = rankk_object(args, torch, mg, copy["gbs"], cores)
        progress("rank-k workload done")
        line["c1"] = c1_object(args, torch, mg)
    if args.workload == "square" and not args.no_batch:
        del res
        torch.cuda.empty_cache()
        b = batch_line(args, torch, mg)
        line["batch512"] = {"fp32_tflops": b["value"], "bf16x3_tflops": b["bf16x3"]["value"],
                            "roofline": b["roofline"],
                            "bf16x3_roofline": b["bf16x3"]["roofline"], "detail": b["detail"]}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
