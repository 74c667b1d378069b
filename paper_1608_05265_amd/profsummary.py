"""Summaries of rocprofv3 CSV output (kernel trace and counter collection).

    python -m paper_1608_05265_amd.profsummary trace <dir-with-kernel_trace.csv>
    python -m paper_1608_05265_amd.profsummary pmc <dir-with-counter_collection.csv>
    python -m paper_1608_05265_amd.profsummary dispatch <dir-with-counter_collection.csv>
    python -m paper_1608_05265_amd.profsummary bytes <read-dir> <write-dir>
    python -m paper_1608_05265_amd.profsummary traffic <fetch-dir> <write-dir> \
        <read-req-dir> <write-req-dir> <kernel-regex> [<form> <hash>]

`trace` groups dispatches by kernel and grid size and prints calls, average,
minimum and maximum duration in microseconds; `pmc` prints the per-dispatch
average of every collected counter, also grouped by kernel and grid size,
plus, when SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE were collected, the
matrix-core busy fraction busy / (SIMDs * GRBM_GUI_ACTIVE / XCDs) (the busy
counter sums the cycles of every SIMD, GRBM_GUI_ACTIVE sums the active
cycles of the 8 XCDs; 1024 SIMDs on MI355X); `dispatch` prints every
dispatch with its counters (for calibration runs that mix kernels of one
name); `bytes` turns the L2-to-memory request counters of two runs into
bytes per dispatch (below); `traffic` sums, over the kernels whose short
name matches the regex (the kernels of one call or one launch, each run
once per call), the per-dispatch means of FETCH_SIZE and WRITE_SIZE, scaled
by their readings for a plain copy of known size, and of the request bytes,
and with a form name and a source hash prints them as the
`traffic_bytes_per_launch` and `ea_bytes_per_launch` lines bench.py reads.
Kernel names are shortened to the template arguments that identify a tile
configuration.
"""
from __future__ import annotations

import collections
import csv
import glob
import os
import re
import sys


def short_name(name: str) -> str:
    m = re.search(r"misgemm::(\w+)<misgemm::RTileBase<misgemm::RShape<([\d, ]+)>, (\w+), (\w+), "
                  r"misgemm::RMath(\w+)>", name)
    if m:
        shape = "x".join(v.strip() for v in m.group(2).split(","))
        return "%s<R%s %s %s,%s>" % (m.group(1), m.group(5), shape, m.group(3), m.group(4))
    m = re.search(r"misgemm::(\w+)<misgemm::(\w+)<misgemm::Shape<([\d, ]+)>, ([^>]*)>", name)
    if m:
        shape = "x".join(v.strip() for v in m.group(3).split(","))
        return "%s<%s %s %s>" % (m.group(1), m.group(2), shape, m.group(4).replace(" ", ""))
    m = re.search(r"misgemm::(\w+)<misgemm::Shape<([\d, ]+)> ?>", name)
    if m:
        return "%s<%s>" % (m.group(1), "x".join(v.strip() for v in m.group(2).split(",")))
    m = re.search(r"misgemm::(\w+)<misgemm::[^,]*?(\w+), misgemm::Shape<([\d, ]+)>", name)
    if m:
        shape = "x".join(v.strip() for v in m.group(3).split(","))
        return "%s<%s %s>" % (m.group(1), m.group(2), shape)
    m = re.search(r"misgemm::(\w+)<(true|false)>", name)
    if m:
        return "%s<%s>" % (m.group(1), m.group(2))
    m = re.search(r"misgemm::(\w+)", name)
    if m:
        return m.group(1)
    return name[:60]


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError("no *%s under %s" % (suffix, d))
    return hits[0]


def trace(d: str):
    rows = list(csv.DictReader(open(_find(d, "kernel_trace.csv"))))
    groups = collections.OrderedDict()
    for r in rows:
        grid = "%sx%sx%s" % (r.get("Grid_Size_X", r.get("Grid_Size", "?")),
                             r.get("Grid_Size_Y", "1"), r.get("Grid_Size_Z", "1"))
        key = (short_name(r["Kernel_Name"]), grid)
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1000.0
        groups.setdefault(key, []).append(dur)
    out = ["%-58s %-16s %6s %11s %11s %11s" % ("kernel", "grid", "calls", "avg_us", "min_us",
                                               "max_us")]
    for (k, g), v in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        out.append("%-58s %-16s %6d %11.2f %11.2f %11.2f" % (k, g, len(v), sum(v) / len(v),
                                                             min(v), max(v)))
    return "\n".join(out)


def pmc(d: str):
    rows = list(csv.DictReader(open(_find(d, "counter_collection.csv"))))
    groups = collections.OrderedDict()
    for r in rows:
        key = (short_name(r["Kernel_Name"]), r.get("Grid_Size", "?"), r["Counter_Name"])
        groups.setdefault(key, {})
        groups[key].setdefault(r["Dispatch_Id"], 0.0)
        groups[key][r["Dispatch_Id"]] += float(r["Counter_Value"])
    out = ["%-58s %-10s %-14s %6s %16s" % ("kernel", "grid", "counter", "disp", "avg_per_disp")]
    for (k, g, c), v in groups.items():
        vals = list(v.values())
        out.append("%-58s %-10s %-14s %6d %16.1f" % (k, g, c, len(vals), sum(vals) / len(vals)))
    return "\n".join(out)


SIMDS, XCDS = 1024, 8


def mfma_busy(d: str):
    """Per (kernel, grid): mean matrix-core busy fraction over dispatches."""
    rows = list(csv.DictReader(open(_find(d, "counter_collection.csv"))))
    per = collections.OrderedDict()
    for r in rows:
        per.setdefault(r["Dispatch_Id"], [short_name(r["Kernel_Name"]), r.get("Grid_Size", "?"),
                                          collections.defaultdict(float)])
        per[r["Dispatch_Id"]][2][r["Counter_Name"]] += float(r["Counter_Value"])
    groups = collections.OrderedDict()
    for name, grid, c in per.values():
        if c.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) > 0 and c.get("GRBM_GUI_ACTIVE", 0.0) > 0:
            frac = c["SQ_VALU_MFMA_BUSY_CYCLES"] / (SIMDS * c["GRBM_GUI_ACTIVE"] / XCDS)
            groups.setdefault((name, grid), []).append(frac)
    out = []
    for (k, g), v in groups.items():
        out.append("%-58s %-10s %-14s %6d %16.3f" % (k, g, "mfma_busy_frac", len(v),
                                                     sum(v) / len(v)))
    return "\n".join(out)


def dispatch(d: str):
    rows = list(csv.DictReader(open(_find(d, "counter_collection.csv"))))
    per = collections.OrderedDict()
    for r in rows:
        key = int(r["Dispatch_Id"])
        per.setdefault(key, [short_name(r["Kernel_Name"]), r.get("Grid_Size", "?"),
                             collections.OrderedDict()])
        c = per[key][2]
        c[r["Counter_Name"]] = c.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    out = ["%-6s %-58s %-10s %s" % ("disp", "kernel", "grid", "counters")]
    for key in sorted(per):
        name, grid, c = per[key]
        out.append("%-6d %-58s %-10s %s" % (key, name, grid,
                                            " ".join("%s=%.1f" % kv for kv in c.items())))
    return "\n".join(out)


# Bytes that leave the L2 (the TCC/EA interface), counted by request size:
# reads 128 * TCC_EA0_RDREQ_128B + 64 * TCC_EA0_RDREQ_64B + 32 * TCC_EA0_RDREQ_32B,
# of which 32 * TCC_EA0_RDREQ_DRAM_32B go to the memory controller (DRAM: the
# Infinity Cache and HBM behind it; the rest goes to GMI/IO); writes
# 64 * TCC_EA0_WRREQ_64B + 32 * (TCC_EA0_WRREQ - TCC_EA0_WRREQ_64B), of which
# 32 * TCC_EA0_WRREQ_WRITE_DRAM_32B go to the memory controller.  (The
# FETCH_SIZE expression of this rocprofv3 prices 128-byte reads through
# TCC_BUBBLE, which reads 0 on gfx950, so it counts them as 64 bytes.)
READ_COUNTERS = ["TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum",
                 "TCC_EA0_RDREQ_DRAM_32B_sum"]
WRITE_COUNTERS = ["TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum",
                  "TCC_EA0_WRREQ_WRITE_DRAM_32B_sum"]


def _per_dispatch(d: str):
    rows = list(csv.DictReader(open(_find(d, "counter_collection.csv"))))
    per = collections.OrderedDict()
    for r in rows:
        key = int(r["Dispatch_Id"])
        per.setdefault(key, [short_name(r["Kernel_Name"]), r.get("Grid_Size", "?"),
                             collections.defaultdict(float)])
        name = r["Counter_Name"]
        per[key][2][name] += float(r["Counter_Value"])
    return per


def read_bytes(c) -> tuple:
    total = (128.0 * c["TCC_EA0_RDREQ_128B_sum"] + 64.0 * c["TCC_EA0_RDREQ_64B_sum"] +
             32.0 * c["TCC_EA0_RDREQ_32B_sum"])
    return total, 32.0 * c["TCC_EA0_RDREQ_DRAM_32B_sum"]


def write_bytes(c) -> tuple:
    w64 = c["TCC_EA0_WRREQ_64B_sum"]
    total = 64.0 * w64 + 32.0 * (c["TCC_EA0_WRREQ_sum"] - w64)
    return total, 32.0 * c["TCC_EA0_WRREQ_WRITE_DRAM_32B_sum"]


def bytes_summary(read_dir: str, write_dir: str):
    """Per (kernel, grid): mean L2-to-memory read and write bytes per
    dispatch (all, and the part sent to the memory controller)."""
    groups = collections.OrderedDict()
    for d, fn, slot in ((read_dir, read_bytes, 0), (write_dir, write_bytes, 1)):
        for name, grid, c in _per_dispatch(d).values():
            g = groups.setdefault((name, grid), [[], []])
            g[slot].append(fn(c))
    out = ["%-58s %-10s %5s %12s %12s %5s %12s %12s" % (
        "kernel", "grid", "nrd", "read_B", "read_dram_B", "nwr", "write_B", "write_dram_B")]
    for (k, g), (rd, wr) in groups.items():
        def mean(v, i):
            return sum(x[i] for x in v) / len(v) if v else float("nan")
        out.append("%-58s %-10s %5d %12.4e %12.4e %5d %12.4e %12.4e" % (
            k, g, len(rd), mean(rd, 0), mean(rd, 1), len(wr), mean(wr, 0), mean(wr, 1)))
    return "\n".join(out)


COPY_KIB = 1048576.0  # the 1 GiB device-to-device copy bench.py runs for calibration


def _counter_means(d: str, counter: str, pattern):
    """Per (kernel, grid) whose short name matches: mean of one counter."""
    groups = collections.OrderedDict()
    for name, grid, c in _per_dispatch(d).values():
        if pattern.search(name):
            groups.setdefault((name, grid), []).append(c[counter])
    return {k: sum(v) / len(v) for k, v in groups.items()}


def copy_scale(d: str, counter: str, default: float) -> float:
    """COPY_KIB over the counter's mean reading for the 1 GiB copies of the
    run (the copy dispatches with the largest reading), else `default`."""
    vals = [c[counter] for name, grid, c in _per_dispatch(d).values()
            if name.startswith("__amd_rocclr_copyBuffer")]
    if not vals:
        return default
    top = max(vals)
    big = [v for v in vals if v > 0.9 * top]
    mean = sum(big) / len(big)
    return COPY_KIB / mean if mean > 0.25 * COPY_KIB else default


def traffic_summary(fetch_dir, write_dir, rd_dir, wr_dir, regex, form=None, src_hash=None):
    pat = re.compile(regex)
    fs = copy_scale(fetch_dir, "FETCH_SIZE", 2.0)
    ws = copy_scale(write_dir, "WRITE_SIZE", 1.0)
    fetch = _counter_means(fetch_dir, "FETCH_SIZE", pat)
    write = _counter_means(write_dir, "WRITE_SIZE", pat)
    rd = collections.OrderedDict()
    for name, grid, c in _per_dispatch(rd_dir).values():
        if pat.search(name):
            rd.setdefault((name, grid), []).append(read_bytes(c))
    wr = collections.OrderedDict()
    for name, grid, c in _per_dispatch(wr_dir).values():
        if pat.search(name):
            wr.setdefault((name, grid), []).append(write_bytes(c))

    def m(v, i):
        return sum(x[i] for x in v) / len(v)
    out = ["copy calibration: FETCH_SIZE x%.3f, WRITE_SIZE x%.3f" % (fs, ws),
           "%-58s %-10s %12s %12s %12s %12s %12s %12s" % (
               "kernel", "grid", "fetch_KiB", "write_KiB", "read_B", "read_dram_B",
               "write_B", "write_dram_B")]
    tot = [0.0] * 6
    for key in fetch:
        row = [fetch.get(key, 0.0), write.get(key, 0.0),
               m(rd[key], 0) if key in rd else 0.0, m(rd[key], 1) if key in rd else 0.0,
               m(wr[key], 0) if key in wr else 0.0, m(wr[key], 1) if key in wr else 0.0]
        tot = [a + b for a, b in zip(tot, row)]
        out.append("%-58s %-10s %12.1f %12.1f %12.4e %12.4e %12.4e %12.4e" % (
            (key[0], key[1]) + tuple(row)))
    scaled = 1024.0 * (fs * tot[0] + ws * tot[1])
    out.append("per call (sum of the rows): fetch %.1f KiB x%.3f + write %.1f KiB x%.3f = "
               "%.4e B; requests: read %.4e B (%.4e to memory), write %.4e B (%.4e to memory)"
               % (tot[0], fs, tot[1], ws, scaled, tot[2], tot[3], tot[4], tot[5]))
    if form and src_hash:
        out.append("traffic_bytes_per_launch %s %s %.4e" % (form, src_hash, scaled))
        out.append("ea_bytes_per_launch %s %s %.4e %.4e %.4e %.4e" % (
            form, src_hash, tot[2], tot[3], tot[4], tot[5]))
    return "\n".join(out)


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    if len(argv) == 3 and argv[0] == "bytes":
        print(bytes_summary(argv[1], argv[2]))
        return 0
    if len(argv) in (6, 8) and argv[0] == "traffic":
        print(traffic_summary(*argv[1:]))
        return 0
    if len(argv) != 2 or argv[0] not in ("trace", "pmc", "dispatch"):
        print(__doc__)
        return 2
    if argv[0] == "trace":
        print(trace(argv[1]))
    elif argv[0] == "pmc":
        print(pmc(argv[1]))
        extra = mfma_busy(argv[1])
        if extra:
            print(extra)
    else:
        print(dispatch(argv[1]))
    return 0


if __name__ == "__main__":
    sys.exit(main())
