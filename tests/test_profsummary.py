"""The counter arithmetic behind the committed traffic figures (profsummary):
FETCH_SIZE and WRITE_SIZE scaled by their readings for the 1 GiB copy,
request bytes by size (128/64/32-byte reads, 64/32-byte writes), means over
the dispatches of each kernel the pattern names, the sum over the kernels of
a call, and the two lines bench.py reads back, checked against hand-computed
values on synthetic counter files; the kernel-name shortening of the
template names the summaries print."""
import csv
import os

import pytest

import bench
from paper_1608_05265_amd import profsummary as ps

FIELDS = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
COPY = "__amd_rocclr_copyBuffer"
PACK = "void misgemm::pack_x3_kernel<true>(misgemm::PackArgs)"
TILE = ("void misgemm::packed_kernel<misgemm::Shape<128, 128, 16, 64, 64, 1> >"
        "(misgemm::PackedArgs, long, long, int)")
OTHER = "void at::native::elementwise_kernel<128, 4>(int)"


def _write(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for disp, (name, counters) in enumerate(rows, 1):
            for cname, val in counters.items():
                w.writerow({"Dispatch_Id": disp, "Kernel_Name": name, "Grid_Size": 4096,
                            "Counter_Name": cname, "Counter_Value": val})


@pytest.fixture
def runs(tmp_path):
    """Four counter runs of the same program: a 1 GiB copy (read half by
    FETCH_SIZE, as on gfx950), two dispatches each of a pack and a tile
    kernel, and an unrelated kernel the pattern must leave out."""
    kib = 1048576.0
    fetch = [(COPY, {"FETCH_SIZE": kib / 2}), (PACK, {"FETCH_SIZE": 100.0}),
             (PACK, {"FETCH_SIZE": 300.0}), (TILE, {"FETCH_SIZE": 1000.0}),
             (TILE, {"FETCH_SIZE": 3000.0}), (OTHER, {"FETCH_SIZE": 7.0e6})]
    write = [(COPY, {"WRITE_SIZE": kib}), (PACK, {"WRITE_SIZE": 50.0}),
             (PACK, {"WRITE_SIZE": 50.0}), (TILE, {"WRITE_SIZE": 10.0}),
             (TILE, {"WRITE_SIZE": 30.0}), (OTHER, {"WRITE_SIZE": 9.0e6})]
    rd = {"TCC_EA0_RDREQ_32B_sum": 1.0, "TCC_EA0_RDREQ_64B_sum": 2.0,
          "TCC_EA0_RDREQ_128B_sum": 3.0, "TCC_EA0_RDREQ_DRAM_32B_sum": 17.0}
    wr = {"TCC_EA0_WRREQ_sum": 10.0, "TCC_EA0_WRREQ_64B_sum": 4.0,
          "TCC_EA0_WRREQ_WRITE_DRAM_32B_sum": 14.0, "TCC_BUBBLE_sum": 0.0}
    rds = [(n, dict(rd)) for n in (PACK, TILE, TILE)] + [(OTHER, {k: 1e9 for k in rd})]
    wrs = [(n, dict(wr)) for n in (PACK, TILE, TILE)] + [(OTHER, {k: 1e9 for k in wr})]
    dirs = {}
    for name, rows in (("fetch", fetch), ("write", write), ("rd", rds), ("wr", wrs)):
        dirs[name] = str(tmp_path / name)
        _write(dirs[name], rows)
    return dirs


def test_short_names():
    assert ps.short_name(PACK) == "pack_x3_kernel<true>"
    assert ps.short_name(TILE) == "packed_kernel<128x128x16x64x64x1>"
    assert ps.short_name(OTHER) == OTHER[:60]


def test_copy_calibration(runs):
    assert ps.copy_scale(runs["fetch"], "FETCH_SIZE", 9.0) == 2.0
    assert ps.copy_scale(runs["write"], "WRITE_SIZE", 9.0) == 1.0


def test_request_bytes_by_size():
    c = {"TCC_EA0_RDREQ_32B_sum": 1.0, "TCC_EA0_RDREQ_64B_sum": 2.0,
         "TCC_EA0_RDREQ_128B_sum": 3.0, "TCC_EA0_RDREQ_DRAM_32B_sum": 17.0}
    assert ps.read_bytes(c) == (32.0 + 128.0 + 384.0, 544.0)
    w = {"TCC_EA0_WRREQ_sum": 10.0, "TCC_EA0_WRREQ_64B_sum": 4.0,
         "TCC_EA0_WRREQ_WRITE_DRAM_32B_sum": 14.0}
    assert ps.write_bytes(w) == (64.0 * 4 + 32.0 * 6, 448.0)


def test_traffic_lines_sum_the_named_kernels(runs, tmp_path, monkeypatch):
    out = ps.traffic_summary(runs["fetch"], runs["write"], runs["rd"], runs["wr"],
                             r"pack_x3|packed_kernel", "bf16x3", "0123456789abcdef")
    # per-dispatch means: pack fetch 200 KiB, write 50 KiB; tile fetch 2000
    # KiB, write 20 KiB; FETCH_SIZE x2, WRITE_SIZE x1, per call the sum
    traffic = 1024.0 * (2.0 * (200.0 + 2000.0) + (50.0 + 20.0))
    read, read_mem = 2 * 544.0, 2 * 544.0  # one mean per kernel: 544 B, 17 x 32 B
    write, write_mem = 2 * 448.0, 2 * 448.0
    lines = [ln for ln in out.splitlines() if ln.startswith(("traffic_bytes", "ea_bytes"))]
    assert lines == [
        "traffic_bytes_per_launch bf16x3 0123456789abcdef %.4e" % traffic,
        "ea_bytes_per_launch bf16x3 0123456789abcdef %.4e %.4e %.4e %.4e"
        % (read, read_mem, write, write_mem)]
    # bench.py reads them back while the source hash matches
    f = tmp_path / "summary.txt"
    f.write_text("\n".join(lines) + "\n")
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: "0123456789abcdef")
    assert bench.measured_traffic("bf16x3", str(f)) == pytest.approx(traffic, rel=1e-4)
    got = bench.measured_bytes("bf16x3", str(f))
    assert got["read"] == pytest.approx(read, rel=1e-4)
    assert got["write_to_memory"] == pytest.approx(write_mem, rel=1e-4)


def test_mfma_busy_fraction(tmp_path):
    """busy / (1024 SIMDs x GRBM_GUI_ACTIVE / 8 XCDs): the busy counter sums
    every SIMD's cycles, GRBM_GUI_ACTIVE the eight XCDs' active cycles."""
    grbm = 8.0e6  # 1e6 cycles per XCD
    rows = [(TILE, {"SQ_VALU_MFMA_BUSY_CYCLES": 0.75 * 1024 * 1.0e6, "GRBM_GUI_ACTIVE": grbm}),
            (TILE, {"SQ_VALU_MFMA_BUSY_CYCLES": 0.25 * 1024 * 1.0e6, "GRBM_GUI_ACTIVE": grbm}),
            (COPY, {"SQ_VALU_MFMA_BUSY_CYCLES": 0.0, "GRBM_GUI_ACTIVE": grbm})]
    _write(str(tmp_path / "mfma"), rows)
    out = ps.mfma_busy(str(tmp_path / "mfma")).splitlines()
    assert len(out) == 1 and out[0].startswith("packed_kernel<128x128x16x64x64x1>")
    assert out[0].split()[-1] == "0.500" and out[0].split()[-2] == "2"
