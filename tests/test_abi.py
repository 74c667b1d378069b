"""The C-ABI library on the CPU: it loads, exports every entry point the
header declares, validates arguments before touching a device, and parses
tuning tables."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "misgemm.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(misgemm_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def mg():
    import paper_1608_05265_amd as mg
    if not os.path.exists(mg.library_path()):
        from paper_1608_05265_amd import build
        build.build()
    return mg


def test_every_declared_symbol_is_exported(mg):
    names = header_functions()
    assert len(names) >= 13
    lib = ctypes.CDLL(mg.library_path())
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", mg.library_path()], capture_output=True,
                         text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    assert set(names) <= exported


def test_configs_and_strings(mg):
    n = mg.num_configs()
    assert n >= 8
    names = set()
    for c in mg.configs():
        assert c["mode"] in (0, 1)
        assert c["bm"] % 16 == 0 and c["bn"] % 16 == 0 and c["threads"] % 64 == 0
        assert 0 < c["lds_bytes"] <= 160 * 1024
        names.add(c["name"])
    assert len(names) == n
    assert mg.status_string(0) == "success"
    assert "position 8" in mg.status_string(-8)
    assert "tuning" in mg.status_string(1003)
    assert "gfx950" in mg.version()
    # split-K variants exist for the small tiles of both forms, not the 256x256 ones
    for mode in (0, 1):
        split = [c for c in mg.configs(mode) if c["splitk"]]
        assert split and all(c["bm"] * c["bn"] <= 128 * 128 and not c["packed"] for c in split)


@pytest.mark.parametrize("case,expected", [
    (dict(transa="X"), -1), (dict(transb="q"), -2), (dict(m=-1), -3), (dict(n=-1), -4),
    (dict(k=-1), -5), (dict(lda=3), -8), (dict(ldb=3), -10), (dict(ldc=3), -13),
    (dict(mode=7), -14), (dict(A=None), -7), (dict(B=None), -9), (dict(C=None), -12),
    (dict(transa="T", lda=4), -8), (dict(transb="T", ldb=4), -10),
])
def test_argument_errors_before_any_launch(mg, case, expected):
    """Invalid arguments are rejected with the BLAS position code; no device
    is needed for that (the check precedes every HIP call)."""
    args = dict(transa="N", transb="N", m=8, n=6, k=5, alpha=1.0, A=0x1000, lda=8, B=0x2000,
                ldb=5, beta=0.0, C=0x3000, ldc=8, mode=0)
    args.update(case)
    lib = mg._load()
    rc = lib.misgemm_sgemm(args["transa"].encode(), args["transb"].encode(), args["m"], args["n"],
                           args["k"], args["alpha"], args["A"], args["lda"], args["B"],
                           args["ldb"], args["beta"], args["C"], args["ldc"], args["mode"], None)
    assert rc == expected


def test_quick_returns_need_no_device(mg):
    lib = mg._load()
    # m == 0, n == 0, and (alpha == 0 or k == 0) with beta == 1 return before any HIP call
    assert lib.misgemm_sgemm(b"N", b"N", 0, 5, 5, 1.0, None, 1, None, 5, 0.0, None, 1, 0, None) == 0
    assert lib.misgemm_sgemm(b"N", b"N", 5, 0, 5, 1.0, None, 5, None, 5, 0.0, None, 5, 0, None) == 0
    assert lib.misgemm_sgemm(b"N", b"N", 5, 5, 5, 0.0, None, 5, None, 5, 1.0, 0x10, 5, 1, None) == 0
    assert lib.misgemm_sgemm(b"T", b"T", 5, 5, 0, 2.0, None, 1, None, 5, 1.0, 0x10, 5, 0, None) == 0
    assert lib.misgemm_sgemm_config(b"N", b"N", 5, 5, 5, 1.0, 0x10, 5, 0x10, 5, 0.0, 0x10, 5, 0,
                                    999, 0, None) == -15
    assert lib.misgemm_sgemm_config(b"N", b"N", 5, 5, 5, 1.0, 0x10, 5, 0x10, 5, 0.0, 0x10, 5, 0,
                                    0, -1, None) == -16
    # split-K factor and tile order are checked before any HIP call
    for splits in (0, -1, 65):
        assert lib.misgemm_sgemm_split(b"N", b"N", 5, 5, 5, 1.0, 0x10, 5, 0x10, 5, 0.0, 0x10, 5,
                                       0, -1, 0, splits, None) == -17
    assert lib.misgemm_sgemm_split(b"N", b"N", 5, 5, 5, 1.0, 0x10, 5, 0x10, 5, 0.0, 0x10, 5, 0,
                                   -1, -1, 2, None) == -16
    assert lib.misgemm_sgemm_split(b"N", b"N", 0, 5, 5, 1.0, None, 1, None, 5, 0.0, None, 1, 0,
                                   -1, 0, 4, None) == 0
    # dgemm: the same argument positions, checked before any HIP call
    dargs = [b"N", b"N", 8, 6, 5, 1.0, 0x1000, 8, 0x2000, 5, 0.0, 0x3000, 8]
    for pos, val, code in [(0, b"X", -1), (1, b"Q", -2), (2, -1, -3), (3, -1, -4),
                           (4, -1, -5), (7, 3, -8), (9, 3, -10), (12, 3, -13)]:
        a = list(dargs)
        a[pos] = val
        assert lib.misgemm_dgemm(*a, 0, None) == code
    assert lib.misgemm_dgemm(*dargs, 7, None) == -14
    assert lib.misgemm_dgemm(b"N", b"N", 0, 5, 5, 1.0, None, 1, None, 5, 0.0, None, 1, 0,
                             None) == 0
    # LU and solve: argument positions checked before any launch
    assert lib.misgemm_sgetrf(-1, None, 1, None, None, 0, None) == -1
    assert lib.misgemm_sgetrf(4, None, 4, 0x2000, 0x3000, 0, None) == -2
    assert lib.misgemm_sgetrf(4, 0x1000, 3, 0x2000, 0x3000, 0, None) == -3
    assert lib.misgemm_sgetrf(4, 0x1000, 4, None, 0x3000, 0, None) == -4
    assert lib.misgemm_sgetrf(4, 0x1000, 4, 0x2000, None, 0, None) == -5
    assert lib.misgemm_sgetrf(4, 0x1000, 4, 0x2000, 0x3000, 9, None) == -6
    assert lib.misgemm_sgetrs(4, -1, 0x1000, 4, 0x2000, 0x3000, 4, 0, None) == -2
    assert lib.misgemm_sgetrs(4, 1, 0x1000, 4, 0x2000, 0x3000, 3, 0, None) == -7
    assert lib.misgemm_sgetrs(4, 1, 0x1000, 4, 0x2000, 0x3000, 4, 5, None) == -8
    assert lib.misgemm_sgetrs(0, 1, None, 1, None, None, 1, 0, None) == 0
    assert lib.misgemm_bf16x3_split(None, 0, None, None) == 0
    assert lib.misgemm_bf16x3_split(None, 3, None, None) == -1
    assert lib.misgemm_batch_launch(None, None) == 1005


def test_tuning_table_parsing(mg, tmp_path):
    cfgs = mg.configs()
    f32 = [c for c in cfgs if c["mode"] == 0]
    x3 = [c for c in cfgs if c["mode"] == 1 and not c["packed"]]
    x3p = [c for c in cfgs if c["mode"] == 1 and c["packed"]]
    good = tmp_path / "good.txt"
    good.write_text("misgemm-tuning 1\n# comment\n0 N T 4096 4096 4096 %s 4\n"
                    "1 T N 1000 2000 300 %s\n" % (f32[-1]["name"], x3[-1]["name"]))
    mg.load_tuning(str(good))
    assert mg.select_config("N", "T", 4096, 4096, 4096, 0) == f32[-1]["id"]
    split = [c for c in f32 if c["splitk"]][0]
    nosplit = [c for c in f32 if not c["splitk"]][0]
    withsplit = tmp_path / "split.txt"
    withsplit.write_text("misgemm-tuning 1\n0 N N 1024 1024 1024 %s 8 4\n"
                         "0 T N 1024 1024 1024 %s 8 1\n" % (split["name"], nosplit["name"]))
    mg.load_tuning(str(withsplit))
    assert mg.select_config("N", "N", 1024, 1024, 1024, 0) == split["id"]
    mg.load_tuning(str(good))
    assert mg.select_config("N", "T", 3000, 5000, 2500, 0) == f32[-1]["id"]   # within 2x
    rule = tmp_path / "rule.txt"
    rule.write_text("misgemm-tuning 1\nbatch2 0 256 fp32p_128x128x16_w64x64 "
                    "fp32_64x64x16_w32x32\nbatch2 1 192 x3p_128x128x16_w64x64 "
                    "x3_64x64x32_w32x32\n")
    mg.load_tuning(str(rule))
    mg.load_tuning(str(good))
    assert mg.select_config("t", "n", 1000, 2000, 300, 1) == x3[-1]["id"]
    # a packed winner listed first is passed over by misgemm_sgemm's choice,
    # which takes the key's non-packed entry
    both = tmp_path / "both.txt"
    both.write_text("misgemm-tuning 1\n1 T N 1000 2000 300 %s\n1 T N 1000 2000 300 %s\n"
                    % (x3p[0]["name"], x3[0]["name"]))
    mg.load_tuning(str(both))
    assert mg.select_config("T", "N", 1000, 2000, 300, 1) == x3[0]["id"]
    mg.load_tuning(str(good))
    bad_cases = ["nonsense\n", "misgemm-tuning 1\n0 N N 1 1 1 no_such_config\n",
                 "misgemm-tuning 1\n1 N N 64 64 64 %s\n" % f32[0]["name"],  # mode mismatch
                 "misgemm-tuning 1\n0 Q N 64 64 64 %s\n" % f32[0]["name"],
                 "misgemm-tuning 1\n0 N N 0 64 64 %s\n" % f32[0]["name"],
                 "misgemm-tuning 1\nbatch 0 %s\n" % f32[0]["name"],  # no persistent variant
                 "misgemm-tuning 1\n0 N N 64 64 64 %s 8 2\n" % nosplit["name"],  # no split-K
                 "misgemm-tuning 1\n0 N N 64 64 64 %s 8 65\n" % split["name"],
                 # two-part batch rules: no persistent variant, bad threshold,
                 # mode mismatch, missing field
                 "misgemm-tuning 1\nbatch2 0 256 %s fp32_64x64x16_w32x32\n" % f32[0]["name"],
                 "misgemm-tuning 1\nbatch2 0 0 fp32p_128x128x16_w64x64 fp32_64x64x16_w32x32\n",
                 "misgemm-tuning 1\nbatch2 1 256 fp32p_128x128x16_w64x64 fp32_64x64x16_w32x32\n",
                 "misgemm-tuning 1\nbatch2 0 256 fp32p_128x128x16_w64x64\n"]
    for i, text in enumerate(bad_cases):
        p = tmp_path / ("bad%d.txt" % i)
        p.write_text(text)
        with pytest.raises(mg.MisgemmError) as ei:
            mg.load_tuning(str(p))
        assert ei.value.status == 1003
    # a failed load keeps the previous table
    assert mg.select_config("N", "T", 4096, 4096, 4096, 0) == f32[-1]["id"]
    with pytest.raises(mg.MisgemmError):
        mg.load_tuning(str(tmp_path / "missing.txt"))
    mg.load_tuning(None)
    assert mg.select_config("N", "T", 4096, 4096, 4096, 0) != -1
    # restore the packaged table, if any, for later tests
    if os.path.exists(mg.TUNING_PATH):
        mg.load_tuning(mg.TUNING_PATH)


def test_workspace_size_and_ws_argument_checks(mg):
    lib = mg._load()
    # FP32 needs no workspace; bf16x3 needs 6 bytes per padded (row, k) pair
    assert mg.workspace_size("N", "N", 1000, 1000, 1000, 0) == 0
    w = mg.workspace_size("N", "T", 1000, 300, 100, 1)
    kpad, mpad, npad = 112, 1024, 512
    assert w == 6 * kpad * (mpad + npad) + 512
    assert lib.misgemm_workspace_size(b"X", b"N", 1, 1, 1, 1) == -1
    assert lib.misgemm_workspace_size(b"N", b"N", 1, 1, 1, 5) == -6
    # short or misaligned caller workspace is rejected before any HIP call
    assert lib.misgemm_sgemm_ws(b"N", b"N", 1000, 300, 100, 1.0, 0x1000, 1000, 0x2000, 100, 0.0,
                                0x3000, 1000, 1, 0x4000, w - 1, None) == -16
    assert lib.misgemm_sgemm_ws(b"N", b"N", 1000, 300, 100, 1.0, 0x1000, 1000, 0x2000, 100, 0.0,
                                0x3000, 1000, 1, 0x4004, w, None) == -15
    assert lib.misgemm_sgemm_ws(b"N", b"N", 1000, 300, 100, 1.0, 0x1000, 999, 0x2000, 100, 0.0,
                                0x3000, 1000, 1, 0x4000, w, None) == -8
    assert any(c["packed"] for c in mg.configs(1))
    assert not any(c["packed"] for c in mg.configs(0))


def test_header_is_plain_c(tmp_path):
    """include/misgemm.h is a C header: a C99 translation unit that includes
    it and names every entry point compiles without warnings (no HIP or
    C++ types in the signatures)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    names = header_functions() + ["sgemm_", "dgemm_"]
    src = tmp_path / "use.c"
    src.write_text('#include "misgemm.h"\nvoid *entry_points[] = {%s};\n'
                   % ", ".join("(void *)&%s" % n for n in names))
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-fsyntax-only",
                        "-I" + inc, str(src)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
