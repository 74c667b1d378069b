"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only): a copy of oracle_sgemm.c built with
-fsanitize=address,undefined runs the oracle pins (all but the one that
compares with torch's conversion) in a child process with the ASan runtime
preloaded; an out-of-bounds access, a use after free or undefined behaviour
in the oracle's loops aborts the child and fails the test."""
import os
import shutil
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

RUNNER = r"""
import sys
sys.path.insert(0, %r)
import oracle
from tests import pins
o = oracle.Oracle(sys.argv[1])
for pin in pins.ALL_SGEMM_PINS + pins.ALL_DGEMM_PINS + pins.ALL_LU_PINS + [
        lambda o: pins.pin_bf16x3_exhaustive(o, 0x3F800000, 0x3F800000 + (1 << 20)),
        pins.pin_bf16x3_method]:
    pin(o)
print("pins held under the sanitizers")
"""


def test_oracle_pins_under_address_sanitizer(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    libasan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True,
                             text=True).stdout.strip()
    if not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("no ASan runtime")
    lib = str(tmp_path / "liboracle_asan.so")
    subprocess.run([gcc, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fopenmp", "-ffp-contract=off", "-fPIC",
                    "-shared", "-o", lib, oracle._SRC, "-lm"], check=True)
    env = dict(os.environ, LD_PRELOAD=libasan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-c", RUNNER % ROOT, lib], env=env, capture_output=True,
                       text=True, timeout=900)
    out = r.stdout[-3000:] + r.stderr[-3000:]
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, out
    assert "pins held" in r.stdout
