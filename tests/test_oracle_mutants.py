"""The pins reject plausible mistakes: each test compiles a copy of the
oracle with one planted mistake (on the CPU) and checks that at least one
pin fails on it."""
import os
import subprocess
import sys
import tempfile

import pytest

import oracle
from tests import pins

# (name, text in oracle_sgemm.c, replacement)
MUTANTS = [
    ("swapped-transpose-index", "return trans ? (double)X[p + i * ld] : (double)X[i + p * ld];",
     "return trans ? (double)X[i + p * ld] : (double)X[p + i * ld];"),
    ("C-not-transposed", "if (t == 'T' || t == 't' || t == 'C' || t == 'c') return 1;",
     "if (t == 'T' || t == 't') return 1;\n    if (t == 'C' || t == 'c') return 0;"),
    ("ld-ignored", "return trans ? (double)X[p + i * ld] : (double)X[i + p * ld];",
     "return trans ? (double)X[p + i * ld] : (double)X[i + p * (ld - (ld > 1))];"),
    ("dropped-beta-term", "                    c += b * c0;\n                    d += fabs(b) * fabs(c0);\n                }\n                Cref",
     "                    d += fabs(b) * fabs(c0);\n                }\n                Cref"),
    ("wrong-beta-sign", "                    c += b * c0;\n                    d += fabs(b) * fabs(c0);\n                }\n                Cref",
     "                    c -= b * c0;\n                    d += fabs(b) * fabs(c0);\n                }\n                Cref"),
    ("den-without-abs", "                        sabs[i] += aabs[i] * abpj;",
     "                        sabs[i] += aabs[i] * bpj;"),
    ("last-term-dropped", "                for (int64_t p = 0; p < k; ++p) {\n                    const double bpj",
     "                for (int64_t p = 0; p + 1 < k; ++p) {\n                    const double bpj"),
    ("alpha-applied-twice", "                double c = a * s[i];", "                double c = a * a * s[i];"),
    ("transposed-B-operand", "                opB[p + j * k] = op_elem(B, ldb, tb, p, j);",
     "                opB[p + j * k] = op_elem(B, ldb, !tb, p, j);"),
    ("beta0-reads-C0", "                if (beta != 0.0f) {\n                    double c0 = (double)C0[i + j * ldc];\n                    c += b * c0;\n                    d += fabs(b) * fabs(c0);\n                }\n                Cref",
     "                if (1) {\n                    double c0 = (double)C0[i + j * ldc];\n                    c += b * c0;\n                    d += fabs(b) * fabs(c0);\n                }\n                Cref"),
    ("bf16-round-half-up", "if (dropped > 0x8000u || (dropped == 0x8000u && (kept & 1u))) kept += 1u;",
     "if (dropped >= 0x8000u) kept += 1u;"),
    ("split-keeps-two-parts", "    for (int t = 0; t < 3; ++t) {\n        uint16_t h = oracle_bf16_rne(r);",
     "    parts[2] = 0;\n    for (int t = 0; t < 2; ++t) {\n        uint16_t h = oracle_bf16_rne(r);"),
    ("method-keeps-five-products", "for (int v = 0; u + v <= 2; ++v)", "for (int v = 0; u + v <= 2 && u * v < 1; ++v)"),
    ("dgemm-sum-in-fp64", "    quad s = 0, sabs = 0;", "    double s = 0, sabs = 0;"),
    ("dgemm-swapped-transpose-index", "    return trans ? X[p + i * ld] : X[i + p * ld];",
     "    return trans ? X[i + p * ld] : X[p + i * ld];"),
    ("dgemm-dropped-beta-term", "        c += (quad)beta * c0;\n", ""),
    ("dgemm-alpha-on-den-only", "    quad c = (quad)alpha * s;", "    quad c = s;"),
    ("lu-last-pivot-on-ties", "            if (fabs(LU[i + j * n]) > best) {",
     "            if (fabs(LU[i + j * n]) >= best) {"),
    ("lu-swap-skips-L-part", "            for (int64_t c = 0; c < n; ++c) {\n                double t = LU[j + c * n];",
     "            for (int64_t c = j; c < n; ++c) {\n                double t = LU[j + c * n];"),
    ("lu-update-skips-last-row", "            for (int64_t i = j + 1; i < n; ++i) LU[i + c * n] -= LU[i + j * n] * u;",
     "            for (int64_t i = j + 1; i + 1 < n; ++i) LU[i + c * n] -= LU[i + j * n] * u;"),
]

HERE = os.path.dirname(os.path.abspath(__file__))


def _pins_hold(lib_path):
    r = subprocess.run([sys.executable, os.path.join(HERE, "_mutant_runner.py"), lib_path],
                       capture_output=True, text=True, timeout=600)
    return r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]


def test_pins_hold_on_real_oracle():
    oracle.build()
    ok, out = _pins_hold(oracle._LIB_PATH)
    assert ok, out


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(name, old, new):
    src = oracle.source_text()
    assert src.count(old) == 1, "mutation anchor not found: " + name
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "mut.so")
        oracle.build_variant(src.replace(old, new), path)
        ok, out = _pins_hold(path)
        assert not ok, "no pin caught the planted mistake " + name + "\n" + out
