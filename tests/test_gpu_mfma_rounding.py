"""How one matrix-core accumulate rounds, measured.

The bf16x3 kernels add all six part products of a K block of 16 into one
FP32 accumulator, one v_mfma_f32_32x32x16_bf16 per part pair.  Whether that
stays within the acceptance bound depends on how many roundings one such
instruction makes: one rounding of c + sum_k a_k b_k per instruction gives
at most 6 * ceil(K/16) roundings on any term's way into the result, far
fewer than the 2K the bound allows; a rounding after every product (16 per
instruction) would not.  This test runs single MFMAs of the FP32 and BF16
instructions on crafted and random operands through the probe library and
compares the results with the exact sum and with the models in
tests/mfma_model.py.

Every output of a case is the same dot product: all 32 rows of op(A) and all
32 columns of op(B) are equal, so the lane layout only decides which k a
lane holds (lanes 0-31 hold k 0..7, lanes 32-63 hold k 8..15 for the bf16
instruction; k 0 and k 1 for the FP32 one), not the result.
"""
from __future__ import annotations

import ctypes
import json
import math
import os

import numpy as np
import pytest

from tests import mfma_model as mm

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# Largest error of one v_mfma_f32_32x32x16_bf16 accumulate, in units of
# u = 2^-24 times |c| + sum_k |a_k b_k|, that the split form's accuracy
# argument allows for (measured: 2.74 over about 3000 crafted, adversarial and
# random cases).  With N = 6 * ceil(K/16) accumulates per output and the
# dropped part products (at most (2 + 2^-8) u |a||b| each), the split form's
# error is at most (1.008 * KAPPA_BF16 * N + 2.004 + 3) u times the bound's
# denominator, within 2 K u for K >= 21 and 12 <= K <= 16.
KAPPA_BF16 = 3.0


def _probe_lib():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1608_05265_amd", "libmisgemm_probe.so"))
    lib.probe_mfma_round.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                     ctypes.c_void_p]
    lib.probe_mfma_round.restype = ctypes.c_int
    return lib


def _bf16_values(rng, n, elo, ehi):
    """n random bf16-representable values: random sign, exponent in
    [elo, ehi], 8-bit significand."""
    e = rng.integers(elo, ehi + 1, n)
    m = rng.integers(0, 128, n)
    s = rng.choice([-1.0, 1.0], n)
    return (s * (128 + m) / 128.0 * np.exp2(e.astype(np.float64))).astype(np.float32)


def _f32_values(rng, n, elo, ehi):
    e = rng.integers(elo, ehi + 1, n)
    m = rng.integers(0, 1 << 23, n)
    s = rng.choice([-1.0, 1.0], n)
    return (s * ((1 << 23) + m) / float(1 << 23) * np.exp2(e.astype(np.float64))).astype(
        np.float32)


def _bf16_cases(rng):
    """(c, a[16], b[16]) triples: crafted ones, then random families."""
    cases = []
    one = np.float32(1.0)

    def vec(vals):
        v = np.zeros(16, np.float32)
        v[:len(vals)] = vals
        return v

    ones = np.ones(16, np.float32)
    # sixteen half-ulps of 1: one rounding gives 1 + 2^-20, per-step
    # rounding to nearest even leaves 1
    cases.append((one, np.full(16, 2.0 ** -12, np.float32), np.full(16, 2.0 ** -12, np.float32)))
    # 1 + 2^-30 - 1 inside the products, at several positions
    for i, j in ((0, 1), (0, 15), (7, 8), (3, 12)):
        a = np.zeros(16, np.float32)
        a[i], a[j], a[(j + 1) % 16 if (j + 1) % 16 != i else 2] = 1.0, 2.0 ** -15, -1.0
        b = np.zeros(16, np.float32)
        b[i], b[j], b[(j + 1) % 16 if (j + 1) % 16 != i else 2] = 1.0, 2.0 ** -15, 1.0
        cases.append((np.float32(0.0), a, b))
    # c tiny, products cancel exactly
    cases.append((np.float32(2.0 ** -30), vec([1.0, -1.0]), vec([1.0, 1.0])))
    # c = 1, products sum to 3/4 ulp of 1 (nearest rounds up, truncation not)
    cases.append((one, vec([2.0 ** -12, 2.0 ** -13]), vec([2.0 ** -12, 2.0 ** -12])))
    # c = 1, products sum to exactly half an ulp: tie, to even
    cases.append((one, vec([2.0 ** -12]), vec([2.0 ** -12])))
    # c = 1 + ulp, products half an ulp: tie, to even (up)
    cases.append((np.float32(1.0 + 2.0 ** -23), vec([2.0 ** -12]), vec([2.0 ** -12])))
    # large c, products far below its ulp but summing above it
    cases.append((np.float32(2.0 ** 10), np.full(16, 2.0 ** -8, np.float32),
                  np.full(16, 2.0 ** -8, np.float32)))
    # every product equal and large: exact
    cases.append((np.float32(0.0), ones * 3.0, ones * 5.0))
    # random families
    for _ in range(600):   # wide exponents, random signs
        cases.append((_f32_values(rng, 1, -30, 30)[0], _bf16_values(rng, 16, -15, 15),
                       _bf16_values(rng, 16, -15, 15)))
    for _ in range(600):   # the bf16x3 regime: large accumulator, small part products
        cases.append((_f32_values(rng, 1, 3, 6)[0], _bf16_values(rng, 16, -9, -6),
                      _bf16_values(rng, 16, -1, 1)))
    for _ in range(600):   # same sign everywhere (no cancellation)
        a = np.abs(_bf16_values(rng, 16, -4, 4))
        b = np.abs(_bf16_values(rng, 16, -4, 4))
        cases.append((abs(_f32_values(rng, 1, -2, 6)[0]), a, b))
    # adversarial for an adder that truncates aligned addends: c = 1 and
    # sixteen equal products just below 2^-23, 2^-24, ... (all their low bits
    # set), same sign
    for sh in range(23, 31):
        cases.append((one, np.full(16, 1.0 - 2.0 ** -8, np.float32),
                      np.full(16, 2.0 ** -sh, np.float32)))
        cases.append((one, np.full(16, -(1.0 - 2.0 ** -8), np.float32),
                      np.full(16, 2.0 ** -sh, np.float32)))
    for _ in range(600):   # the bf16x3 regime, same sign: accumulator ~2^4, parts ~2^-8
        a = np.abs(_bf16_values(rng, 16, -9, -6))
        b = np.abs(_bf16_values(rng, 16, -1, 1))
        cases.append((abs(_f32_values(rng, 1, 3, 6)[0]), a, b))
    for _ in range(600):   # heavy cancellation: pairs of opposite products plus small ones
        a = _bf16_values(rng, 16, -2, 2)
        b = _bf16_values(rng, 16, -2, 2)
        a[8:] = -a[:8]
        b[8:] = b[:8]
        a[rng.integers(0, 16)] *= np.float32(2.0 ** -20)
        cases.append((_f32_values(rng, 1, -40, -20)[0], a, b))
    return cases


def _f32_cases(rng):
    cases = []
    one = np.float32(1.0)
    cases.append((one, np.array([2.0 ** -12, 2.0 ** -12], np.float32),
                  np.array([2.0 ** -12, 2.0 ** -12], np.float32)))
    cases.append((np.float32(2.0 ** -30), np.array([1.0, -1.0], np.float32),
                  np.array([1.0, 1.0], np.float32)))
    cases.append((np.float32(0.0), np.array([1.0, 2.0 ** -30], np.float32),
                  np.array([1.0, 1.0], np.float32)))
    for _ in range(1500):
        cases.append((_f32_values(rng, 1, -30, 30)[0], _f32_values(rng, 2, -15, 15),
                      _f32_values(rng, 2, -15, 15)))
    for _ in range(1500):
        a = _f32_values(rng, 2, -2, 2)
        b = _f32_values(rng, 2, -2, 2)
        a[1] = -a[0] * np.float32(1.0 + 2.0 ** -22)
        b[1] = b[0]
        cases.append((_f32_values(rng, 1, -40, -10)[0], a, b))
    return cases


def _run(kind, cases):
    """One MFMA per case on the GPU; returns (results, outputs agree)."""
    import torch
    n = len(cases)
    kk = 16 if kind == 1 else 2
    per = kk // 2          # k values a lane holds
    a_lane = np.zeros((n, 64, per), np.float32)
    b_lane = np.zeros((n, 64, per), np.float32)
    for t, (c, a, b) in enumerate(cases):
        for half in range(2):
            a_lane[t, 32 * half:32 * half + 32, :] = a[per * half:per * half + per]
            b_lane[t, 32 * half:32 * half + 32, :] = b[per * half:per * half + per]
    cvals = np.array([c for c, _, _ in cases], np.float32)
    c_lane = np.repeat(cvals, 64 * 16).reshape(n, 64, 16)
    dev = torch.device("cuda:0")
    if kind == 1:
        # bf16 bit patterns: the high halves of the (exactly representable) floats
        bits = lambda x: torch.from_numpy(
            (x.view(np.uint32) >> 16).astype(np.uint16).view(np.int16).reshape(-1))
        a_t = bits(a_lane).to(dev)
        b_t = bits(b_lane).to(dev)
    else:
        a_t = torch.from_numpy(a_lane.reshape(-1)).to(dev)
        b_t = torch.from_numpy(b_lane.reshape(-1)).to(dev)
    c_t = torch.from_numpy(c_lane.reshape(-1).copy()).to(dev)
    out = torch.empty_like(c_t)
    rc = _probe_lib().probe_mfma_round(kind, a_t.data_ptr(), b_t.data_ptr(), c_t.data_ptr(),
                                       out.data_ptr(), n,
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, "probe launch failed: %d" % rc
    torch.cuda.synchronize()
    o = out.cpu().numpy().reshape(n, 64 * 16)
    agree = bool(np.all(o == o[:, :1]) or np.all((o == o[:, :1]) | (np.isnan(o))))
    return [float(x) for x in o[:, 0]], agree


def _summarize(kind, cases, results):
    prods = [[float(np.float64(x) * np.float64(y)) for x, y in zip(a, b)] for _, a, b in cases]
    flat = [(float(c), p) for (c, _, _), p in zip(cases, prods)]
    errs = [mm.normalized_error(d, c, p) for d, (c, p) in zip(results, flat)]
    match = mm.classify(results, flat)
    # signed error over |c| (in u) for the cases whose accumulator dominates
    # (|c| >= 8 * sum |p|): a rounding adder averages to ~0, a truncating one
    # shows a bias toward zero
    bias = [(mm.to_int(d) - mm.exact(c, p)) / abs(mm.to_int(c)) * 2.0 ** 24 *
            (1 if c > 0 else -1)
            for d, (c, p) in zip(results, flat)
            if c != 0 and abs(c) >= 8 * sum(abs(x) for x in p) and sum(abs(x) for x in p) > 0]
    return {"kind": "bf16 32x32x16" if kind == 1 else "fp32 32x32x2", "cases": len(cases),
            "acc_dominated_cases": len(bias),
            "acc_dominated_mean_signed_err_u": float(np.mean(bias)) if bias else None,
            "acc_dominated_max_abs_err_u": float(np.max(np.abs(bias))) if bias else None,
            "models_matched": match, "max_err_u": max(errs),
            "mean_err_u": float(np.mean(errs)),
            "crafted": [(float(c), d, mm.to_float(mm.exact(c, p)))
                        for d, (c, p) in list(zip(results, flat))[:28]]}


@pytest.mark.parametrize("kind", [1, 0], ids=["bf16", "fp32"])
def test_mfma_accumulate_rounding(kind):
    rng = np.random.default_rng(160805265 + 77 + kind)
    cases = _bf16_cases(rng) if kind == 1 else _f32_cases(rng)
    results, agree = _run(kind, cases)
    assert agree, "outputs of one case differ across lanes"
    s = _summarize(kind, cases, results)
    out_dir = os.environ.get("MISGEMM_RESULTS_DIR")
    if out_dir:  # optional copy of the summary for later reading
        os.makedirs(out_dir, exist_ok=True)
        with open(os.path.join(out_dir, "mfma_rounding_%d.json" % kind), "w") as f:
            json.dump(s, f, indent=1)
    print(json.dumps(s))
    assert math.isfinite(s["max_err_u"])
    # no bias where the accumulator dominates: the adder rounds to nearest
    # (a truncating adder would drift toward zero on same-sign data)
    assert abs(s["acc_dominated_mean_signed_err_u"]) < 0.1
    if kind == 0:
        # the FP32 instruction is a chain of fused multiply-adds in k order:
        # c, then + a_0 b_0, then + a_1 b_1, each rounded to nearest even
        assert s["models_matched"]["seq"] == s["cases"]
        assert s["max_err_u"] <= 2.0
    else:
        # the BF16 instruction does not round after every product: sixteen
        # half-ulp products of 1 survive (1 + 2^-20, not 1) ...
        c0, d0, ex0 = s["crafted"][0]
        assert d0 == ex0 == 1.0 + 2.0 ** -20
        # ... and one accumulate errs by at most KAPPA_BF16 u (|c| + sum |p|),
        # the figure the single-accumulator bound of the split form rests on
        assert s["max_err_u"] <= KAPPA_BF16
