"""Models of one matrix-core accumulate d = c + sum_k a_k * b_k, evaluated
exactly on the CPU, for the rounding probe of the FP32 and BF16 MFMA
instructions (tests/test_gpu_mfma_rounding.py).

Every value is an exact integer multiple of 2^-SCALE (products of two FP32 or
two bf16 numbers are exact in FP64 and far above 2^-SCALE), so sums are exact
integer additions and each model only differs in where it rounds:

  fused        one round-to-nearest-even of the exact c + sum of products;
  seq          round after every addition, c first, products in k order;
  sum_then_acc the products summed exactly, rounded once, then added to c
               with a second rounding;
  trunc<b>     every addend truncated (toward zero) to a multiple of
               2^(E - 23 - b), E the largest addend exponent, the truncated
               addends summed exactly and the sum rounded to nearest even
               (an aligned adder that keeps b guard bits).

The probe's bound argument needs only the error statistic
|d - exact| / (|c| + sum |a_k b_k|), which `normalized_error` gives in units
of u = 2^-24.
"""
from __future__ import annotations

import math
from typing import Callable, Dict, List, Sequence

SCALE = 400
U = 2.0 ** -24


def to_int(v: float) -> int:
    """v (a finite float) as an exact integer multiple of 2^-SCALE."""
    num, den = float(v).as_integer_ratio()
    assert (1 << SCALE) % den == 0, "value below 2^-%d" % SCALE
    return num * ((1 << SCALE) // den)


def to_float(x: int) -> float:
    """An integer multiple of 2^-SCALE that is FP32-representable, as a float."""
    if x == 0:
        return 0.0
    s = -1.0 if x < 0 else 1.0
    x = abs(x)
    tz = (x & -x).bit_length() - 1
    return s * math.ldexp(x >> tz, tz - SCALE)


def round_f32(x: int, nearest: bool = True) -> int:
    """Round an exact value to FP32 (normal and subnormal range, no overflow):
    to nearest, ties to even, or toward zero."""
    if x == 0:
        return 0
    sign = -1 if x < 0 else 1
    ax = abs(x)
    e = ax.bit_length() - 1 - SCALE          # exponent of the leading bit
    ulp = max(e - 23, -149)
    shift = ulp + SCALE
    if shift <= 0:
        return x
    q, r = divmod(ax, 1 << shift)
    if nearest:
        half = 1 << (shift - 1)
        if r > half or (r == half and (q & 1)):
            q += 1
    return sign * (q << shift)


def exact(c: float, prods: Sequence[float]) -> int:
    return to_int(c) + sum(to_int(p) for p in prods)


def fused(c: float, prods: Sequence[float]) -> int:
    return round_f32(exact(c, prods))


def seq(c: float, prods: Sequence[float]) -> int:
    acc = to_int(c)
    for p in prods:
        acc = round_f32(acc + to_int(p))
    return acc


def sum_then_acc(c: float, prods: Sequence[float]) -> int:
    s = round_f32(sum(to_int(p) for p in prods))
    return round_f32(to_int(c) + s)


def trunc_model(bits: int) -> Callable[[float, Sequence[float]], int]:
    def f(c: float, prods: Sequence[float]) -> int:
        vals = [to_int(c)] + [to_int(p) for p in prods]
        nz = [abs(v) for v in vals if v != 0]
        if not nz:
            return 0
        e = max(v.bit_length() for v in nz) - 1
        step = max(e - 23 - bits, 0)
        tot = 0
        for v in vals:
            m = (abs(v) >> step) << step
            tot += m if v >= 0 else -m
        return round_f32(tot)
    f.__name__ = "trunc%d" % bits
    return f


MODELS: Dict[str, Callable[[float, Sequence[float]], int]] = {
    "fused": fused, "seq": seq, "sum_then_acc": sum_then_acc}
for _b in (0, 1, 2, 3, 4, 8, 16, 24):
    MODELS["trunc%d" % _b] = trunc_model(_b)


def normalized_error(d: float, c: float, prods: Sequence[float]) -> float:
    """|d - exact| / (|c| + sum |p|), in units of u = 2^-24 (0 when the
    denominator is 0 and d equals the exact value)."""
    ex = exact(c, prods)
    den = abs(to_int(c)) + sum(abs(to_int(p)) for p in prods)
    diff = abs(to_int(d) - ex)
    if den == 0:
        return 0.0 if diff == 0 else math.inf
    # (diff / den) / 2^-24 without losing precision on huge integers
    return (diff << 24) / den if diff < (1 << 900) else math.inf


def classify(results: List[float], cases: List[tuple]) -> Dict[str, int]:
    """For every model, how many of the cases it reproduces bit for bit."""
    out = {}
    for name, f in MODELS.items():
        out[name] = sum(1 for d, (c, prods) in zip(results, cases) if to_int(d) == f(c, prods))
    return out
