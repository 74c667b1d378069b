"""The accumulate models of tests/mfma_model.py against numpy's own FP32
arithmetic (round to nearest even) on the CPU, so the GPU rounding probe
compares the matrix cores with correct models."""
import numpy as np

from tests import mfma_model as mm


def test_round_f32_matches_numpy():
    rng = np.random.default_rng(5)
    x = rng.standard_normal(20000) * np.exp2(rng.integers(-140, 100, 20000))
    # exact ties of FP32 (a value halfway between two floats) as well
    f = rng.standard_normal(2000).astype(np.float32).astype(np.float64)
    ties = f + np.spacing(f.astype(np.float32)).astype(np.float64) / 2
    for v in np.concatenate([x, ties]):
        assert mm.to_int(float(np.float32(v))) == mm.round_f32(mm.to_int(float(v))), v


def test_seq_matches_numpy_float32_sums():
    rng = np.random.default_rng(6)
    for _ in range(300):
        c = np.float32(rng.standard_normal())
        prods = (rng.standard_normal(16) * np.exp2(rng.integers(-30, 5, 16))).astype(np.float32)
        acc = c
        for p in prods:
            acc = np.float32(acc + p)
        assert mm.to_int(float(acc)) == mm.seq(float(c), [float(p) for p in prods])


def test_models_separate_on_crafted_cases():
    one = 1.0
    half_ulps = [2.0 ** -24] * 16
    assert mm.to_float(mm.fused(one, half_ulps)) == 1.0 + 2.0 ** -20
    assert mm.to_float(mm.seq(one, half_ulps)) == 1.0
    assert mm.to_float(mm.fused(0.0, [1.0, 2.0 ** -30, -1.0])) == 2.0 ** -30
    assert mm.to_float(mm.seq(0.0, [1.0, 2.0 ** -30, -1.0])) == 0.0
    # three quarters of an ulp: nearest rounds up, a truncating adder does not
    assert mm.to_float(mm.fused(one, [2.0 ** -24, 2.0 ** -25])) == 1.0 + 2.0 ** -23
    assert mm.to_float(mm.trunc_model(0)(one, [2.0 ** -24, 2.0 ** -25])) == 1.0
    assert mm.normalized_error(1.0, one, half_ulps) == (2.0 ** -20 / (1 + 2.0 ** -20)) / 2.0 ** -24
