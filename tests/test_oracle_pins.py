"""The CPU oracle against its pins (no GPU)."""
import numpy as np
import pytest

import oracle
from tests import pins


@pytest.fixture(scope="module")
def o():
    oracle.build()
    return oracle.Oracle(oracle._LIB_PATH)


@pytest.mark.parametrize("pin", pins.ALL_SGEMM_PINS, ids=lambda f: f.__name__)
def test_sgemm_pin(o, pin):
    pin(o)


@pytest.mark.parametrize("pin", pins.ALL_DGEMM_PINS, ids=lambda f: f.__name__)
def test_dgemm_pin(o, pin):
    pin(o)


@pytest.mark.parametrize("pin", pins.ALL_LU_PINS, ids=lambda f: f.__name__)
def test_lu_pin(o, pin):
    pin(o)


def test_hpl_residual_formula():
    """The residual of Table VII's footnote on a case worked by hand: A = 2 I (n = 2),
    x = (1, 1), b = (2, 2.5): ||Ax - b|| = 0.5, ||A|| = 2, ||x|| = 1,
    ||b|| = 2.5, so 0.5 / (eps * (2 + 2.5) * 2)."""
    eps = 2.0 ** -24
    r = oracle.hpl_scaled_residual(2 * np.eye(2), [1.0, 1.0], [2.0, 2.5], eps)
    assert r == 0.5 / (eps * 4.5 * 2)


def test_dgemm_bounds():
    assert oracle.tol_d(4096) == 2 * 4096 * 2.0 ** -53
    assert oracle.tol_d(2) == 5 * 2.0 ** -53
    # FP32 computation of FP64 data: the FP32 bound (times (1 + u)^2) plus
    # the input rounding of both factors
    assert oracle.tol_false_d(100) == oracle.tol(100) * (1 + 2.0 ** -22) + 2.0 ** -23 + 2.0 ** -47


def test_false_dgemm_input_rounding_term_is_attained():
    """The false dgemm bound's input-rounding term (2u + u^2) is attained:
    a one-term product whose factors 1 + u - 2^-50 both round down to 1 in
    FP32 has an exact FP32 product, so its whole error is the input
    rounding, 2u to within a factor 1 - 2^-22 (computed from the definition:
    FP32 rounding of the inputs, the FP32 product, FP64 comparison).  A
    derivation that under-counted that term (one factor's rounding, say)
    would not cover this case."""
    u = 2.0 ** -24
    a = b = 1.0 + u - 2.0 ** -50
    fa, fb = np.float32(a), np.float32(b)
    assert fa == 1.0 and fb == 1.0                      # both rounded down by almost u
    c32 = float(np.float32(fa * fb))                    # the FP32 path's product
    err = abs(c32 - a * b) / (abs(a) * abs(b))          # alpha = 1, beta = 0
    assert (1 - 2.0 ** -22) * 2 * u <= err <= 2 * u + 2.0 ** -47
    assert err > u                                      # more than one factor's rounding
    assert err <= oracle.tol_false_d(1)


def test_bf16_rne_matches_torch(o):
    pins.pin_bf16_rne_vs_torch(o)


def test_bf16x3_split_exhaustive(o):
    checked, r1, r2 = pins.pin_bf16x3_exhaustive(o)
    # every finite pattern with 2^-110 <= |x| < 0x1.fep127 (both signs)
    assert checked > 3_800_000_000


def test_bf16x3_split_digest(o):
    pins.pin_bf16x3_digest(o)


def test_bf16x3_method(o):
    pins.pin_bf16x3_method(o)


def test_tolerance_and_metric():
    assert oracle.tol(4096) == 2 * 4096 * 2.0 ** -24
    assert oracle.tol(1) == 4 * 2.0 ** -24  # k + 3 dominates at tiny k
    assert oracle.tol(0) == 3 * 2.0 ** -24
    cref = np.array([1.0, 0.0, 0.0, 2.0])
    den = np.array([1.0, 0.0, 0.0, 1.0])
    e = oracle.normalized_error(np.array([1.0 + 2 ** -20, 0.0, -0.0, np.nan]), cref, den)
    assert e[0] == 2 ** -20 and e[1] == 0 and e[2] == 0 and np.isinf(e[3])
    e = oracle.normalized_error(np.array([1.0, 1e-30, 0.0, 2.0]), cref, den)
    assert np.isinf(e[1])
