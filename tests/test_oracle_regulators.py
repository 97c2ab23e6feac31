"""Pins of the oracle's polynomial-exponential regulator (paper Sec. 3.1, shape s_N):
R = k^2 exp(-sum_{i=1}^{N} (l2/k^2)^i / i).

* value: 40-digit mpmath evaluation of the defining formula;
* scale derivative k dR/dk at fixed l2: mpmath's numerical derivative in k of the same formula
  (pins the sign, the factor 2 and the 1 + sum y^i structure);
* N -> infinity: sum_i y^i/i -> -log(1 - y) for y < 1, so R -> k^2 (1 - y), the flat regulator,
  with k dR/dk -> 2 k^2 -- both reached by the oracle at N = 64 within the truncated tail.
"""
import math

import mpmath as mp
import pytest

import oracle


def _R_mp(l2, k, n):
    y = mp.mpf(l2) / (mp.mpf(k) ** 2)
    return mp.mpf(k) ** 2 * mp.exp(-mp.fsum(y ** i / i for i in range(1, n + 1)))


@pytest.mark.parametrize("n", [1, 3, 8, 16])
@pytest.mark.parametrize("l2,k", [(0.0, 1.0), (1e-4, 1.0), (0.3, 1.0), (0.9, 1.3), (2.0, 0.7),
                                  (5.0, 2.0), (1.5, 1.0)])
def test_poly_exp_value_and_scale_derivative(n, l2, k):
    mp.mp.dps = 40
    kind = oracle.reg_polyexp(n)
    ref = _R_mp(l2, k, n)
    got = oracle.regulator(l2, k, kind)
    # the rounding of y = l2/k^2 enters exp(-S) amplified by y S'(y) = sum_i y^i
    y = l2 / (k * k)
    cond = 1.0 + sum(y ** i for i in range(1, n + 1))
    assert abs(got - float(ref)) <= 2.3e-16 * (cond + 3) * float(ref) + 1e-300
    dref = mp.diff(lambda kk: _R_mp(l2, kk, n), mp.mpf(k)) * k
    dgot = oracle.regulator_dot(l2, k, kind)
    assert abs(dgot - float(dref)) <= 1e-14 * cond * abs(float(dref)) + 1e-300


@pytest.mark.parametrize("y", [0.0, 0.1, 0.3, 0.5])
def test_poly_exp_approaches_flat_regulator(y):
    k = 1.7
    l2 = y * k * k
    kind = oracle.reg_polyexp(64)
    # tail of -log(1-y) beyond i = 64 bounds the difference
    tail = sum(y ** i / i for i in range(65, 400))
    flat = oracle.regulator(l2, k, oracle.REG_LITIM)
    assert abs(oracle.regulator(l2, k, kind) - flat) <= k * k * (1 - y) * (math.expm1(tail) + 4e-16)
    assert abs(oracle.regulator_dot(l2, k, kind) - 2 * k * k) <= 2 * k * k * (65 * tail + 1e-14)
