"""Pins of the oracle's flat-regulator threshold functions l_n^d(w) (the closed form of the LPA
integral with R = (k^2 - q^2) Theta(k^2 - q^2)):

* n = 1 against the oracle's own LPA quadrature with the flat regulator on [0, k] (q_max = 1: the
  integrand is a polynomial there, so Gauss-Legendre is exact), in several dimensions and k;
* n = 2 against the quadrature of the mass derivative, dI/dm2 = -Omega_d/(2 pi)^d k^(d-4) l_2^d;
* the derivative ladder dl_n/dw = -(n + [n == 0]) l_{n+1}, by central differences;
* l_n^d(0) = (2/d)(n + [n == 0]).
"""
import math

import numpy as np
import pytest

import oracle


def _pref(d):
    # Omega_d/(2 pi)^d with Omega_d = 2 pi^(d/2)/Gamma(d/2), the unit sphere's surface
    return 2.0 * math.pi ** (0.5 * d) / math.gamma(0.5 * d) / (2.0 * math.pi) ** d


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("k", [1.0, 1.7])
def test_threshold_is_the_flat_regulator_lpa_integral(d, k):
    m2 = np.array([-0.5, 0.0, 0.3, 2.0, 9.0]) * k * k
    I = oracle.integrate(oracle.LPA, 8, 1.0, d=d, k=k, m2=m2, regulator=oracle.REG_LITIM)
    ref = _pref(d) * k ** (d - 2) * oracle.litim_threshold(d, 1, m2 / (k * k))
    assert np.allclose(I, ref, rtol=2e-14, atol=0.0)
    dI = oracle.integrate(oracle.LPA, 8, 1.0, d=d, k=k, m2=m2, regulator=oracle.REG_LITIM,
                          dm2=True)
    dref = -_pref(d) * k ** (d - 4) * oracle.litim_threshold(d, 2, m2 / (k * k))
    assert np.allclose(dI, dref, rtol=2e-14, atol=0.0)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 5])
def test_threshold_derivative_ladder(n):
    w = np.array([-0.6, 0.0, 0.4, 3.0])
    h = 1e-5
    fd = (oracle.litim_threshold(3, n, w + h) - oracle.litim_threshold(3, n, w - h)) / (2 * h)
    ref = -(n if n > 0 else 1) * oracle.litim_threshold(3, n + 1, w)
    assert np.allclose(fd, ref, rtol=1e-8, atol=0.0)


@pytest.mark.parametrize("d,n", [(1, 0), (3, 0), (3, 1), (4, 2), (2, 7)])
def test_threshold_at_zero_mass(d, n):
    assert oracle.litim_threshold(d, n, 0.0)[0] == pytest.approx((2.0 / d) * (n if n else 1),
                                                                 rel=1e-15)
