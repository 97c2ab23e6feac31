"""Pins of the oracle's mass derivative dI/dm2 (forward-mode derivative of the integrals).

* Every family, regulator and temperature: Richardson-extrapolated central differences of the
  oracle's own integral I(m2) (error O(h^4) with h = 2e-3), a quantity computed by a
  different route (no product rule), agree to 1e-9 relative.
* Flat regulator, LPA, q_max = 1: every radial node has q < k, so G = 1/(k^2 + m2) is constant
  and I = C/(k^2 + m2)^2 exactly; hence dI/dm2 = -2 I/(k^2 + m2) to rounding.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2412_13043_amd import workloads as wl


def _richardson(f, m2, h):
    d1 = (f(m2 + h) - f(m2 - h)) / (2 * h)
    d2 = (f(m2 + h / 2) - f(m2 - h / 2)) / h
    return (4 * d2 - d1) / 3


def _check(f, fd, m2, h=2e-3, tol=1e-9):
    got = fd(m2)
    ref = _richardson(f, m2, h)
    assert np.max(np.abs(got - ref) / np.abs(ref)) <= tol


@pytest.mark.parametrize("reg", [oracle.REG_EXP, oracle.reg_polyexp(8)])
def test_dm2_lpa_and_vertex_families_against_differences(reg):
    m2 = np.array([-0.3, 0.2, 1.1, 2.5])
    for d in (3, 4):
        f = lambda m: oracle.integrate(oracle.LPA, 24, 6.0, d=d, m2=m, regulator=reg)
        fd = lambda m: oracle.integrate(oracle.LPA, 24, 6.0, d=d, m2=m, regulator=reg, dm2=True)
        _check(f, fd, m2)
    p = np.array([1e-2, 0.5, 3.0, 20.0])
    Z = wl.dressing_table(3)
    f = lambda m: oracle.integrate(oracle.TWO_POINT, 12, 10.0, n_x=6, ext=p, m2=m, Z=Z,
                                   regulator=reg)
    fd = lambda m: oracle.integrate(oracle.TWO_POINT, 12, 10.0, n_x=6, ext=p, m2=m, Z=Z,
                                    regulator=reg, dm2=True)
    _check(f, fd, m2)
    A = np.array([0.3, 1.2, 2.0, 3.1])
    f = lambda m: oracle.integrate(oracle.THREE_POINT, 8, 10.0, n_x=5, n_phi=4, ext=(p, A), m2=m,
                                   Z=Z, regulator=reg)
    fd = lambda m: oracle.integrate(oracle.THREE_POINT, 8, 10.0, n_x=5, n_phi=4, ext=(p, A),
                                    m2=m, Z=Z, regulator=reg, dm2=True)
    _check(f, fd, m2)


@pytest.mark.parametrize("stat", [oracle.BOSONIC, oracle.FERMIONIC])
def test_dm2_finite_temperature_against_differences(stat):
    m2 = np.array([-0.2, 0.4, 1.7])
    kw = dict(T=0.2, statistics=stat, freq_max=5.0, n_tail=4)
    f = lambda m: oracle.integrate_ft(oracle.LPA_T, 20, 6.0, m2=m, **kw)
    fd = lambda m: oracle.integrate_ft(oracle.LPA_T, 20, 6.0, m2=m, dm2=True, **kw)
    _check(f, fd, m2)
    p, p0 = np.array([0.1, 1.0, 5.0]), np.array([0.0, 0.7, -0.3])
    Z = wl.dressing_table(5)
    f = lambda m: oracle.integrate_ft(oracle.TWO_POINT_T, 10, 10.0, n_x=5, ext=(p, p0), m2=m,
                                      Z=Z, **kw)
    fd = lambda m: oracle.integrate_ft(oracle.TWO_POINT_T, 10, 10.0, n_x=5, ext=(p, p0), m2=m,
                                       Z=Z, dm2=True, **kw)
    _check(f, fd, m2)


@pytest.mark.parametrize("d,k", [(3, 1.0), (4, 1.7), (2, 0.6)])
def test_dm2_flat_regulator_closed_form(d, k):
    m2 = np.array([-0.5, 0.0, 0.9, 4.0]) * k * k
    I = oracle.integrate(oracle.LPA, 16, 1.0, d=d, k=k, m2=m2, regulator=oracle.REG_LITIM)
    dI = oracle.integrate(oracle.LPA, 16, 1.0, d=d, k=k, m2=m2, regulator=oracle.REG_LITIM,
                          dm2=True)
    assert np.max(np.abs(dI - (-2.0 * I / (k * k + m2))) / np.abs(dI)) <= 1e-14
