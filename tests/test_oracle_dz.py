"""Pins of the oracle's derivatives of the two-point integral in its dressing-table entries,
dI_e/dZ_i (the forward-mode derivatives an implicit stepper of a dressing flow needs; paper
Sec. 5.2 and App. F), against routes that do not use the derivative code:

* central finite differences of the (separately pinned) integral in each table entry, for every
  regulator, with momenta that put nodes in the clamped regions below and above the table;
* the row sums: shifting every entry by c shifts Z(l2) by c, so sum_i dI/dZ_i is the derivative
  in c, taken by finite differences;
* a one-entry table (Z(l2) = Z_0 everywhere);
* the entries no node reaches are exactly 0, and the others are not: the reached cells come
  from the node momenta directly (brute force over the GL nodes).
"""
import math

import numpy as np
import pytest

import oracle

N_Q, N_X, Q_MAX = 9, 7, 10.0
XMIN, XMAX = 0.05, 20.0


def _I(Z, p, m2, reg, n_q=N_Q, n_x=N_X):
    return oracle.integrate(oracle.TWO_POINT, n_q, Q_MAX, n_x=n_x, ext=p, m2=m2, Z=Z,
                            x_min=XMIN, x_max=XMAX, regulator=reg)


def _J(Z, p, m2, reg, n_q=N_Q, n_x=N_X):
    return oracle.integrate_dz(n_q, Q_MAX, n_x=n_x, ext=p, m2=m2, Z=Z, x_min=XMIN, x_max=XMAX,
                               regulator=reg)


def _case(seed, nZ=9, n=6):
    rng = np.random.default_rng(seed)
    Z = rng.uniform(0.8, 1.4, nZ)
    p = np.concatenate([[1e-3, 40.0], 10 ** rng.uniform(-1.5, 1.2, n - 2)])
    m2 = rng.uniform(0.2, 1.5, n)
    return Z, p, m2


@pytest.mark.parametrize("reg", [oracle.REG_EXP, oracle.reg_polyexp(8), oracle.REG_LITIM])
def test_dz_matches_central_differences(reg):
    Z, p, m2 = _case(1)
    J = _J(Z, p, m2, reg)
    h = 1e-5
    for i in range(Z.size):
        Zp, Zm = Z.copy(), Z.copy()
        Zp[i] += h
        Zm[i] -= h
        fd = (_I(Zp, p, m2, reg) - _I(Zm, p, m2, reg)) / (2 * h)
        # O(h^2) truncation and eps * I / h rounding, relative to the row's scale
        scale = np.max(np.abs(J), axis=1)
        assert np.all(np.abs(fd - J[:, i]) <= 1e-7 * scale + 1e-18), i


def test_dz_row_sums_are_the_shift_derivative():
    Z, p, m2 = _case(2, nZ=13)
    J = _J(Z, p, m2, oracle.REG_EXP)
    h = 1e-5
    fd = (_I(Z + h, p, m2, oracle.REG_EXP) - _I(Z - h, p, m2, oracle.REG_EXP)) / (2 * h)
    assert np.allclose(J.sum(axis=1), fd, rtol=1e-8, atol=0.0)


def test_dz_one_entry_table():
    _, p, m2 = _case(3)
    Z = np.array([1.2])
    J = _J(Z, p, m2, oracle.REG_EXP)
    assert J.shape == (p.size, 1)
    h = 1e-5
    fd = (_I(Z + h, p, m2, oracle.REG_EXP) - _I(Z - h, p, m2, oracle.REG_EXP)) / (2 * h)
    assert np.allclose(J[:, 0], fd, rtol=1e-8, atol=0.0)
    # every propagator depends on Z_0 with dG/dZ = -G^2 l2 < 0
    assert np.all(J < 0)


def test_dz_zero_exactly_where_no_node_reaches():
    nZ = 40
    Z = 1.0 + 0.01 * np.arange(nZ)
    p = np.array([0.3, 2.5])
    m2 = np.array([0.5, 0.9])
    xmin, xmax = 1e-3, 1e4  # the table reaches far beyond every |l|
    J = oracle.integrate_dz(N_Q, Q_MAX, n_x=N_X, ext=p, m2=m2, Z=Z, x_min=xmin, x_max=xmax)
    q, _ = oracle.gauss_legendre(N_Q, 0.0, Q_MAX)
    x, _ = oracle.gauss_legendre(N_X, -1.0, 1.0)
    delta = (math.log(xmax) - math.log(xmin)) / (nZ - 1)
    for e in range(p.size):
        reached = set()
        for qa in q:
            l2s = [qa * qa] + [qa * qa + p[e] ** 2 + 2 * qa * p[e] * xb for xb in x]
            for l2 in l2s:
                s = min(max((0.5 * math.log(l2) - math.log(xmin)) / delta, 0.0), nZ - 1)
                i = min(int(math.floor(s)), nZ - 2)
                reached.update({i, i + 1} if s > i else {i})
        for i in range(nZ):
            if i in reached:
                assert J[e, i] < 0, (e, i)
            else:
                assert J[e, i] == 0.0, (e, i)


@pytest.mark.parametrize("stat,scaled", [(oracle.BOSONIC, False), (oracle.FERMIONIC, True)])
def test_dz_finite_temperature_matches_central_differences(stat, scaled):
    # the finite-temperature two-point integral (Matsubara sum with tails), each table entry
    Z, p, m2 = _case(4, nZ=8, n=5)
    rng = np.random.default_rng(5)
    p0 = rng.uniform(-1.0, 1.0, p.size)
    ft = dict(T=0.2, freq_max=3.0, statistics=stat, n_tail=3, freq_scaled=scaled)

    def I(Zv):
        return oracle.integrate_ft(oracle.TWO_POINT_T, 8, Q_MAX, n_x=6, ext=(p, p0), m2=m2,
                                   Z=Zv, x_min=XMIN, x_max=XMAX, **ft)

    J = oracle.integrate_ft_dz(8, Q_MAX, n_x=6, ext=(p, p0), m2=m2, Z=Z, x_min=XMIN,
                               x_max=XMAX, **ft)
    h = 1e-5
    scale = np.max(np.abs(J), axis=1)
    for i in range(Z.size):
        Zp, Zm = Z.copy(), Z.copy()
        Zp[i] += h
        Zm[i] -= h
        fd = (I(Zp) - I(Zm)) / (2 * h)
        assert np.all(np.abs(fd - J[:, i]) <= 1e-7 * scale + 1e-18), i
    fd = (I(Z + h) - I(Z - h)) / (2 * h)
    assert np.allclose(J.sum(axis=1), fd, rtol=1e-8, atol=0.0)


@pytest.mark.parametrize("reg", [oracle.REG_EXP, oracle.reg_polyexp(8), oracle.REG_LITIM])
def test_dz_three_point_matches_central_differences(reg):
    # the three-point integral: radial leg, the first inner leg (cos1 only) and the second
    # (cos1 and phi); angles spanning [0, pi]
    Z, p, m2 = _case(6, nZ=8, n=5)
    alpha = np.array([0.0, 0.4, 1.5, 2.6, math.pi])
    kw = dict(n_x=5, n_phi=4, x_min=XMIN, x_max=XMAX, regulator=reg)

    def I(Zv):
        return oracle.integrate(oracle.THREE_POINT, 6, Q_MAX, ext=(p, alpha), m2=m2, Z=Zv, **kw)

    J = oracle.integrate_dz_three(6, Q_MAX, ext=(p, alpha), m2=m2, Z=Z, **kw)
    h = 1e-5
    scale = np.max(np.abs(J), axis=1)
    for i in range(Z.size):
        Zp, Zm = Z.copy(), Z.copy()
        Zp[i] += h
        Zm[i] -= h
        fd = (I(Zp) - I(Zm)) / (2 * h)
        assert np.all(np.abs(fd - J[:, i]) <= 1e-7 * scale + 1e-18), i
    fd = (I(Z + h) - I(Z - h)) / (2 * h)
    assert np.allclose(J.sum(axis=1), fd, rtol=1e-8, atol=0.0)


@pytest.mark.parametrize("stat,reg", [(oracle.BOSONIC, oracle.REG_EXP),
                                      (oracle.FERMIONIC, oracle.reg_polyexp(8)),
                                      (oracle.BOSONIC, oracle.REG_LITIM)])
def test_dz_three_point_finite_temperature_matches_central_differences(stat, reg):
    # the finite-temperature three-point integral: radial leg and both inner legs, each with
    # its own frequency shift
    Z, p, m2 = _case(7, nZ=8, n=5)
    alpha = np.array([0.0, 0.4, 1.5, 2.6, math.pi])
    rng = np.random.default_rng(8)
    p01, p02 = rng.uniform(-1.0, 1.0, p.size), rng.uniform(-1.0, 1.0, p.size)
    kw = dict(n_x=5, n_phi=4, T=0.25, freq_max=3.0, statistics=stat, n_tail=2, x_min=XMIN,
              x_max=XMAX, regulator=reg)

    def I(Zv):
        return oracle.integrate_ft(oracle.THREE_POINT_T, 6, Q_MAX, ext=(p, alpha, p01, p02),
                                   m2=m2, Z=Zv, **kw)

    J = oracle.integrate_ft_three_dz(6, Q_MAX, ext=(p, alpha, p01, p02), m2=m2, Z=Z, **kw)
    h = 1e-5
    scale = np.max(np.abs(J), axis=1)
    for i in range(Z.size):
        Zp, Zm = Z.copy(), Z.copy()
        Zp[i] += h
        Zm[i] -= h
        fd = (I(Zp) - I(Zm)) / (2 * h)
        assert np.all(np.abs(fd - J[:, i]) <= 1e-7 * scale + 1e-18), i
    fd = (I(Z + h) - I(Z - h)) / (2 * h)
    assert np.allclose(J.sum(axis=1), fd, rtol=1e-8, atol=0.0)
