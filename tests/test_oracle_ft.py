"""Pins of the finite-temperature oracle (Matsubara sums, d = 3 + 1, spatial regulator).

What pins what:

* The frequency set: with no tail the rule is exactly the Matsubara frequencies 2 pi T (n + eta)
  with |w| <= lambda, each weighted T (a plain numpy listing, symmetric, bosonic and fermionic).
* The frequency rule as a whole: T sum_n (w_n^2 + E^2)^-k for k = 1, 2, 3 in closed form
  (coth/tanh and their derivatives), reached within the Euler-Maclaurin bound of the midpoint
  boundary between the explicit frequencies and the tail integral.
* The LPA family: its frequency sum done analytically, the radial sum by numpy's leggauss and a
  numpy regulator, so the measure 4 pi/(2 pi)^3, the factor T and the frequency placement are
  pinned (a dropped T, a wrong power of 2 pi or a fermionic/bosonic swap each fail).
* The two-point family at p = 0, p0 = 0: the cubic closed form (angle weights sum to 2).
* The shifted leg (w + p0): mpmath's nsum of the infinite two-sided series at p = 0 for bosonic
  and fermionic external frequencies, including the paper's fermionic choice p0 = pi T exp(-k/pi T).
* Dressing on the spatial momentum and the cos1 geometry: a numpy brute-force listing at tiny
  sizes with a random table and p != 0.
* Units: dimensional scaling in k (LPA: I ~ k^2; two-point: I ~ k^0) with T, m2, p, p0, the
  frequency cutoff and the table range scaled along; the k-scaled frequency domain.
* Invariance: bosonic I(p0) = I(-p0) (the rule is symmetric in w).
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_2412_13043_amd import workloads as wl

PI = math.pi


def closed_sum(k, E, T, fermionic):
    """T sum_n (w_n^2 + E^2)^-k, k = 1, 2, 3, over all Matsubara frequencies.

    With x = E/(2T), g = coth x (bosonic) or tanh x (fermionic) and g', g'' its x-derivatives:
    S1 = g/(2E), S2 = -dS1/d(E^2), S3 = -(1/2) dS2/d(E^2)."""
    x = E / (2.0 * T)
    if fermionic:
        g = math.tanh(x)
        g1 = 1.0 / math.cosh(x) ** 2
        g2 = -2.0 * g1 * g
    else:
        g = 1.0 / math.tanh(x)
        g1 = -1.0 / math.sinh(x) ** 2
        g2 = -2.0 * g1 * g
    if k == 1:
        return g / (2.0 * E)
    if k == 2:
        return g / (4.0 * E ** 3) - g1 / (8.0 * T * E ** 2)
    return 3.0 * g / (16.0 * E ** 5) - 3.0 * g1 / (32.0 * T * E ** 4) + g2 / (64.0 * T * T * E ** 3)


def em_bound(k, E, T, Omega):
    """Euler-Maclaurin leading term of the midpoint boundary on both sides:
    (h^2/24)(1/pi)|f'(Omega)| with h = 2 pi T, f = (w^2 + E^2)^-k (doubled for safety)."""
    h = 2.0 * PI * T
    fp = 2.0 * k * Omega / (Omega * Omega + E * E) ** (k + 1)
    return 2.0 * h * h / 24.0 / PI * fp


def omega_of(stat, T, lam):
    eta = 0.5 if stat == oracle.FERMIONIC else 0.0
    n_hi = math.floor(lam / (2 * PI * T) - eta)
    return 2 * PI * T * (n_hi + eta) + PI * T


def reg_numpy(q2):
    """Exponential regulator (k = 1) and its k d/dk, written independently with numpy."""
    y = np.asarray(q2, dtype=np.float64)
    em = np.expm1(y)
    R = y / em
    Rd = 2.0 * y * y * np.exp(y) / (em * em)
    return R, Rd


# ------------------------------------------------------------------------------------------
# Frequency rule
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("stat", [oracle.BOSONIC, oracle.FERMIONIC])
@pytest.mark.parametrize("T,frac", [(0.05, 0.3), (0.2, 0.7), (1.0, 0.1), (3.0, 0.55)])
def test_bounded_rule_is_the_matsubara_set(stat, T, frac):
    eta = 0.5 if stat == oracle.FERMIONIC else 0.0
    n_edge = 7
    lam = 2 * PI * T * (n_edge + eta + frac)  # between two frequencies
    w, c = oracle.matsubara_rule(stat, T, lam, 0)
    n = np.arange(-200, 201)
    ref = 2 * PI * T * (n + eta)
    ref = ref[np.abs(ref) <= lam]
    assert w.size == ref.size
    assert np.max(np.abs(w - ref)) <= 1e-15 * lam
    assert np.all(c == T)
    assert np.allclose(w, -w[::-1], rtol=0, atol=1e-15 * lam)
    if stat == oracle.BOSONIC:
        assert w.size == 2 * n_edge + 1 and 0.0 in w
    else:
        assert w.size == 2 * n_edge + 2


@pytest.mark.parametrize("stat", [oracle.BOSONIC, oracle.FERMIONIC])
@pytest.mark.parametrize("T", [0.05, 0.2, 1.0])
@pytest.mark.parametrize("E", [0.3, 1.0, 3.0])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_rule_reaches_closed_matsubara_sums(stat, T, E, k):
    lam = 40.0
    w, c = oracle.matsubara_rule(stat, T, lam, 48)
    got = float(np.sum(c * (w * w + E * E) ** (-k)))
    ref = closed_sum(k, E, T, stat == oracle.FERMIONIC)
    tol = em_bound(k, E, T, omega_of(stat, T, lam)) + 1e-14 * ref
    assert abs(got - ref) <= tol, (got, ref, tol)


@pytest.mark.parametrize("stat", [oracle.BOSONIC, oracle.FERMIONIC])
def test_bounded_rule_misses_exactly_the_tail(stat):
    # without the tail the rule is short by the two tail integrals, (1/(pi E))(pi/2 - atan(Omega/E))
    # for f = 1/(w^2 + E^2), to the same Euler-Maclaurin accuracy
    T, E, lam = 0.2, 1.3, 25.0
    w, c = oracle.matsubara_rule(stat, T, lam, 0)
    got = float(np.sum(c / (w * w + E * E)))
    Om = omega_of(stat, T, lam)
    tail = (PI / 2 - math.atan(Om / E)) / (PI * E)
    ref = closed_sum(1, E, T, stat == oracle.FERMIONIC)
    assert abs((ref - got) - tail) <= em_bound(1, E, T, Om) + 1e-14 * ref


def test_rule_rejects_bad_arguments():
    for args in [(2, 0.1, 1.0, 0), (0, 0.0, 1.0, 0), (0, 0.1, -1.0, 0), (0, 0.1, 1.0, -1),
                 (1, 1.0, 1.0, 0)]:  # fermionic with lambda < pi T: no explicit frequency
        with pytest.raises(ValueError):
            oracle.matsubara_rule(*args)


# ------------------------------------------------------------------------------------------
# LPA at finite temperature
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("stat", [oracle.BOSONIC, oracle.FERMIONIC])
@pytest.mark.parametrize("T", [0.1, 0.5])
def test_lpa_ft_against_analytic_frequency_sum(stat, T):
    n_q, q_max, lam, n_tail = 32, 6.0, 60.0, 40
    m2 = np.array([-0.3, 0.0, 0.4, 2.7])
    got = oracle.integrate_ft(oracle.LPA_T, n_q, q_max, T=T, statistics=stat, freq_max=lam,
                              n_tail=n_tail, m2=m2)
    xq, wq = np.polynomial.legendre.leggauss(n_q)
    q = 0.5 * q_max * (xq + 1.0)
    wq = 0.5 * q_max * wq
    R, Rd = reg_numpy(q * q)
    Om = omega_of(stat, T, lam)
    for e, m in enumerate(m2):
        E = np.sqrt(q * q + R + m)
        s2 = np.array([closed_sum(2, Ei, T, stat == oracle.FERMIONIC) for Ei in E])
        ref = float(np.sum(wq * q * q * Rd * s2)) / (2 * PI * PI)
        tol = float(np.sum(wq * q * q * Rd * np.array(
            [em_bound(2, Ei, T, Om) for Ei in E]))) / (2 * PI * PI) + 1e-13 * ref
        assert abs(got[e] - ref) <= tol, (e, got[e], ref, tol)


# ------------------------------------------------------------------------------------------
# Two-point at finite temperature
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("stat", [oracle.BOSONIC, oracle.FERMIONIC])
def test_two_point_ft_zero_momentum_cubic_closed_form(stat):
    n_q, n_x, q_max, T, lam, n_tail = 24, 5, 6.0, 0.25, 50.0, 40
    m2 = np.array([0.1, 0.8])
    got = oracle.integrate_ft(oracle.TWO_POINT_T, n_q, q_max, T=T, statistics=stat, freq_max=lam,
                              n_tail=n_tail, n_x=n_x, ext=(np.zeros(2), np.zeros(2)), m2=m2)
    xq, wq = np.polynomial.legendre.leggauss(n_q)
    q = 0.5 * q_max * (xq + 1.0)
    wq = 0.5 * q_max * wq
    R, Rd = reg_numpy(q * q)
    Om = omega_of(stat, T, lam)
    for e, m in enumerate(m2):
        E = np.sqrt(q * q + R + m)
        s3 = np.array([closed_sum(3, Ei, T, stat == oracle.FERMIONIC) for Ei in E])
        ref = 2.0 * float(np.sum(wq * q * q * Rd * s3)) / (4 * PI * PI)
        tol = 2.0 * float(np.sum(wq * q * q * Rd * np.array(
            [em_bound(3, Ei, T, Om) for Ei in E]))) / (4 * PI * PI) + 1e-13 * ref
        assert abs(got[e] - ref) <= tol


@pytest.mark.parametrize("stat,p0", [(oracle.BOSONIC, 2 * PI * 0.3), (oracle.BOSONIC, 4 * PI * 0.3),
                                     (oracle.FERMIONIC, PI * 0.3 * math.exp(-1.0 / (PI * 0.3))),
                                     (oracle.FERMIONIC, PI * 0.3)])
def test_two_point_ft_shifted_leg_against_infinite_series(stat, p0):
    # p = 0, Z = 1: per radial node the frequency sum is T sum_n G(w_n)^2 G(w_n + p0) with
    # G(w) = 1/(w^2 + E^2); mpmath sums the two-sided infinite series
    n_q, n_x, q_max, T, lam, n_tail = 6, 3, 5.0, 0.3, 30.0, 40
    m = 0.35
    got = oracle.integrate_ft(oracle.TWO_POINT_T, n_q, q_max, T=T, statistics=stat, freq_max=lam,
                              n_tail=n_tail, n_x=n_x, ext=(np.zeros(1), np.full(1, p0)),
                              m2_scalar=m, n_ext=1)[0]
    xq, wq = np.polynomial.legendre.leggauss(n_q)
    q = 0.5 * q_max * (xq + 1.0)
    wq = 0.5 * q_max * wq
    R, Rd = reg_numpy(q * q)
    eta = 0.5 if stat == oracle.FERMIONIC else 0.0
    mp.mp.dps = 30
    ref = 0.0
    bound = 0.0
    Om = omega_of(stat, T, lam)
    for a in range(n_q):
        E2 = mp.mpf(q[a] * q[a] + R[a] + m)

        def term(n):
            w = 2 * mp.pi * T * (n + eta)
            return 1 / ((w * w + E2) ** 2 * ((w + p0) ** 2 + E2))

        s = T * mp.nsum(term, [-mp.inf, mp.inf])
        ref += float(wq[a] * q[a] ** 2 * Rd[a]) * 2.0 * float(s)
        # the summand decays like w^-6; bound its boundary term by the k = 3 one at the
        # smaller of the two denominators
        bound += float(wq[a] * q[a] ** 2 * Rd[a]) * 2.0 * 4.0 * em_bound(
            3, math.sqrt(max(float(E2), 1e-12)), T, Om - abs(p0))
    ref /= 4 * PI * PI
    bound /= 4 * PI * PI
    assert abs(got - ref) <= bound + 1e-13 * ref, (got, ref, bound)


def test_two_point_ft_brute_force_listing():
    # tiny sizes, a random dressing table on the spatial momentum, p != 0, p0 != 0, no tail:
    # every term listed with numpy
    rng = np.random.default_rng(7)
    Z = 1.0 + 0.3 * rng.random(9)
    xmin, xmax = 1e-2, 1e2
    n_q, n_x, q_max, T, lam = 3, 4, 4.0, 0.4, 9.0
    p = np.array([0.2, 1.7])
    p0 = np.array([2 * PI * T, -0.9])
    m = np.array([0.3, 1.1])
    for stat in (oracle.BOSONIC, oracle.FERMIONIC):
        got = oracle.integrate_ft(oracle.TWO_POINT_T, n_q, q_max, T=T, statistics=stat,
                                  freq_max=lam, n_x=n_x, ext=(p, p0), m2=m, Z=Z, x_min=xmin,
                                  x_max=xmax)
        eta = 0.5 if stat == oracle.FERMIONIC else 0.0
        n = np.arange(-100, 101)
        w = 2 * PI * T * (n + eta)
        w = w[np.abs(w) <= lam]
        xq, wq = np.polynomial.legendre.leggauss(n_q)
        q = 0.5 * q_max * (xq + 1.0)
        wq = 0.5 * q_max * wq
        xx, wx = np.polynomial.legendre.leggauss(n_x)

        def zd(l2):
            s = (0.5 * np.log(l2) - np.log(xmin)) / ((np.log(xmax) - np.log(xmin)) / (Z.size - 1))
            return np.interp(s, np.arange(Z.size), Z)

        for e in range(2):
            tot = 0.0
            for wj in w:
                for a in range(n_q):
                    q2 = q[a] ** 2
                    Rq, Rdq = reg_numpy(q2)
                    gq = 1.0 / (wj * wj + zd(q2) * q2 + Rq + m[e])
                    for b in range(n_x):
                        l2 = q2 + p[e] ** 2 + 2 * q[a] * p[e] * xx[b]
                        Rl, _ = reg_numpy(l2)
                        gl = 1.0 / ((wj + p0[e]) ** 2 + zd(l2) * l2 + Rl + m[e])
                        tot += T * wq[a] * wx[b] * q2 * Rdq * gq * gq * gl
            ref = tot * 2 * PI / (2 * PI) ** 3
            assert abs(got[e] - ref) <= 1e-13 * abs(ref)


@pytest.mark.parametrize("stat", [oracle.BOSONIC, oracle.FERMIONIC])
def test_two_point_ft_bosonic_reflection(stat):
    T = 0.2
    p0 = 2 * PI * T * 2 if stat == oracle.BOSONIC else 0.77
    p = np.array([0.0, 0.5, 3.0])
    kw = dict(T=T, statistics=stat, freq_max=12.0, n_tail=16, n_x=8)
    a = oracle.integrate_ft(oracle.TWO_POINT_T, 16, 6.0, ext=(p, np.full(3, p0)), m2_scalar=0.4,
                            **kw)
    b = oracle.integrate_ft(oracle.TWO_POINT_T, 16, 6.0, ext=(p, np.full(3, -p0)),
                            m2_scalar=0.4, **kw)
    # the rule is symmetric in w for both statistics, so w -> -w maps one sum onto the other
    assert np.max(np.abs(a - b) / a) < 1e-13


@pytest.mark.parametrize("family", [oracle.LPA_T, oracle.TWO_POINT_T])
def test_ft_dimensional_scaling_in_k(family):
    # I(k; T, m2, p, p0, lambda, Z range) = k^s I(1; T/k, m2/k^2, p/k, p0/k, lambda/k, range/k)
    # with s = 2 (LPA) and 0 (two-point); q_max is in units of k already
    k = 1.7
    rng = np.random.default_rng(3)
    Z = 1.0 + 0.2 * rng.random(16)
    T, lam = 0.3, 15.0
    m2 = np.array([0.2, 1.5])
    p = np.array([0.4, 2.0])
    p0 = np.array([0.5, -1.1])
    common = dict(statistics=oracle.FERMIONIC, n_tail=12, n_x=6)
    ext_k = (p, p0) if family == oracle.TWO_POINT_T else None
    ext_1 = (p / k, p0 / k) if family == oracle.TWO_POINT_T else None
    zk = dict(Z=Z, x_min=1e-2 * k, x_max=1e2 * k) if family == oracle.TWO_POINT_T else {}
    z1 = dict(Z=Z, x_min=1e-2, x_max=1e2) if family == oracle.TWO_POINT_T else {}
    a = oracle.integrate_ft(family, 20, 6.0, k=k, T=T, freq_max=lam, ext=ext_k, m2=m2, **zk,
                            **common)
    b = oracle.integrate_ft(family, 20, 6.0, k=1.0, T=T / k, freq_max=lam / k, ext=ext_1,
                            m2=m2 / k ** 2, **z1, **common)
    s = 2 if family == oracle.LPA_T else 0
    assert np.max(np.abs(a - k ** s * b) / np.abs(a)) < 1e-12
    # the k-scaled frequency domain is freq_max * k
    c = oracle.integrate_ft(family, 20, 6.0, k=k, T=T, freq_max=lam / k, freq_scaled=True,
                            ext=ext_k, m2=m2, **zk, **common)
    assert np.array_equal(a, c)


# ------------------------------------------------------------------------------------------
# Three-point at finite temperature
# ------------------------------------------------------------------------------------------
def _rotation3(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    return q * np.sign(np.diag(r))


@pytest.mark.parametrize("alpha", [0.0, 1.1, PI])
def test_three_point_ft_rotation_invariance(alpha):
    # the reduced (x, phi) form against explicit spatial 3-vectors on a spherical product rule,
    # external vectors rotated at random, shifted leg frequencies, a dressing table
    rng = np.random.default_rng(int(10 * alpha) + 1)
    Z = wl.dressing_table(3, 32)
    p, m2, p01, p02 = 0.9, 0.45, 2 * PI * 0.3, -0.7
    ft = dict(T=0.3, statistics=oracle.FERMIONIC, freq_max=6.0, n_tail=4)
    reduced = oracle.integrate_ft(oracle.THREE_POINT_T, 24, 6.0, n_x=512, n_phi=48,
                                  ext=([p], [alpha], [p01], [p02]), m2_scalar=m2, Z=Z, **ft)[0]
    Q = _rotation3(rng)
    p1 = Q @ np.array([p, 0.0, 0.0])
    p2 = Q @ np.array([p * math.cos(alpha), p * math.sin(alpha), 0.0])
    sph = oracle.vertex_ft_spherical(24, 72, 72, 6.0, p1, p2, p01, p02, m2, Z=Z, **ft)
    assert abs(sph - reduced) / reduced < 2e-6, (alpha, sph, reduced)


@pytest.mark.parametrize("stat,p01,p02", [(oracle.BOSONIC, 2 * PI * 0.3, -4 * PI * 0.3),
                                          (oracle.FERMIONIC, 0.8, 0.2)])
def test_three_point_ft_zero_momentum_against_infinite_series(stat, p01, p02):
    # p = 0, Z = 1: the angles drop out (sum of the x and folded phi weights: 2 x 2 pi = 4 pi)
    # and per radial node the frequency sum is T sum_n G(w_n)^2 G(w_n + p01) G(w_n + p02),
    # G(w) = 1/(w^2 + E^2); mpmath sums the two-sided infinite series
    n_q, q_max, T, lam, n_tail = 6, 5.0, 0.3, 30.0, 40
    m = 0.35
    got = oracle.integrate_ft(oracle.THREE_POINT_T, n_q, q_max, T=T, statistics=stat,
                              freq_max=lam, n_tail=n_tail, n_x=3, n_phi=4,
                              ext=([0.0], [0.7], [p01], [p02]), m2_scalar=m)[0]
    xq, wq = np.polynomial.legendre.leggauss(n_q)
    q = 0.5 * q_max * (xq + 1.0)
    wq = 0.5 * q_max * wq
    R, Rd = reg_numpy(q * q)
    eta = 0.5 if stat == oracle.FERMIONIC else 0.0
    mp.mp.dps = 30
    ref = 0.0
    bound = 0.0
    Om = omega_of(stat, T, lam)
    for a in range(n_q):
        E2 = mp.mpf(q[a] * q[a] + R[a] + m)

        def term(n):
            w = 2 * mp.pi * T * (n + eta)
            return 1 / ((w * w + E2) ** 2 * ((w + p01) ** 2 + E2) * ((w + p02) ** 2 + E2))

        s = T * mp.nsum(term, [-mp.inf, mp.inf])
        ref += float(wq[a] * q[a] ** 2 * Rd[a]) * float(s)
        # the summand decays like w^-8; bound the boundary term by the k = 4 one at the
        # smallest of the denominators
        bound += float(wq[a] * q[a] ** 2 * Rd[a]) * 8.0 * em_bound(
            4, math.sqrt(max(float(E2), 1e-12)), T, Om - max(abs(p01), abs(p02)))
    ref *= 4 * PI / (2 * PI) ** 3
    bound *= 4 * PI / (2 * PI) ** 3
    assert abs(got - ref) <= bound + 1e-13 * ref, (got, ref, bound)


def test_three_point_ft_mass_derivative_against_differences():
    Z = wl.dressing_table(5, 24)
    ext = (np.array([0.3, 1.4]), np.array([0.4, 2.5]), np.array([0.6, -1.2]),
           np.array([0.0, 0.9]))
    kw = dict(T=0.25, statistics=oracle.BOSONIC, freq_max=8.0, n_tail=6, n_x=8, n_phi=6, Z=Z,
              ext=ext)
    m = np.array([0.5, 0.8])
    d = oracle.integrate_ft(oracle.THREE_POINT_T, 12, 6.0, m2=m, dm2=True, **kw)
    f = lambda mm: oracle.integrate_ft(oracle.THREE_POINT_T, 12, 6.0, m2=mm, **kw)
    h = 1e-3
    d1 = (f(m + h) - f(m - h)) / (2 * h)
    d2 = (f(m + 2 * h) - f(m - 2 * h)) / (4 * h)
    rich = (4 * d1 - d2) / 3
    assert np.max(np.abs(d - rich) / np.abs(d)) < 1e-9


def test_three_point_ft_dimensional_scaling_in_k():
    # I(k; ...) = k^-2 I(1; T/k, m2/k^2, p/k, p0i/k, lambda/k, range/k): one more propagator
    # than the two-point family
    k = 1.7
    rng = np.random.default_rng(4)
    Z = 1.0 + 0.2 * rng.random(16)
    T, lam = 0.3, 15.0
    m2 = np.array([0.2, 1.5])
    p, al = np.array([0.4, 2.0]), np.array([0.3, 2.9])
    p01, p02 = np.array([0.5, -1.1]), np.array([-0.2, 0.7])
    common = dict(statistics=oracle.FERMIONIC, n_tail=12, n_x=6, n_phi=5)
    a = oracle.integrate_ft(oracle.THREE_POINT_T, 20, 6.0, k=k, T=T, freq_max=lam,
                            ext=(p, al, p01, p02), m2=m2, Z=Z, x_min=1e-2 * k, x_max=1e2 * k,
                            **common)
    b = oracle.integrate_ft(oracle.THREE_POINT_T, 20, 6.0, k=1.0, T=T / k, freq_max=lam / k,
                            ext=(p / k, al, p01 / k, p02 / k), m2=m2 / k ** 2, Z=Z, x_min=1e-2,
                            x_max=1e2, **common)
    assert np.max(np.abs(a - k ** -2 * b) / np.abs(a)) < 1e-12
