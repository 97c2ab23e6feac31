"""Pins of the FP64 oracle to things other than itself (CPU only).

Each check is chosen so that a plausible slip in the oracle -- a dropped factor, a wrong sign,
a swapped angle, a wrong measure or prefactor, an off-by-one in the table lookup -- fails at
least one of them:

* Gauss-Legendre rules: numpy's ``leggauss`` (library routine), weight sums, exactness on
  monomials up to degree 2n-1, symmetry.
* Regulator and its scale derivative: 40-digit mpmath evaluation of the defining formula
  R = l2/(exp(l2/k^2) - 1), and k dR/dk by mpmath differentiation with respect to k (pins the
  sign and the factor of the RG-scale derivative, paper Sec. 2.1 / Sec. 3.1).
* Dressing lookup: ``numpy.interp`` on log coordinates (library routine), grid nodes, clamps.
* Flat-regulator threshold functions: closed forms (exact for GL with n >= 2).
* Angular measures: closed forms of int sqrt(1-x^2)/(A+Bx) dx and int sin(phi)/(C+D cos phi)
  dphi, reached by the full oracle within the quadrature error bound.
* Brute-force Cartesian midpoint sums in d = 4 (pins measure, normalisation, leg geometry).
* A full hyperspherical rule with externals along random directions (rotation invariance).
* Convergence under node doubling, asserting rates.
* LPA flow right-hand side: the textbook flat-regulator LPA flow of the O(N) model.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_2412_13043_amd import workloads as wl

PI = math.pi


# ------------------------------------------------------------------------------------------
# Gauss-Legendre
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 3, 7, 16, 32, 64, 128])
def test_gl_matches_numpy_leggauss(n):
    # numpy's own rule loses accuracy in the smallest weights as n grows (~1e-13 at n = 32,
    # ~3e-11 at n = 128); the 40-digit check below is the tight pin
    x, w = oracle.gauss_legendre(n, -1.0, 1.0)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.max(np.abs(x - xr)) < 4e-16
    assert np.max(np.abs(w - wr) / wr) < 2e-14 * n * n


@pytest.mark.parametrize("n", [5, 32, 128])
def test_gl_matches_mpmath_newton(n):
    # 40-digit Newton on mpmath's Legendre polynomials
    x, w = oracle.gauss_legendre(n, -1.0, 1.0)
    idx = range(n) if n <= 32 else [0, 1, 2, n // 3, n // 2, n - 1]
    for xi, wi in zip(x[list(idx)], w[list(idx)]):
        t = mp.mpf(xi)
        for _ in range(4):
            t = t - mp.legendre(n, t) / mp.diff(lambda s: mp.legendre(n, s), t)
        dp = mp.diff(lambda s: mp.legendre(n, s), t)
        wref = 2 / ((1 - t * t) * dp * dp)
        assert abs(xi - float(t)) <= 2.3e-16
        assert abs(wi - float(wref)) <= 2.3e-16 * float(wref)


@pytest.mark.parametrize("n,a,b", [(5, 0.0, 6.0), (32, 0.0, 6.0), (64, 0.0, 10.0),
                                   (32, -1.0, 1.0), (16, 0.0, PI), (17, -2.5, 3.25)])
def test_gl_exactness_and_symmetry(n, a, b):
    x, w = oracle.gauss_legendre(n, a, b)
    assert np.all(np.diff(x) > 0) and np.all((x > a) & (x < b))
    assert abs(w.sum() - (b - a)) < 1e-14 * (b - a)
    # exact on monomials (t)^j, j <= 2n-1, with t = (x - mid)/half in [-1, 1]
    mid, half = 0.5 * (a + b), 0.5 * (b - a)
    t = (x - mid) / half
    for j in range(0, 2 * n):
        exact = 0.0 if j % 2 else 2.0 / (j + 1)
        got = np.sum(w * t ** j) / half
        assert abs(got - exact) < 5e-14, (j, got, exact)
    # symmetric nodes / weights about the midpoint
    assert np.max(np.abs(t + t[::-1])) < 1e-15 * max(1.0, n)
    assert np.max(np.abs(w - w[::-1]) / w) < 1e-13


# ------------------------------------------------------------------------------------------
# Regulator
# ------------------------------------------------------------------------------------------
mp.mp.dps = 40


def _R_mp(l2, k):
    l2, k = mp.mpf(l2), mp.mpf(k)
    if l2 == 0:
        return k * k
    return l2 / mp.expm1(l2 / (k * k))


def _Rdot_mp(l2, k):
    # k d/dk R_k(l2) at fixed l2, by high-precision numerical differentiation
    return mp.mpf(k) * mp.diff(lambda kk: _R_mp(l2, kk), mp.mpf(k))


@pytest.mark.parametrize("y", [1e-12, 1e-8, 6.7e-5, 0.01, 0.3, 0.69, 0.7, 1.0, 5.0, 40.0, 100.0,
                               700.0])
@pytest.mark.parametrize("k", [1.0, 0.37])
def test_exponential_regulator_vs_mpmath(y, k):
    l2 = y * k * k
    R = oracle.regulator(l2, k)
    Rd = oracle.regulator_dot(l2, k)
    R_ref = float(_R_mp(l2, k))
    Rd_ref = float(_Rdot_mp(l2, k))
    # y = l2/k^2 is rounded once (0.5 ulp), which exp(-y) amplifies by its condition number y
    cond = 2.3e-16 * y
    assert abs(R - R_ref) <= (4e-16 + cond) * abs(R_ref) + 1e-300
    assert abs(Rd - Rd_ref) <= (8e-16 + cond) * abs(Rd_ref) + 1e-300
    assert Rd > 0.0  # k dR/dk > 0: the integrals are positive


def test_exponential_regulator_limits():
    assert oracle.regulator(0.0, 1.0) == 1.0
    assert oracle.regulator_dot(0.0, 1.0) == 2.0
    assert oracle.regulator(1e4, 1.0) == 0.0  # exp(-1e4) underflows: no overflow, no NaN
    assert oracle.regulator_dot(1e4, 1.0) == 0.0
    assert oracle.regulator(-1e-18, 1.0) == 1.0  # rounding residue below zero is clamped


def test_litim_regulator():
    k = 1.3
    for l2 in [0.0, 0.5, 1.0, 1.68, 1.7, 4.0]:
        R = oracle.regulator(l2, k, kind=oracle.REG_LITIM)
        Rd = oracle.regulator_dot(l2, k, kind=oracle.REG_LITIM)
        inside = l2 < k * k
        assert R == pytest.approx((k * k - l2) if inside else 0.0, abs=1e-15)
        assert Rd == pytest.approx(2 * k * k if inside else 0.0, abs=1e-15)
    # shape function r(x) = (1/x - 1) Theta(1 - x) with R = l2 r(l2/k^2)
    l2 = 0.4 * k * k
    assert oracle.regulator(l2, k, kind=oracle.REG_LITIM) == pytest.approx(
        l2 * (1 / 0.4 - 1), rel=1e-15)


# ------------------------------------------------------------------------------------------
# Dressing lookup and propagator
# ------------------------------------------------------------------------------------------
def test_dressing_vs_numpy_interp():
    Z = wl.dressing_table(1)
    lx = np.linspace(math.log(wl.Z_XMIN), math.log(wl.Z_XMAX), wl.Z_POINTS)
    rng = np.random.default_rng(0)
    ell = np.exp(rng.uniform(math.log(1e-4), math.log(1e4), 2000))
    ref = np.interp(np.log(ell), lx, Z)  # clamps at both ends like the oracle
    got = np.array([oracle.dressing(Z, wl.Z_XMIN, wl.Z_XMAX, e * e) for e in ell])
    assert np.max(np.abs(got - ref)) < 2e-14


def test_dressing_nodes_and_clamps():
    Z = wl.dressing_table(7)
    lx = np.linspace(math.log(wl.Z_XMIN), math.log(wl.Z_XMAX), wl.Z_POINTS)
    for i in [0, 1, 17, 128, 254, 255]:
        l2 = math.exp(2 * lx[i])
        assert oracle.dressing(Z, wl.Z_XMIN, wl.Z_XMAX, l2) == pytest.approx(Z[i], abs=1e-13)
    assert oracle.dressing(Z, wl.Z_XMIN, wl.Z_XMAX, 0.0) == Z[0]
    assert oracle.dressing(Z, wl.Z_XMIN, wl.Z_XMAX, 1e-30) == Z[0]
    assert oracle.dressing(Z, wl.Z_XMIN, wl.Z_XMAX, 1e30) == Z[-1]
    assert oracle.dressing(None, wl.Z_XMIN, wl.Z_XMAX, 3.0) == 1.0


def test_propagator_definition_mpmath():
    Z = wl.dressing_table(3)
    for l2, m2 in [(0.0, 0.5), (1e-9, -0.95), (0.3, 0.1), (2.0, 2.0), (1.2e4, 0.5)]:
        z = oracle.dressing(Z, wl.Z_XMIN, wl.Z_XMAX, l2)
        D = mp.mpf(z) * l2 + _R_mp(l2, 1.0) + m2
        ref = 1 / D
        got = oracle.propagator(l2, m2, Z=Z)
        # the sum Z l2 + R + m2 cancels near the pole; rounding is amplified by kappa
        kappa = float((abs(mp.mpf(z) * l2 + _R_mp(l2, 1.0)) + abs(m2)) / D)
        assert abs(got - float(ref)) <= 2.3e-16 * (4 + 2 * kappa) * abs(float(ref))


# ------------------------------------------------------------------------------------------
# Flat-regulator threshold functions (exact with GL n >= 2 on [0, k])
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("d", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("m2", [-0.5, 0.0, 0.5, 3.0])
def test_lpa_litim_closed_form(d, m2):
    k = 1.7
    n = max(2, (d + 1) // 2 + 1)
    got = oracle.integrate(oracle.LPA, n, 1.0, d=d, k=k, m2=[m2], regulator=oracle.REG_LITIM)[0]
    omega = 2 * PI ** (d / 2) / math.gamma(d / 2)
    exact = omega / (2 * PI) ** d * 2 * k * k * (k ** d / d) / (k * k + m2) ** 2
    assert abs(got - exact) <= 1e-14 * exact
    if d == 3:
        assert got == pytest.approx(k ** 5 / (3 * PI ** 2 * (k * k + m2) ** 2), rel=1e-14)


def test_lpa_litim_worked_value():
    # GL(4), m2 = 0.5, k = 1: 1/(3 pi^2 1.5^2)
    got = oracle.integrate(oracle.LPA, 4, 1.0, m2=[0.5], regulator=oracle.REG_LITIM)[0]
    assert got == pytest.approx(0.0150105457247908, rel=1e-14)


def test_two_point_litim_p0_closed_form():
    # p = 0, Z = 1, flat regulator: integrand Rdot G^3 does not depend on x, so
    # I = k^6/(16 pi^2 (k^2+m2)^3) * [sum_b w_b sqrt(1-x_b^2)]/(pi/2)   (discrete identity)
    k, m2, n_x = 1.0, 0.5, 32
    got = oracle.integrate(oracle.TWO_POINT, 4, 1.0, n_x=n_x, ext=[0.0], m2_scalar=m2,
                           regulator=oracle.REG_LITIM)[0]
    x, w = np.polynomial.legendre.leggauss(n_x)
    ang = np.sum(w * np.sqrt(1 - x * x))
    exact = k ** 6 / (16 * PI ** 2 * (k * k + m2) ** 3) * ang / (PI / 2)
    assert abs(got - exact) <= 2e-15 * exact
    # and the angular factor tends to pi/2 at the O(N^-3) rate of GL with a sqrt weight
    errs = []
    for n in (32, 64, 128):
        xx, ww = np.polynomial.legendre.leggauss(n)
        errs.append(abs(np.sum(ww * np.sqrt(1 - xx * xx)) - PI / 2))
    assert 6.0 < errs[0] / errs[1] < 10.0 and 6.0 < errs[1] / errs[2] < 10.0


# ------------------------------------------------------------------------------------------
# Angular closed forms (external legs beyond the flat regulator's support: p > 2k)
# ------------------------------------------------------------------------------------------
def _two_point_litim_reference(p, m2, k=1.0):
    # int_0^k dq q^3 2k^2/(k^2+m2)^2 * pi (A - sqrt(A^2 - B^2))/B^2, A = q^2+p^2+m2, B = 2 q p
    def f(q):
        A = q * q + p * p + m2
        B = 2 * q * p
        if B == 0:
            ang = PI / (2 * A)
        else:
            ang = PI * (A - mp.sqrt(A * A - B * B)) / (B * B)
        return q ** 3 * 2 * k * k / (k * k + m2) ** 2 * ang
    return float(mp.quad(f, [0, k]) * 4 * PI / (2 * PI) ** 4)


@pytest.mark.parametrize("p", [2.5, 4.0, 30.0])
def test_two_point_angular_closed_form(p):
    m2 = 0.3
    ref = _two_point_litim_reference(p, m2)
    got = [oracle.integrate(oracle.TWO_POINT, 16, 1.0, n_x=n, ext=[p], m2_scalar=m2,
                            regulator=oracle.REG_LITIM)[0] for n in (64, 128, 512)]
    errs = [abs(g - ref) / ref for g in got]
    assert errs[2] < 2e-8
    assert 5.0 < errs[0] / errs[1] < 11.0  # O(N^-3) with GL nodes and sqrt(1-x^2) weights


def test_three_point_phi_closed_form():
    # flat regulator, p > 2k, Z = 1: the phi integral has the closed form
    # int_0^pi sin(phi)/(C + D cos(phi)) dphi = ln((C+D)/(C-D))/D.
    from scipy import integrate as si
    p, alpha, m2, k = 3.0, 1.1, 0.4, 1.0
    ca, sa = math.cos(alpha), math.sin(alpha)

    def inner(x, q):
        sx = math.sqrt(1 - x * x)
        g1 = 1.0 / (q * q + p * p + 2 * q * p * x + m2)
        C = q * q + p * p - 2 * q * p * x * ca + m2
        D = -2 * q * p * sx * sa
        phi_int = 2.0 / C if abs(D) < 1e-300 else math.log((C + D) / (C - D)) / D
        return sx * g1 * phi_int

    def radial(q):
        v, _ = si.quad(inner, -1.0, 1.0, args=(q,), epsabs=0, epsrel=1e-13, limit=200)
        return q ** 3 * 2 * k * k / (k * k + m2) ** 2 * v

    ref, _ = si.quad(radial, 0.0, k, epsabs=0, epsrel=1e-12, limit=200)
    ref *= 2 * PI / (2 * PI) ** 4
    got = oracle.integrate(oracle.THREE_POINT, 8, 1.0, n_x=256, n_phi=24,
                           ext=([p], [alpha]), m2_scalar=m2, regulator=oracle.REG_LITIM)[0]
    assert abs(got - ref) / ref < 3e-7


# ------------------------------------------------------------------------------------------
# Brute-force Cartesian midpoint sums in d = 4 (exponential regulator, Z = 1)
# ------------------------------------------------------------------------------------------
def _np_R(l2):
    y = np.maximum(l2, 1e-300)
    return y / np.expm1(y)


def _np_G(l2, m2):
    return 1.0 / (l2 + _np_R(l2) + m2)


def _np_Rdot(l2):
    y = np.maximum(l2, 1e-300)
    em = np.expm1(y)
    return 2 * y * y * (em + 1) / (em * em)


def _cartesian(p1, p2, m2, L, n, legs):
    h = 2 * L / n
    g = -L + h * (np.arange(n) + 0.5)
    q1, q2, q3 = np.meshgrid(g, g, g, indexing="ij")
    total = 0.0
    for a in g:  # chunk over the first component
        qq = a * a + q1 * q1 + q2 * q2 + q3 * q3
        f = _np_Rdot(qq) * _np_G(qq, m2) ** 2
        l1 = (a + p1[0]) ** 2 + (q1 + p1[1]) ** 2 + (q2 + p1[2]) ** 2 + (q3 + p1[3]) ** 2
        f = f * _np_G(l1, m2)
        if legs == 3:
            l2 = (a - p2[0]) ** 2 + (q1 - p2[1]) ** 2 + (q2 - p2[2]) ** 2 + (q3 - p2[3]) ** 2
            f = f * _np_G(l2, m2)
        total += f.sum()
    return total * h ** 4 / (2 * PI) ** 4


def test_two_point_vs_cartesian_bruteforce():
    p, m2 = 0.8, 0.5
    bf = _cartesian([p, 0, 0, 0], None, m2, 7.0, 44, 2)
    bf2 = _cartesian([p, 0, 0, 0], None, m2, 7.0, 52, 2)
    assert abs(bf - bf2) / bf < 1e-9  # the midpoint sum has converged
    got = oracle.integrate(oracle.TWO_POINT, 64, 10.0, n_x=1024, ext=[p], m2_scalar=m2)[0]
    assert abs(got - bf2) / bf2 < 1e-8


def test_three_point_vs_cartesian_bruteforce():
    p, alpha, m2 = 0.9, 2.0, 0.7
    p1 = [p, 0, 0, 0]
    p2 = [p * math.cos(alpha), p * math.sin(alpha), 0, 0]
    bf = _cartesian(p1, p2, m2, 7.0, 48, 3)
    got = oracle.integrate(oracle.THREE_POINT, 64, 10.0, n_x=512, n_phi=48,
                           ext=([p], [alpha]), m2_scalar=m2)[0]
    assert abs(got - bf) / bf < 1e-7


# ------------------------------------------------------------------------------------------
# Rotation invariance: reduced angle forms vs a full hyperspherical rule, random directions
# ------------------------------------------------------------------------------------------
def _rand_unit(rng):
    v = rng.normal(size=4)
    return v / np.linalg.norm(v)


def _rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(4, 4)))
    return q * np.sign(np.diag(r))


def test_two_point_rotation_invariance():
    rng = np.random.default_rng(5)
    Z = wl.dressing_table(1)
    p, m2 = 1.3, 0.5
    reduced = oracle.integrate(oracle.TWO_POINT, 48, 10.0, n_x=1024, ext=[p], m2_scalar=m2, Z=Z)[0]
    for _ in range(2):
        p1 = p * _rand_unit(rng)
        hyp = oracle.vertex_hyperspherical(2, 48, 96, 24, 24, 10.0, p1, np.zeros(4), m2, Z=Z)
        assert abs(hyp - reduced) / reduced < 1e-6


def test_three_point_rotation_invariance_and_special_angles():
    rng = np.random.default_rng(6)
    p, m2 = 0.7, 0.6
    for alpha in (0.0, 1.2, PI):
        reduced = oracle.integrate(oracle.THREE_POINT, 40, 10.0, n_x=512, n_phi=48,
                                   ext=([p], [alpha]), m2_scalar=m2)[0]
        Q = _rotation(rng)
        p1 = Q @ np.array([p, 0, 0, 0])
        p2 = Q @ np.array([p * math.cos(alpha), p * math.sin(alpha), 0, 0])
        hyp = oracle.vertex_hyperspherical(3, 40, 72, 36, 36, 10.0, p1, p2, m2)
        assert abs(hyp - reduced) / reduced < 2e-6, alpha
        # swapping the roles of the two external legs leaves the integral unchanged
        hyp_sw = oracle.vertex_hyperspherical(3, 40, 72, 36, 36, 10.0, p2, p1, m2)
        assert abs(hyp_sw - hyp) / hyp < 1e-9


def test_three_point_alpha_zero_factorises():
    # at alpha = 0 nothing depends on phi: the phi sum is sum_c w_c sin(phi_c) times a
    # two-angle-free product, i.e. I3 = [sum_c w_c sin phi_c]/2 * I3(phi-exact)
    p, m2, n_phi = 0.5, 0.4, 16
    a = oracle.integrate(oracle.THREE_POINT, 32, 10.0, n_x=32, n_phi=n_phi, ext=([p], [0.0]),
                         m2_scalar=m2)[0]
    b = oracle.integrate(oracle.THREE_POINT, 32, 10.0, n_x=32, n_phi=2 * n_phi,
                         ext=([p], [0.0]), m2_scalar=m2)[0]
    x, w = oracle.gauss_legendre(n_phi, 0.0, PI)
    x2, w2 = oracle.gauss_legendre(2 * n_phi, 0.0, PI)
    sa = np.sum(w * np.sin(x))
    sb = np.sum(w2 * np.sin(x2))
    assert abs(a / sa - b / sb) / (a / sa) < 1e-14


# ------------------------------------------------------------------------------------------
# Convergence under node doubling
# ------------------------------------------------------------------------------------------
def test_lpa_radial_spectral_convergence_vs_mpmath():
    # exponential regulator, m2 = 0.5: GL32 on [0, 6k] reaches the exact integral over [0, 6k]
    m2 = 0.5

    def f(q):
        q2 = q * q
        R = _R_mp(q2, 1)
        Rd = mp.mpf(1) * mp.diff(lambda kk: _R_mp(q2, kk), mp.mpf(1))
        return q2 * Rd / (q2 + R + m2) ** 2

    mp.mp.dps = 30
    exact = float(mp.quad(f, [0, 1, 3, 6]) / (2 * mp.pi ** 2))
    mp.mp.dps = 40
    g16 = oracle.integrate(oracle.LPA, 16, 6.0, m2=[m2])[0]
    g32 = oracle.integrate(oracle.LPA, 32, 6.0, m2=[m2])[0]
    assert abs(g32 - exact) / exact < 5e-15
    assert 1e-9 < abs(g16 - exact) / exact < 1e-5


def test_two_point_tabulated_z_convergence():
    # with a piecewise-linear Z the angular error is dominated by the sqrt weight (~N^-3)
    Z = wl.dressing_table(1)
    p = 0.6
    vals = [oracle.integrate(oracle.TWO_POINT, 64, 10.0, n_x=n, ext=[p], m2_scalar=0.5, Z=Z)[0]
            for n in (32, 64, 128, 1024)]
    e = [abs(v - vals[-1]) for v in vals[:3]]
    assert e[0] > e[1] > e[2]
    assert e[0] / e[1] > 3.0


# ------------------------------------------------------------------------------------------
# LPA flow right-hand side
# ------------------------------------------------------------------------------------------
def test_fd_derivatives_exact_for_quadratics():
    rng = np.random.default_rng(2)
    x = np.sort(rng.uniform(0, 1, 9))
    f = 0.3 - 1.7 * x + 2.2 * x * x
    d1, d2 = oracle.fd_derivatives(x, f)
    assert np.max(np.abs(d1 - (-1.7 + 4.4 * x))) < 1e-11
    assert np.max(np.abs(d2 - 4.4)) < 1e-9


def test_lpa_flow_rhs_litim_textbook():
    # Flat regulator, d = 3: k dV/dk = k^5/(6 pi^2) [1/(k^2+m_s^2) + (N-1)/(k^2+m_p^2)], so with
    # t = log(Lambda/k): du/dt = k^5/(6 pi^2) [(3u'+2 rho u'')/(k^2+m_s^2)^2 + (N-1) u'/(k^2+m_p^2)^2]
    rho = np.linspace(0, 1, 16)
    u = -0.2 + 0.7 * rho + 0.4 * rho ** 2
    up, upp = 0.7 + 0.8 * rho, 0.8
    ms = u + 2 * rho * up
    N = 4
    got = oracle.lpa_flow_rhs(rho, u, 4, 1.0, regulator=oracle.REG_LITIM, n_comp=N, m2_floor=-0.9)
    ref = (1.0 / (6 * PI ** 2)) * ((3 * up + 2 * rho * upp) / (1 + ms) ** 2 +
                                   (N - 1) * up / (1 + u) ** 2)
    assert np.max(np.abs(got - ref) / np.abs(ref)) < 1e-10
