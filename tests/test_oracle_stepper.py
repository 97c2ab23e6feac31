"""Pins of the oracle's adaptive Dormand-Prince 5(4) stepper (CPU only).

* The tableau: row sums equal the nodes; the fifth-order weights satisfy every order condition
  up to order 5 listed below (exact rational arithmetic), the embedded weights those up to
  order 4 but not the order-5 quadrature condition; first same as last.
* Convergence orders measured on closed-form solutions: global error of fixed steps O(h^5),
  the embedded error estimate of one step O(h^5).
* Adaptive runs reach closed-form solutions within the requested tolerance, accepted steps have
  err <= 1, and a too-large first step is rejected and shrunk.
* scipy's solve_ivp(method="RK45") (a library Dormand-Prince with its own controller) reaches
  the same state of the oracle's LPA flow with k(t) = exp(-t) at tight tolerances.
"""
import math
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from oracle import stepper as rk
from paper_2412_13043_amd import workloads as wl


def test_tableau_consistency_and_order_conditions():
    A, B, BH, C = rk.A, rk.B, rk.BHAT, rk.C
    s = 7
    a = [[A[i][j] if j < len(A[i]) else F(0) for j in range(s)] for i in range(s)]
    for i in range(s):
        assert sum(a[i]) == C[i]
    assert a[6][:6] == B[:6] and C[6] == 1  # first same as last
    def quad(w, k):
        return sum(w[i] * C[i] ** (k - 1) for i in range(s))
    for k in range(1, 6):
        assert quad(B, k) == F(1, k)
    for k in range(1, 5):
        assert quad(BH, k) == F(1, k)
    assert quad(BH, 5) != F(1, 5)
    ac = [sum(a[i][j] * C[j] for j in range(s)) for i in range(s)]
    ac2 = [sum(a[i][j] * C[j] ** 2 for j in range(s)) for i in range(s)]
    ac3 = [sum(a[i][j] * C[j] ** 3 for j in range(s)) for i in range(s)]
    aac = [sum(a[i][j] * ac[j] for j in range(s)) for i in range(s)]
    for w, order in ((B, 5), (BH, 4)):
        assert sum(w[i] * ac[i] for i in range(s)) == F(1, 6)
        assert sum(w[i] * C[i] * ac[i] for i in range(s)) == F(1, 8)
        assert sum(w[i] * ac2[i] for i in range(s)) == F(1, 12)
        assert sum(w[i] * aac[i] for i in range(s)) == F(1, 24)
        if order == 5:
            assert sum(w[i] * C[i] ** 2 * ac[i] for i in range(s)) == F(1, 10)
            assert sum(w[i] * ac3[i] for i in range(s)) == F(1, 20)
            assert sum(w[i] * C[i] * aac[i] for i in range(s)) == F(1, 30)
            assert sum(w[i] * ac[i] ** 2 for i in range(s)) == F(1, 20)
            assert sum(w[i] * C[i] * ac2[i] for i in range(s)) == F(1, 15)
            a_ac2 = sum(w[i] * sum(a[i][j] * ac2[j] for j in range(s)) for i in range(s))
            assert a_ac2 == F(1, 60)
            a_cac = sum(w[i] * sum(a[i][j] * C[j] * ac[j] for j in range(s)) for i in range(s))
            assert a_cac == F(1, 40)
            a_aac = sum(w[i] * sum(a[i][j] * aac[j] for j in range(s)) for i in range(s))
            assert a_aac == F(1, 120)


def _fixed_error(h):
    # y' = y cos t, y(0) = 1: y = exp(sin t)
    st = rk.Dopri5(lambda t, y: y * math.cos(t), [1.0], rtol=1e-6, atol=1e-6, h0=h,
                   h_min=1e-12, h_max=1.0, max_steps=10 ** 6, fixed_step=True)
    assert st.advance(2.0) == "ok"
    return abs(st.y[0] - math.exp(math.sin(2.0)))


def test_fixed_step_global_error_is_fifth_order():
    e1, e2, e3 = _fixed_error(0.2), _fixed_error(0.1), _fixed_error(0.05)
    assert 22 < e1 / e2 < 44 and 22 < e2 / e3 < 44


def test_embedded_error_estimate_is_fifth_order_in_h():
    # one controlled step from the same state at h and h/2: err scales like h^5
    errs = []
    for h in (0.2, 0.1, 0.05):
        st = rk.Dopri5(lambda t, y: -y + np.sin(3 * t), [1.0, 2.0], rtol=1e-3, atol=1e-3, h0=h,
                       h_min=1e-12, h_max=10.0, max_steps=1)
        st.advance(h)
        errs.append(st.last_err)
    assert 20 < errs[0] / errs[1] < 48 and 20 < errs[1] / errs[2] < 48


@pytest.mark.parametrize("rtol", [1e-6, 1e-10])
def test_adaptive_reaches_closed_forms(rtol):
    st = rk.Dopri5(lambda t, y: np.array([-y[0], y[0] - 2 * y[1]]), [1.0, 0.0], rtol=rtol,
                   atol=rtol * 1e-2, h0=0.5, h_min=1e-12, h_max=1.0, max_steps=10 ** 5)
    assert st.advance(3.0) == "ok"
    exact = np.array([math.exp(-3), math.exp(-3) - math.exp(-6)])
    assert np.max(np.abs(st.y - exact)) <= 50 * rtol
    assert st.t == 3.0 and st.last_err <= 1.0


def test_large_first_step_is_rejected_and_shrunk():
    st = rk.Dopri5(lambda t, y: -50.0 * y, [1.0], rtol=1e-8, atol=1e-10, h0=1.0, h_min=1e-12,
                   h_max=1.0, max_steps=10 ** 5)
    assert st.advance(1.0) == "ok"
    assert st.rejected >= 1
    assert abs(st.y[0] - math.exp(-50.0)) <= 1e-8 * 1e-3 + 1e-10
    st2 = rk.Dopri5(lambda t, y: -50.0 * y, [1.0], rtol=1e-8, atol=1e-10, h0=1.0, h_min=0.5,
                    h_max=1.0, max_steps=10 ** 5)
    assert st2.advance(1.0) == "h_min"


def test_lpa_flow_matches_scipy_rk45():
    from scipy.integrate import solve_ivp

    # symmetric phase (positive masses), k from 1 to exp(-1.5); the floor follows k^2
    rho = wl.lpa_rho_grid(24)
    u0 = 0.3 + rho

    def f(t, u):
        k = math.exp(-t)
        return oracle.lpa_flow_rhs(rho, u, 16, 6.0, k=k, n_comp=4, m2_floor=-0.9 * k * k)

    st = rk.Dopri5(f, u0, rtol=1e-11, atol=1e-13, h0=1e-2, h_min=1e-12, h_max=1.0,
                   max_steps=10 ** 5)
    assert st.advance(1.5) == "ok"
    ref = solve_ivp(f, (0.0, 1.5), u0, method="RK45", rtol=1e-11, atol=1e-13)
    assert ref.success
    assert np.max(np.abs(st.y - ref.y[:, -1])) <= 1e-8 * np.max(np.abs(ref.y[:, -1]))


def test_abm4_weights_integrate_cubics_exactly():
    # AB4 over [t_n, t_n + 1] from f at t_n, t_n - 1, t_n - 2, t_n - 3 (unit step), AM4 from
    # t_n + 1, t_n, t_n - 1, t_n - 2: exact for every cubic (monomials 1, s, s^2, s^3)
    for k in range(4):
        exact = F(1, k + 1)  # int_0^1 s^k ds
        ab = sum(rk.AB4[j] * F(-j) ** k for j in range(4))
        am = rk.AM4[0] * F(1) ** k + sum(rk.AM4[j + 1] * F(-j) ** k for j in range(3))
        assert ab == exact and am == exact
    assert sum(rk.RK4_B) == 1


def test_abm4_exact_for_cubic_right_hand_sides():
    # y' = 1 + 2t - 3t^2 + 4t^3: the RK4 start (Simpson for y-independent f) and AB4/AM4 are
    # exact, including a shortened last step
    f = lambda t, y: np.array([1 + 2 * t - 3 * t * t + 4 * t ** 3])
    st = rk.Abm4(f, [0.5], h0=0.1, max_steps=1000)
    assert st.advance(1.95) == "ok"
    T = 1.95
    assert abs(st.y[0] - (0.5 + T + T * T - T ** 3 + T ** 4)) <= 1e-13
    assert st.accepted == 20 and st.t == T


def _abm_error(h):
    st = rk.Abm4(lambda t, y: y * math.cos(t), [1.0], h0=h, max_steps=10 ** 6)
    assert st.advance(2.0) == "ok"
    return abs(st.y[0] - math.exp(math.sin(2.0)))


def test_abm4_global_error_is_fourth_order():
    e1, e2, e3 = _abm_error(0.1), _abm_error(0.05), _abm_error(0.025)
    assert 11 < e1 / e2 < 22 and 11 < e2 / e3 < 22


def test_abm4_evaluation_count():
    # three RK4 start steps (the first evaluates f at t0 as well), then two evaluations per step
    st = rk.Abm4(lambda t, y: -y, [1.0], h0=0.1, max_steps=100)
    st.advance(1.0)
    assert st.accepted == 10 and st.evals == 1 + 3 * 4 + 7 * 2


def test_respace_is_exact_for_cubic_histories():
    # the history of f(t) = cubic at spacing h, moved to 0.37 h and 1.5 h, equals the cubic at
    # the new points
    cub = lambda t: 2.0 - 3.0 * t + 0.5 * t ** 2 + 0.25 * t ** 3
    h, tn = 0.3, 1.7
    hist = [np.array([cub(tn - j * h)]) for j in range(4)]
    for ratio in (0.37, 1.0, 1.5):
        got = rk.respace(hist, ratio)
        want = [cub(tn - j * ratio * h) for j in range(4)]
        assert np.allclose([g[0] for g in got], want, rtol=0, atol=1e-13), ratio


@pytest.mark.parametrize("rtol", [1e-6, 1e-10])
def test_variable_abm4_reaches_closed_forms(rtol):
    # a solution whose time scale grows: the step grows with it, accepted steps have err <= 1
    st = rk.Abm4Var(lambda t, y: np.array([-y[0], y[0] - 2 * y[1]]), [1.0, 0.0], rtol=rtol,
                    atol=rtol * 1e-2, h0=0.01, h_min=1e-12, h_max=1.0, max_steps=10 ** 5)
    assert st.advance(6.0) == "ok"
    exact = np.array([math.exp(-6), math.exp(-6) - math.exp(-12)])
    assert np.max(np.abs(st.y - exact)) <= 50 * rtol
    assert st.t == 6.0 and st.last_err <= 1.0
    assert st.h > 0.01  # it grew from h0


def test_variable_abm4_rejects_and_shrinks():
    # y' = -30 (y - cos t): a first multistep step of 0.1 is far outside the tolerance
    f = lambda t, y: -30.0 * (y - math.cos(t))
    st = rk.Abm4Var(f, [1.0], rtol=1e-8, atol=1e-10, h0=0.02, h_min=1e-10, h_max=0.5,
                    max_steps=10 ** 5)
    assert st.advance(2.0) == "ok"
    assert st.rejected >= 1
    # exact: y = (900 cos t + 30 sin t)/901 + (1 - 900/901) e^{-30 t}
    exact = (900 * math.cos(2.0) + 30 * math.sin(2.0)) / 901 + (1 / 901) * math.exp(-60.0)
    assert abs(st.y[0] - exact) <= 1e-6
    # evaluation count: f at the start point, then 4 per RK4 start step (three stages and the
    # new point), 2 per accepted multistep step (predicted and new point), 1 per rejection
    starts = 3
    assert st.evals == 1 + 4 * starts + 2 * (st.accepted - starts) + st.rejected
