"""Pins of the oracle's Runge-Kutta-Fehlberg 7(8) stepper (CPU only).

* The tableau against the Butcher order conditions themselves: for every rooted tree t with up
  to 8 vertices (200 trees, enumerated here) the elementary weight sum_i b_i Phi_i(t) equals
  1/gamma(t) in exact rational arithmetic -- for the eighth-order weights up to order 8, for
  the seventh-order weights up to order 7 and not for every tree of order 8.  A mistyped
  coefficient breaks some condition of low order.
* Row sums equal the nodes; the error weights are 41/840 on stages 1, 11, 12, 13 (signs - - + +).
* Fixed-step global errors on closed-form solutions fall as h^8 and the error estimate of one
  step as h^8 (it is dominated by the seventh-order solution's error).
* Adaptive runs reach closed forms within the tolerance, and scipy's solve_ivp(method="DOP853")
  (a library eighth-order Dormand-Prince pair with its own controller) reaches the same state
  of the oracle's LPA flow.
"""
import math
from fractions import Fraction as F
from functools import lru_cache

import numpy as np
import pytest

import oracle
from oracle import stepper as rk
from paper_2412_13043_amd import workloads as wl


@lru_cache(maxsize=None)
def _trees(n):
    """Rooted trees with n vertices, each a sorted tuple of its subtrees (canonical form)."""
    if n == 1:
        return ((),)
    smaller = [t for m in range(1, n) for t in _trees(m)]
    order = {t: _order(t) for t in smaller}
    out = set()

    def grow(start, left, kids):
        if left == 0:
            out.add(tuple(sorted(kids)))
            return
        for i in range(start, len(smaller)):
            t = smaller[i]
            if order[t] <= left:
                grow(i, left - order[t], kids + [t])

    grow(0, n - 1, [])
    return tuple(sorted(out))


def _order(t):
    return 1 + sum(_order(c) for c in t)


def _gamma(t):
    g = _order(t)
    for c in t:
        g *= _gamma(c)
    return g


def _weights(a, s):
    memo = {}

    def phi(t):
        # Phi_i(t) for every stage i: the product over subtrees of sum_j a_ij Phi_j(subtree)
        if t in memo:
            return memo[t]
        v = [F(1)] * s
        for c in t:
            pc = phi(c)
            v = [v[i] * sum(a[i][j] * pc[j] for j in range(s)) for i in range(s)]
        memo[t] = v
        return v
    return phi


def test_tree_counts():
    assert [len(_trees(n)) for n in range(1, 9)] == [1, 1, 2, 4, 9, 20, 48, 115]


def test_tableau_satisfies_every_order_condition():
    s = 13
    a = [[rk.A78[i][j] if j < len(rk.A78[i]) else F(0) for j in range(s)] for i in range(s)]
    for i in range(s):
        assert sum(a[i]) == rk.C78[i], i
    phi = _weights(a, s)
    failed7_at8 = 0
    for n in range(1, 9):
        for t in _trees(n):
            want = F(1, _gamma(t))
            w8 = sum(rk.B8[i] * phi(t)[i] for i in range(s))
            w7 = sum(rk.B7[i] * phi(t)[i] for i in range(s))
            assert w8 == want, (n, t)
            if n <= 7:
                assert w7 == want, (n, t)
            else:
                failed7_at8 += w7 != want
    assert failed7_at8 > 0
    e = [rk.B8[i] - rk.B7[i] for i in range(s)]
    assert e == [F(-41, 840)] + [F(0)] * 9 + [F(-41, 840), F(41, 840), F(41, 840)]


def _fixed_error(h):
    # y1' = -y2, y2' = y1, y3' = -y3^2, y4' = y4 cos t: (cos t, sin t, 1/(1 + t), exp(sin t))
    f = lambda t, y: np.array([-y[1], y[0], -y[2] ** 2, math.cos(t) * y[3]])
    st = rk.Rkf78(f, [1.0, 0.0, 1.0, 1.0], rtol=1e-6, atol=1e-6, h0=h, h_min=1e-12, h_max=2.0,
                  max_steps=10 ** 6, fixed_step=True)
    assert st.advance(4.0) == "ok"
    T = 4.0
    return float(np.max(np.abs(st.y - [math.cos(T), math.sin(T), 1 / (1 + T),
                                       math.exp(math.sin(T))])))


def test_fixed_step_global_error_is_eighth_order():
    e1, e2 = _fixed_error(0.8), _fixed_error(0.4)
    # 2^8 = 256 asymptotically; 2^7.5 = 181 at these step sizes
    assert e1 / e2 > 181


def test_error_estimate_is_eighth_order_in_h():
    # y' = -y: the estimate of one step is 41/840 h (k1 + k11 - k12 - k13) = C h^8 y (1 + O(h))
    # with C != 0, so halving h divides it by 2^8 = 256 (nonlinear problems approach the same
    # ratio from further away at these step sizes)
    errs = []
    for h in (0.2, 0.1):
        st = rk.Rkf78(lambda t, y: -y, [1.0], rtol=0.0, atol=1.0, h0=h, h_min=1e-12, h_max=1.0,
                      max_steps=10)
        st.advance(h)
        errs.append(st.last_err)
    assert 245 < errs[0] / errs[1] < 270


@pytest.mark.parametrize("rtol", [1e-6, 1e-11])
def test_adaptive_reaches_closed_forms(rtol):
    st = rk.Rkf78(lambda t, y: np.array([-y[0], y[0] - 2 * y[1]]), [1.0, 0.0], rtol=rtol,
                  atol=rtol * 1e-2, h0=0.5, h_min=1e-12, h_max=1.0, max_steps=10 ** 5)
    assert st.advance(3.0) == "ok"
    exact = np.array([math.exp(-3), math.exp(-3) - math.exp(-6)])
    assert np.max(np.abs(st.y - exact)) <= 50 * rtol
    assert st.t == 3.0 and st.last_err <= 1.0
    assert st.evals == 13 * (st.accepted + st.rejected) - st.rejected


def test_lpa_flow_matches_scipy_dop853():
    from scipy.integrate import solve_ivp

    rho = wl.lpa_rho_grid(24)
    u0 = 0.3 + rho

    def f(t, u):
        k = math.exp(-t)
        return oracle.lpa_flow_rhs(rho, u, 16, 6.0, k=k, n_comp=4, m2_floor=-0.9 * k * k)

    st = rk.Rkf78(f, u0, rtol=1e-11, atol=1e-13, h0=1e-2, h_min=1e-12, h_max=1.0,
                  max_steps=10 ** 5)
    assert st.advance(1.5) == "ok"
    ref = solve_ivp(f, (0.0, 1.5), u0, method="DOP853", rtol=1e-11, atol=1e-13)
    assert ref.success
    assert np.max(np.abs(st.y - ref.y[:, -1])) <= 1e-8 * np.max(np.abs(ref.y[:, -1]))
