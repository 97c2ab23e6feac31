"""GPU flow steppers (Dormand-Prince 5(4), Fehlberg 7(8), fixed- and variable-step ABM4) against the
oracle's steppers driving the oracle's right-hand sides at k(t) = Lambda exp(-t).

Both sides run the same algorithm; their right-hand sides differ by rounding only (1e-15
relative for the integrals, ~1e-13 for the LPA finite differences), so they take the same
accepted and rejected steps and end at states that agree to the accumulated rounding.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import stepper as rk
from paper_2412_13043_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2412_13043_amd import frg

    ctx = frg.Context(0)
    yield frg, ctx, torch
    torch.cuda.synchronize()
    ctx.close()


def _d(torch, a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), dtype=torch.float64,
                        device="cuda")


def _lpa_rhs(rho, n_q, q_max, lam, n_comp, floor, ft=None):
    def f(t, u):
        k = lam * math.exp(-t)
        fl = floor * (k / lam) ** 2
        if ft is None:
            return oracle.lpa_flow_rhs(rho, u, n_q, q_max, k=k, n_comp=n_comp, m2_floor=fl)
        d1, d2 = oracle.fd_derivatives(rho, u)
        ms = np.maximum(u + 2 * rho * d1, fl)
        mp = np.maximum(u, fl)
        Is = oracle.integrate_ft(oracle.LPA_T, n_q, q_max, k=k, m2=ms, **ft)
        Ip = oracle.integrate_ft(oracle.LPA_T, n_q, q_max, k=k, m2=mp, **ft)
        return 0.5 * (Is * (3 * d1 + 2 * rho * d2) + (n_comp - 1) * Ip * d1)
    return f


def _close(got, ref, tol):
    scale = np.abs(ref) + 1e-3 * np.max(np.abs(ref))
    return float(np.max(np.abs(got - ref) / scale)) <= tol


@pytest.mark.parametrize("fixed", [False, True])
def test_lpa_flow_stepper_matches_oracle(env, fixed):
    frg, ctx, torch = env
    rho = wl.lpa_rho_grid()
    u0 = 0.3 + rho
    lam = 1.0
    desc = frg.make_desc(frg.FRG_FAMILY_LPA, wl.LPA_NQ, wl.LPA_QMAX, k=lam)
    state, grid = _d(torch, u0), _d(torch, rho)
    cfg = dict(rtol=1e-8, atol=1e-10, h0=0.05, h_min=1e-8, h_max=0.5, max_steps=10000)
    st = ctx.stepper(desc, state, grid, n_comp=4, m2_floor=-0.9, fixed_step=fixed, **cfg)
    ref = rk.Dopri5(_lpa_rhs(rho, wl.LPA_NQ, wl.LPA_QMAX, lam, 4, -0.9), u0, fixed_step=fixed,
                    **cfg)
    for t_end in (0.4, 1.2):  # two calls: the stepper carries t, h and its first stage over
        rc, stats = st.advance(t_end)
        assert ref.advance(t_end) == "ok"
        assert stats.t == t_end
        assert (stats.accepted, stats.rejected) == (ref.accepted, ref.rejected)
        assert stats.rhs_evals == ref.evals
        assert _close(state.cpu().numpy(), ref.y, 1e-10), t_end
    st.close()


def test_two_point_flow_stepper_matches_oracle(env):
    frg, ctx, torch = env
    rng = np.random.default_rng(12)
    n = 48
    p = 10 ** rng.uniform(-2, 1, n)
    Z = wl.dressing_table(8)
    m0 = rng.uniform(0.2, 1.5, n)
    lam, coef, floor = 2.0, -3.0, -0.5
    desc = frg.make_desc(frg.FRG_FAMILY_TWO_POINT, 16, 10.0, n_x=8, k=lam)
    state, grid, tZ = _d(torch, m0), _d(torch, p), _d(torch, Z)
    cfg = dict(rtol=1e-9, atol=1e-11, h0=0.02, h_min=1e-8, h_max=0.5, max_steps=10000)
    st = ctx.stepper(desc, state, grid, Z=tZ, x_min=wl.Z_XMIN, x_max=wl.Z_XMAX,
                     m2_floor=floor, coef=coef, **cfg)

    def f(t, m):
        k = lam * math.exp(-t)
        fl = floor * (k / lam) ** 2
        return coef * oracle.integrate(2, 16, 10.0, n_x=8, k=k, ext=p, m2=np.maximum(m, fl),
                                       Z=Z)

    ref = rk.Dopri5(f, m0, **cfg)
    rc, stats = st.advance(1.0)
    assert ref.advance(1.0) == "ok"
    assert (stats.accepted, stats.rejected) == (ref.accepted, ref.rejected)
    got = state.cpu().numpy()
    assert np.max(np.abs(got - ref.y) / np.abs(ref.y)) <= 1e-11
    st.close()


def test_finite_temperature_three_point_flow_stepper_matches_oracle(env):
    # the three-point vertex flow at finite temperature (state m2 per (p, alpha) point, each
    # inner leg with its own frequency shift), the frequency rule rebuilt at every stage's k
    frg, ctx, torch = env
    rng = np.random.default_rng(14)
    n = 24
    p = 10 ** rng.uniform(-2, 1, n)
    alpha = rng.uniform(0.0, math.pi, n)
    p01 = 2 * math.pi * 0.2 * rng.integers(-1, 2, n)
    p02 = 2 * math.pi * 0.2 * rng.integers(-1, 2, n)
    Z = wl.dressing_table(9)
    m0 = rng.uniform(0.2, 1.5, n)
    lam, coef, floor = 1.5, 4.0, -0.5
    ft = dict(T=0.2, freq_max=4.0, statistics=0, n_tail=3)
    desc = frg.make_desc(frg.FRG_FAMILY_THREE_POINT_T, 8, 8.0, n_x=5, n_phi=4, k=lam, **ft)
    state = _d(torch, m0)
    grid, tZ = _d(torch, np.concatenate([p, alpha, p01, p02])), _d(torch, Z)
    cfg = dict(rtol=1e-9, atol=1e-11, h0=0.02, h_min=1e-8, h_max=0.5, max_steps=10000)
    st = ctx.stepper(desc, state, grid, Z=tZ, x_min=wl.Z_XMIN, x_max=wl.Z_XMAX,
                     m2_floor=floor, coef=coef, **cfg)

    def f(t, m):
        k = lam * math.exp(-t)
        fl = floor * (k / lam) ** 2
        return coef * oracle.integrate_ft(oracle.THREE_POINT_T, 8, 8.0, n_x=5, n_phi=4, k=k,
                                          ext=(p, alpha, p01, p02), m2=np.maximum(m, fl), Z=Z,
                                          **ft)

    ref = rk.Dopri5(f, m0, **cfg)
    rc, stats = st.advance(0.6)
    assert ref.advance(0.6) == "ok"
    assert (stats.accepted, stats.rejected) == (ref.accepted, ref.rejected)
    got = state.cpu().numpy()
    assert np.max(np.abs(got - ref.y) / np.abs(ref.y)) <= 1e-11
    st.close()


def test_finite_temperature_lpa_stepper_with_k_scaled_frequencies(env):
    # x0 frequency domain: Lambda_w = 6 k shrinks with k, so the number of Matsubara
    # frequencies changes during the run
    frg, ctx, torch = env
    rho = wl.lpa_rho_grid(32)
    u0 = 0.4 + 0.8 * rho
    lam = 1.0
    ft = dict(T=0.12, freq_max=6.0, freq_scaled=True, statistics=0, n_tail=4)
    desc = frg.make_desc(frg.FRG_FAMILY_LPA_T, 24, 6.0, k=lam, **ft)
    state, grid = _d(torch, u0), _d(torch, rho)
    cfg = dict(rtol=1e-8, atol=1e-10, h0=0.05, h_min=1e-8, h_max=0.5, max_steps=10000)
    st = ctx.stepper(desc, state, grid, n_comp=4, m2_floor=-0.9, **cfg)
    ref = rk.Dopri5(_lpa_rhs(rho, 24, 6.0, lam, 4, -0.9, ft=ft), u0, **cfg)
    rc, stats = st.advance(1.0)
    assert ref.advance(1.0) == "ok"
    assert (stats.accepted, stats.rejected) == (ref.accepted, ref.rejected)
    assert _close(state.cpu().numpy(), ref.y, 1e-10)
    st.close()


def test_abm4_stepper_matches_oracle(env):
    # Adams-Bashforth-Moulton 4 PECE, steps of h0: RK4 start, then two right-hand sides per
    # step; the second call ends with a shortened RK4 step and restarts the history
    frg, ctx, torch = env
    rho = wl.lpa_rho_grid()
    u0 = 0.3 + rho
    desc = frg.make_desc(frg.FRG_FAMILY_LPA, wl.LPA_NQ, wl.LPA_QMAX, k=1.0)
    state, grid = _d(torch, u0), _d(torch, rho)
    st = ctx.stepper(desc, state, grid, n_comp=4, m2_floor=-0.9, h0=0.05, max_steps=10000,
                     method=1)
    ref = rk.Abm4(_lpa_rhs(rho, wl.LPA_NQ, wl.LPA_QMAX, 1.0, 4, -0.9), u0, h0=0.05,
                  max_steps=10000)
    for t_end in (0.4, 1.23, 1.5):
        rc, stats = st.advance(t_end)
        assert ref.advance(t_end) == "ok"
        assert stats.t == t_end and stats.accepted == ref.accepted
        assert stats.rhs_evals == ref.evals and stats.rejected == 0
        assert _close(state.cpu().numpy(), ref.y, 1e-10), t_end
    st.close()
    # two-point vertex flow
    rng = np.random.default_rng(21)
    p = 10 ** rng.uniform(-2, 1, 40)
    Z = wl.dressing_table(8)
    m0 = rng.uniform(0.2, 1.5, 40)
    d2 = frg.make_desc(frg.FRG_FAMILY_TWO_POINT, 16, 10.0, n_x=8, k=2.0)
    state, tp, tZ = _d(torch, m0), _d(torch, p), _d(torch, Z)
    st = ctx.stepper(d2, state, tp, Z=tZ, x_min=wl.Z_XMIN, x_max=wl.Z_XMAX, m2_floor=-0.5,
                     coef=-3.0, h0=0.1, max_steps=1000, method=1)

    def f(t, m):
        k = 2.0 * math.exp(-t)
        return -3.0 * oracle.integrate(2, 16, 10.0, n_x=8, k=k, ext=p,
                                       m2=np.maximum(m, -0.5 * (k / 2.0) ** 2), Z=Z)

    ref = rk.Abm4(f, m0, h0=0.1, max_steps=1000)
    rc, stats = st.advance(0.95)
    assert ref.advance(0.95) == "ok"
    assert stats.rhs_evals == ref.evals
    assert np.max(np.abs(state.cpu().numpy() - ref.y) / np.abs(ref.y)) <= 1e-11
    st.close()
    with pytest.raises(frg.FrgError) as ei:
        ctx.stepper(desc, _d(torch, u0), grid, h0=0.05, method=4)
    assert ei.value.status == frg.FRG_E_INVAL


def test_variable_abm4_stepper_matches_oracle(env):
    # variable-step ABM4: RK4 start, Milne's estimate, re-spaced history; the same accepted and
    # rejected steps and right-hand sides as the oracle's on the LPA flow (two calls, the
    # second ending with a shortened step) and on a two-point vertex flow
    frg, ctx, torch = env
    rho = wl.lpa_rho_grid()
    u0 = 0.3 + rho
    desc = frg.make_desc(frg.FRG_FAMILY_LPA, wl.LPA_NQ, wl.LPA_QMAX, k=1.0)
    state, grid = _d(torch, u0), _d(torch, rho)
    cfg = dict(rtol=1e-8, atol=1e-10, h0=0.01, h_min=1e-8, h_max=0.5, max_steps=10000)
    st = ctx.stepper(desc, state, grid, n_comp=4, m2_floor=-0.9, method=3, **cfg)
    ref = rk.Abm4Var(_lpa_rhs(rho, wl.LPA_NQ, wl.LPA_QMAX, 1.0, 4, -0.9), u0, **cfg)
    for t_end in (0.5, 2.0):
        rc, stats = st.advance(t_end)
        assert ref.advance(t_end) == "ok"
        assert stats.t == t_end
        assert (stats.accepted, stats.rejected, stats.rhs_evals) == (ref.accepted,
                                                                     ref.rejected, ref.evals)
        assert _close(state.cpu().numpy(), ref.y, 1e-10), t_end
    assert ref.h > 0.01  # the step grew
    st.close()
    rng = np.random.default_rng(41)
    p = 10 ** rng.uniform(-2, 1, 40)
    Z = wl.dressing_table(10)
    m0 = rng.uniform(0.2, 1.5, 40)
    d2 = frg.make_desc(frg.FRG_FAMILY_TWO_POINT, 16, 10.0, n_x=8, k=2.0)
    state, tp, tZ = _d(torch, m0), _d(torch, p), _d(torch, Z)
    cfg = dict(rtol=1e-9, atol=1e-11, h0=0.02, h_min=1e-8, h_max=0.5, max_steps=1000)
    st = ctx.stepper(d2, state, tp, Z=tZ, x_min=wl.Z_XMIN, x_max=wl.Z_XMAX, m2_floor=-0.5,
                     coef=-3.0, method=3, **cfg)

    def f(t, m):
        k = 2.0 * math.exp(-t)
        return -3.0 * oracle.integrate(2, 16, 10.0, n_x=8, k=k, ext=p,
                                       m2=np.maximum(m, -0.5 * (k / 2.0) ** 2), Z=Z)

    ref = rk.Abm4Var(f, m0, **cfg)
    rc, stats = st.advance(1.0)
    assert ref.advance(1.0) == "ok"
    assert (stats.accepted, stats.rejected, stats.rhs_evals) == (ref.accepted, ref.rejected,
                                                                 ref.evals)
    assert np.max(np.abs(state.cpu().numpy() - ref.y) / np.abs(ref.y)) <= 1e-10
    st.close()


@pytest.mark.parametrize("fixed", [False, True])
def test_rkf78_stepper_matches_oracle(env, fixed):
    # Fehlberg 7(8): 13 right-hand sides per attempt, the first kept over a rejection; the
    # same accepted and rejected steps as the oracle's, two calls on the LPA flow, then a
    # two-point vertex flow
    frg, ctx, torch = env
    rho = wl.lpa_rho_grid()
    u0 = 0.3 + rho
    desc = frg.make_desc(frg.FRG_FAMILY_LPA, wl.LPA_NQ, wl.LPA_QMAX, k=1.0)
    state, grid = _d(torch, u0), _d(torch, rho)
    # adaptive: a first step of 0.3 (rejected); fixed: steps of 0.05, where explicit steps of
    # the LPA flow do not amplify the two sides' rounding differences
    cfg = dict(rtol=1e-10, atol=1e-12, h0=0.05 if fixed else 0.3, h_min=1e-8, h_max=1.0,
               max_steps=10000)
    st = ctx.stepper(desc, state, grid, n_comp=4, m2_floor=-0.9, fixed_step=fixed, method=2,
                     **cfg)
    ref = rk.Rkf78(_lpa_rhs(rho, wl.LPA_NQ, wl.LPA_QMAX, 1.0, 4, -0.9), u0, fixed_step=fixed,
                   **cfg)
    for t_end in (0.5, 2.0):
        rc, stats = st.advance(t_end)
        assert ref.advance(t_end) == "ok"
        assert stats.t == t_end
        assert (stats.accepted, stats.rejected) == (ref.accepted, ref.rejected)
        assert stats.rhs_evals == ref.evals
        assert _close(state.cpu().numpy(), ref.y, 1e-10), t_end
    st.close()
    rng = np.random.default_rng(31)
    p = 10 ** rng.uniform(-2, 1, 40)
    Z = wl.dressing_table(9)
    m0 = rng.uniform(0.2, 1.5, 40)
    d2 = frg.make_desc(frg.FRG_FAMILY_TWO_POINT, 16, 10.0, n_x=8, k=2.0)
    state, tp, tZ = _d(torch, m0), _d(torch, p), _d(torch, Z)
    cfg = dict(rtol=1e-10, atol=1e-12, h0=0.1, h_min=1e-8, h_max=0.5, max_steps=1000)
    st = ctx.stepper(d2, state, tp, Z=tZ, x_min=wl.Z_XMIN, x_max=wl.Z_XMAX, m2_floor=-0.5,
                     coef=-3.0, fixed_step=fixed, method=2, **cfg)

    def f(t, m):
        k = 2.0 * math.exp(-t)
        return -3.0 * oracle.integrate(2, 16, 10.0, n_x=8, k=k, ext=p,
                                       m2=np.maximum(m, -0.5 * (k / 2.0) ** 2), Z=Z)

    ref = rk.Rkf78(f, m0, fixed_step=fixed, **cfg)
    rc, stats = st.advance(1.0)
    assert ref.advance(1.0) == "ok"
    assert (stats.accepted, stats.rejected, stats.rhs_evals) == (ref.accepted, ref.rejected,
                                                                 ref.evals)
    assert np.max(np.abs(state.cpu().numpy() - ref.y) / np.abs(ref.y)) <= 1e-11
    st.close()


def test_abm4_finite_temperature_lpa_flow(env):
    # ABM4 on the finite-temperature LPA flow with a k-scaled frequency domain (the frequency
    # count changes during the run) against the oracle's ABM4 on the oracle's right-hand side
    frg, ctx, torch = env
    rho = wl.lpa_rho_grid(32)
    u0 = 0.4 + 0.8 * rho
    ft = dict(T=0.12, freq_max=6.0, freq_scaled=True, statistics=0, n_tail=4)
    desc = frg.make_desc(frg.FRG_FAMILY_LPA_T, 24, 6.0, k=1.0, **ft)
    state, grid = _d(torch, u0), _d(torch, rho)
    st = ctx.stepper(desc, state, grid, n_comp=4, m2_floor=-0.9, h0=0.04, max_steps=10000,
                     method=1)
    ref = rk.Abm4(_lpa_rhs(rho, 24, 6.0, 1.0, 4, -0.9, ft=ft), u0, h0=0.04, max_steps=10000)
    rc, stats = st.advance(0.9)
    assert ref.advance(0.9) == "ok"
    assert (stats.accepted, stats.rhs_evals) == (ref.accepted, ref.evals)
    assert _close(state.cpu().numpy(), ref.y, 1e-10)
    st.close()


def test_stepper_limits_and_errors(env):
    frg, ctx, torch = env
    rho = wl.lpa_rho_grid()
    desc = frg.make_desc(frg.FRG_FAMILY_LPA, 16, 6.0)
    state, grid = _d(torch, 0.3 + rho), _d(torch, rho)
    for bad in [dict(rtol=0.0), dict(atol=-1.0), dict(h0=0.0), dict(h_min=0.0),
                dict(h_min=1.0, h_max=0.5), dict(max_steps=0), dict(h_max=float("inf"))]:
        kw = dict(rtol=1e-8, atol=1e-10, h0=0.05, h_min=1e-8, h_max=0.5, max_steps=100)
        kw.update(bad)
        with pytest.raises(frg.FrgError) as ei:
            ctx.stepper(desc, state, grid, **kw)
        assert ei.value.status == frg.FRG_E_INVAL, bad
    # max_steps: stops early with FRG_E_TIMEOUT, the state valid at stats.t
    u0 = 0.3 + rho
    st = ctx.stepper(desc, state, grid, rtol=1e-8, atol=1e-10, h0=0.01, h_min=1e-8, h_max=0.01,
                     max_steps=5)
    rc, stats = st.advance(1.0, ok=(frg.FRG_OK, frg.FRG_E_TIMEOUT))
    assert rc == frg.FRG_E_TIMEOUT and stats.accepted == 5 and abs(stats.t - 0.05) < 1e-12
    ref = rk.Dopri5(_lpa_rhs(rho, 16, 6.0, 1.0, 4, -0.9), u0, rtol=1e-8, atol=1e-10, h0=0.01,
                    h_min=1e-8, h_max=0.01, max_steps=5)
    assert ref.advance(1.0) == "max_steps"
    assert _close(state.cpu().numpy(), ref.y, 1e-11)
    with pytest.raises(frg.FrgError):
        st.advance(0.01)  # before the current t
    st.close()
