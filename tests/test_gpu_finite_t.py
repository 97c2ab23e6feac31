"""GPU parity of the finite-temperature families (Matsubara sum x spatial quadrature) against the
FP64 oracle, through the C ABI.

Tolerance as for the vacuum families: 1e-12 relative per external point in float64, the stated
bound per result in the float32 form, bitwise equality across tile shapes, fused launches and
flow right-hand-side modes.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2412_13043_amd import workloads as wl

pytestmark = pytest.mark.gpu
TOL = 1e-12


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


def _rel(got, ref):
    return float(np.max(np.abs(got - ref) / np.abs(ref)))


def _n_freq(stat, T, lam, n_tail):
    return len(oracle.matsubara_rule(stat, T, lam, n_tail)[0])


def _run(env, desc, n_ext, *, ext=None, m2=None, m2_scalar=0.0, Z=None, err=False, ctx=None):
    frg, ctx0, torch = env
    c = ctx or ctx0
    out = torch.full((n_ext,), float("nan"), dtype=torch.float64, device="cuda")
    eo = torch.full((n_ext,), float("nan"), dtype=torch.float64, device="cuda") if err else None
    c.integrate(desc, out, ext=None if ext is None else _d(torch, ext),
                m2=None if m2 is None else _d(torch, m2), m2_scalar=m2_scalar,
                Z=None if Z is None else _d(torch, Z), x_min=wl.Z_XMIN, x_max=wl.Z_XMAX,
                err_out=eo)
    torch.cuda.synchronize()
    if err:
        return out.cpu().numpy(), eo.cpu().numpy()
    return out.cpu().numpy()


# ------------------------------------------------------------------------------------------
# LPA at finite temperature
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("stat", [0, 1])
@pytest.mark.parametrize("T,lam,n_tail,scaled,k", [(0.1, 10.0, 8, False, 1.0),
                                                   (0.5, 4.0, 0, False, 1.0),
                                                   (0.05, 3.0, 16, True, 1.7),
                                                   (2.0, 13.0, 1, False, 0.6)])
def test_lpa_ft_parity(env, stat, T, lam, n_tail, scaled, k):
    frg = env[0]
    rho, u, m2 = wl.lpa_potential()
    m2 = m2 * k * k
    desc = frg.make_desc(frg.FRG_FAMILY_LPA_T, wl.LPA_NQ, wl.LPA_QMAX, k=k, T=T, freq_max=lam,
                         statistics=stat, n_tail=n_tail, freq_scaled=scaled)
    got = _run(env, desc, m2.size, m2=m2)
    ref = oracle.integrate_ft(oracle.LPA_T, wl.LPA_NQ, wl.LPA_QMAX, k=k, T=T, statistics=stat,
                              freq_max=lam, freq_scaled=scaled, n_tail=n_tail, m2=m2)
    assert _rel(got, ref) <= TOL


def test_lpa_ft_fp32_within_bound(env):
    frg = env[0]
    rho, u, m2 = wl.lpa_batch(8)
    m2 = m2.reshape(-1)
    kw = dict(T=0.2, freq_max=8.0, statistics=0, n_tail=4)
    desc = frg.make_desc(frg.FRG_FAMILY_LPA_T, wl.LPA_NQ, wl.LPA_QMAX, precision=1,
                         near_pole_tau=0.1, **kw)
    got, err = _run(env, desc, m2.size, m2=m2, err=True)
    ref = oracle.integrate_ft(oracle.LPA_T, wl.LPA_NQ, wl.LPA_QMAX, m2=m2, **kw)
    rel = np.abs(got - ref) / np.abs(ref)
    assert np.all(rel <= err) and np.all(err < 1e-4)


# ------------------------------------------------------------------------------------------
# Two-point at finite temperature
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("stat", [0, 1])
@pytest.mark.parametrize("n_ext,n_q,n_x,T,lam,n_tail,useZ", [
    (37, 13, 6, 0.2, 6.0, 4, True),     # ragged external tile and cos1 rounds
    (1, 1, 1, 1.0, 7.0, 0, False),      # smallest: one point, one node per dimension
    (130, 24, 16, 0.05, 2.0, 8, True),  # many frequencies
    (64, 64, 32, 0.1, 10.0, 8, True),   # the benchmark's node counts
])
def test_two_point_ft_parity(env, stat, n_ext, n_q, n_x, T, lam, n_tail, useZ):
    frg = env[0]
    rng = np.random.default_rng(100 + n_ext + stat)
    p = 10 ** rng.uniform(-3, 2, n_ext)
    if stat == 0:
        p0 = 2 * math.pi * T * rng.integers(-2, 3, n_ext)
    else:
        p0 = np.full(n_ext, math.pi * T * math.exp(-1.0 / (math.pi * T)))
    m2 = rng.uniform(-0.5, 2.0, n_ext)
    Z = wl.dressing_table(9) if useZ else None
    desc = frg.make_desc(frg.FRG_FAMILY_TWO_POINT_T, n_q, 10.0, n_x=n_x, T=T, freq_max=lam,
                         statistics=stat, n_tail=n_tail)
    got = _run(env, desc, n_ext, ext=np.concatenate([p, p0]), m2=m2, Z=Z)
    ref = oracle.integrate_ft(oracle.TWO_POINT_T, n_q, 10.0, n_x=n_x, T=T, statistics=stat,
                              freq_max=lam, n_tail=n_tail, ext=(p, p0), m2=m2, Z=Z)
    assert _rel(got, ref) <= TOL


@pytest.mark.parametrize("stat,k,scaled", [(0, 1.7, True), (1, 0.45, False), (1, 2.3, True)])
def test_two_point_ft_scale_and_scaled_domain(env, stat, k, scaled):
    frg = env[0]
    rng = np.random.default_rng(200 + stat)
    n = 45
    p = k * 10 ** rng.uniform(-3, 2, n)
    p0 = rng.uniform(-1.0, 1.0, n) * k
    m2 = rng.uniform(-0.4, 1.5, n) * k * k
    Z = wl.dressing_table(11)
    kw = dict(T=0.15 * k, statistics=stat, freq_max=5.0 if scaled else 5.0 * k, n_tail=5)
    desc = frg.make_desc(frg.FRG_FAMILY_TWO_POINT_T, 20, 8.0, n_x=10, k=k, freq_scaled=scaled,
                         **kw)
    got = _run(env, desc, n, ext=np.concatenate([p, p0]), m2=m2, Z=Z)
    ref = oracle.integrate_ft(oracle.TWO_POINT_T, 20, 8.0, n_x=10, k=k, freq_scaled=scaled,
                              ext=(p, p0), m2=m2, Z=Z, **kw)
    assert _rel(got, ref) <= TOL


@pytest.mark.parametrize("tau", [0.0, 0.1])
def test_two_point_ft_fp32_within_bound(env, tau):
    frg = env[0]
    n = 96
    rng = np.random.default_rng(5)
    p = 10 ** rng.uniform(-3, 2, n)
    p0 = 2 * math.pi * 0.1 * rng.integers(-1, 2, n)
    m2 = rng.uniform(-0.9, -0.5, n)  # close to the pole at the lowest frequency
    Z = wl.dressing_table(3)
    kw = dict(T=0.1, freq_max=5.0, statistics=0, n_tail=4)
    desc = frg.make_desc(frg.FRG_FAMILY_TWO_POINT_T, 32, 10.0, n_x=16, precision=1,
                         near_pole_tau=tau, **kw)
    got, err = _run(env, desc, n, ext=np.concatenate([p, p0]), m2=m2, Z=Z, err=True)
    ref = oracle.integrate_ft(oracle.TWO_POINT_T, 32, 10.0, n_x=16, ext=(p, p0), m2=m2, Z=Z,
                              **kw)
    rel = np.abs(got - ref) / np.abs(ref)
    assert np.all(rel <= err), (rel / err).max()
    assert np.all(err < 1e-3)


@pytest.mark.parametrize("precision", [0, 1])
def test_two_point_ft_tile_shapes_give_identical_bits(env, tmp_path, monkeypatch, precision):
    # the tile shape is looked up under the vacuum key (family 2, n_q n_f radial nodes)
    frg, _, torch = env
    n_q, n_x, n = 5, 6, 37
    kw = dict(T=0.3, freq_max=4.0, statistics=1, n_tail=2)
    n_f = _n_freq(1, 0.3, 4.0, 2)
    rng = np.random.default_rng(77)
    p = 10 ** rng.uniform(-3, 2, n)
    p0 = np.full(n, 0.2)
    m2 = rng.uniform(-0.3, 2.0, n)
    Z = wl.dressing_table(7)
    desc = frg.make_desc(frg.FRG_FAMILY_TWO_POINT_T, n_q, 10.0, n_x=n_x, precision=precision,
                         near_pole_tau=0.1 if precision else 0.0, **kw)
    target = 16 * torch.cuda.get_device_properties(0).multi_processor_count
    nq_eff = n_q * n_f
    shapes = [(0, 1, 0), (0, 7, 0), (2, 1, 0), (3, 2, 0), (6, 1, 0), (0, 1, 2), (2, 1, 3),
              (1, 4, 2)]
    results = []
    for lq, ch, lx in shapes:
        cache = tmp_path / f"ft_{lq}_{ch}_{lx}.txt"
        cache.write_text(f"2 {precision} {nq_eff} {n_x} 0 {n} {target} {lq} {ch} {lx}\n")
        monkeypatch.setenv("FRG_AUTOTUNE_CACHE", str(cache))
        ctx = frg.Context(0)
        try:
            results.append(_run(env, desc, n, ext=np.concatenate([p, p0]), m2=m2, Z=Z, err=True,
                                ctx=ctx))
        finally:
            torch.cuda.synchronize()
            ctx.close()
    for (o, e), shape in zip(results[1:], shapes[1:]):
        assert np.array_equal(o, results[0][0]), shape
        assert np.array_equal(e, results[0][1]), shape
    if precision == 0:
        ref = oracle.integrate_ft(oracle.TWO_POINT_T, n_q, 10.0, n_x=n_x, ext=(p, p0), m2=m2,
                                  Z=Z, **kw)
        assert _rel(results[0][0], ref) <= TOL


def test_maximum_frequency_rule(env):
    # n_q n_f at the limit FRG_MAX_FT_NODES: 64 radial nodes x 1024 frequencies
    frg = env[0]
    T, lam, n_tail = 0.01, 2 * math.pi * 0.01 * 404.5, 107  # 809 explicit + 214 tail = 1023
    n_f = _n_freq(0, T, lam, n_tail)
    assert n_f == 1023 and 64 * n_f <= frg.FRG_MAX_FT_NODES
    m2 = np.array([0.1, 1.0, 3.0])
    desc = frg.make_desc(frg.FRG_FAMILY_LPA_T, 64, 6.0, T=T, freq_max=lam, n_tail=n_tail)
    got = _run(env, desc, 3, m2=m2)
    ref = oracle.integrate_ft(oracle.LPA_T, 64, 6.0, T=T, freq_max=lam, n_tail=n_tail, m2=m2)
    assert _rel(got, ref) <= TOL
    p, p0 = np.array([0.3, 4.0]), np.array([0.0, 2 * math.pi * T])
    desc = frg.make_desc(frg.FRG_FAMILY_TWO_POINT_T, 64, 6.0, n_x=2, T=T, freq_max=lam,
                         n_tail=n_tail)
    got = _run(env, desc, 2, ext=np.concatenate([p, p0]), m2_scalar=0.4)
    ref = oracle.integrate_ft(oracle.TWO_POINT_T, 64, 6.0, n_x=2, T=T, freq_max=lam,
                              n_tail=n_tail, ext=(p, p0), m2_scalar=0.4, n_ext=2)
    assert _rel(got, ref) <= TOL


def test_ft_invalid_descriptors_rejected(env):
    frg, ctx, torch = env
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    ext = torch.ones(8, dtype=torch.float64, device="cuda")
    good = dict(n_x=4, T=0.2, freq_max=3.0, n_tail=2)
    for kw in [dict(T=0.0), dict(freq_max=0.0), dict(statistics=3), dict(n_tail=-2),
               dict(statistics=1, T=2.0, freq_max=1.0), dict(T=1e-5, freq_max=1.0)]:
        args = dict(good)
        args.update(kw)
        desc = frg.make_desc(frg.FRG_FAMILY_TWO_POINT_T, 8, 6.0, **args)
        with pytest.raises(frg.FrgError) as ei:
            ctx.integrate(desc, out, ext=ext, m2_scalar=0.5)
        assert ei.value.status == frg.FRG_E_INVAL, kw
    desc = frg.make_desc(frg.FRG_FAMILY_TWO_POINT_T, 8, 6.0, **good)
    with pytest.raises(frg.FrgError):  # two-point needs (p, p0)
        ctx.integrate(desc, out, m2_scalar=0.5)


# ------------------------------------------------------------------------------------------
# Fused launches, the benchmark's shape and flows
# ------------------------------------------------------------------------------------------
def test_multi_mixes_finite_and_zero_temperature_bitwise(env):
    frg, ctx, torch = env
    rng = np.random.default_rng(21)
    n = 50
    p = 10 ** rng.uniform(-3, 2, n)
    p0 = np.zeros(n)
    Z = wl.dressing_table(4)
    m2 = rng.uniform(-0.3, 1.5, n)
    cases = [
        (frg.make_desc(frg.FRG_FAMILY_TWO_POINT_T, 16, 10.0, n_x=8, T=0.2, freq_max=6.0,
                       n_tail=4), np.concatenate([p, p0 + 0.4])),
        (frg.make_desc(frg.FRG_FAMILY_TWO_POINT, 16, 10.0, n_x=8), p),
        (frg.make_desc(frg.FRG_FAMILY_LPA_T, 32, 6.0, T=0.3, freq_max=5.0, statistics=1,
                       n_tail=3), None),
        (frg.make_desc(frg.FRG_FAMILY_TWO_POINT_T, 8, 10.0, n_x=4, T=0.1, freq_max=3.0,
                       statistics=1, precision=1, near_pole_tau=0.1), np.concatenate([p, p0])),
        (frg.make_desc(frg.FRG_FAMILY_THREE_POINT, 6, 10.0, n_x=4, n_phi=3),
         np.concatenate([p, rng.uniform(0, math.pi, n)])),
    ]
    alone = [_run(env, d, n, ext=e, m2=m2, Z=Z, err=True) for d, e in cases]
    outs = [torch.full((n,), float("nan"), dtype=torch.float64, device="cuda") for _ in cases]
    errs = [torch.full((n,), float("nan"), dtype=torch.float64, device="cuda") for _ in cases]
    keep = [(_d(torch, e) if e is not None else None) for _, e in cases]
    tm, tz = _d(torch, m2), _d(torch, Z)
    batches = [frg.make_batch(n, o, ext=k, m2=tm, Z=tz, x_min=wl.Z_XMIN, x_max=wl.Z_XMAX,
                              err_out=eo) for o, eo, k in zip(outs, errs, keep)]
    for rep in range(2):
        ctx.integrate_multi([d for d, _ in cases], batches)
        torch.cuda.synchronize()
        for i, (o, eo) in enumerate(zip(outs, errs)):
            assert np.array_equal(o.cpu().numpy(), alone[i][0]), (rep, i)
            assert np.array_equal(eo.cpu().numpy(), alone[i][1]), (rep, i)
    ref = oracle.integrate_ft(oracle.TWO_POINT_T, 16, 10.0, n_x=8, T=0.2, freq_max=6.0, n_tail=4,
                              ext=(p, p0 + 0.4), m2=m2, Z=Z)
    assert _rel(alone[0][0], ref) <= TOL


def test_two_point_ft_benchmark_batch_sampled(env):
    # the benchmark's fused launch (16 right-hand sides x 256 momenta x 47 frequencies x 64 x 32),
    # sampled points against the oracle
    frg, ctx, torch = env
    p, p0, m2, Z = wl.two_point_ft_batch()
    B = Z.shape[0]
    desc = frg.make_desc(frg.FRG_FAMILY_TWO_POINT_T, wl.FT_NQ, wl.FT_QMAX, n_x=wl.FT_NX,
                         T=wl.FT_T, freq_max=wl.FT_FREQ_MAX, n_tail=wl.FT_N_TAIL)
    te = _d(torch, np.concatenate([p, p0]))
    tZ = _d(torch, Z)
    out = torch.full((B, p.size), float("nan"), dtype=torch.float64, device="cuda")
    batches = [frg.make_batch(p.size, out[b], ext=te, m2_scalar=m2, Z=tZ[b], x_min=wl.Z_XMIN,
                              x_max=wl.Z_XMAX) for b in range(B)]
    ctx.integrate_multi([desc] * B, batches)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.all(np.isfinite(got)) and np.all(got > 0)
    rng = np.random.default_rng(0)
    for b in (0, B - 1):
        idx = np.sort(rng.choice(p.size, 6, replace=False))
        idx[0] = 0
        ref = oracle.integrate_ft(oracle.TWO_POINT_T, wl.FT_NQ, wl.FT_QMAX, n_x=wl.FT_NX,
                                  T=wl.FT_T, freq_max=wl.FT_FREQ_MAX, n_tail=wl.FT_N_TAIL,
                                  ext=(p[idx], p0[idx]), m2_scalar=m2, Z=Z[b])
        assert _rel(got[b, idx], ref) <= TOL


@pytest.fixture(params=["direct", "graph"])
def flow_ctx(request, env, monkeypatch):
    frg, ctx, torch = env
    if request.param == "direct":
        yield ctx
        return
    monkeypatch.setenv("FRG_FLOW_GRAPH", "1")
    gctx = frg.Context(0)
    try:
        yield gctx
    finally:
        torch.cuda.synchronize()
        gctx.close()


def test_flow_rhs_lpa_finite_temperature(env, flow_ctx):
    # the finite-temperature O(N) LPA flow: du/dt = 1/2 [I_T(m_s^2)(3u' + 2 rho u'')
    # + (N-1) I_T(m_p^2) u'], composed here from the oracle's integrals and derivatives
    frg, _, torch = env
    ctx = flow_ctx
    rho = wl.lpa_rho_grid()
    trho = _d(torch, rho)
    kw = dict(T=0.15, freq_max=8.0, statistics=0, n_tail=6)
    desc = frg.make_desc(frg.FRG_FAMILY_LPA_T, wl.LPA_NQ, wl.LPA_QMAX, **kw)
    state = _d(torch, -0.3 + rho)
    dudt = torch.empty_like(state)
    for rep, (a, b, c) in enumerate([(0.3, 1.0, 0.0), (0.1, 0.7, 0.4), (0.3, 1.0, 0.0)]):
        u = -a + b * rho + c * rho ** 2
        state.copy_(torch.from_numpy(u))
        ctx.flow_rhs(desc, state, trho, dudt, n_comp=4, m2_floor=-0.9)
        torch.cuda.synchronize()
        d1, d2 = oracle.fd_derivatives(rho, u)
        ms = np.maximum(u + 2 * rho * d1, -0.9)
        mp_ = np.maximum(u, -0.9)
        Is = oracle.integrate_ft(oracle.LPA_T, wl.LPA_NQ, wl.LPA_QMAX, m2=ms, **kw)
        Ip = oracle.integrate_ft(oracle.LPA_T, wl.LPA_NQ, wl.LPA_QMAX, m2=mp_, **kw)
        ref = 0.5 * (Is * (3 * d1 + 2 * rho * d2) + 3 * Ip * d1)
        got = dudt.cpu().numpy()
        assert np.max(np.abs(got - ref) / (np.abs(ref) + 1e-3 * np.max(np.abs(ref)))) <= 1e-11, rep


def test_flow_rhs_two_point_finite_temperature(env, flow_ctx):
    frg, _, torch = env
    ctx = flow_ctx
    rng = np.random.default_rng(8)
    n = 80
    p = 10 ** rng.uniform(-3, 2, n)
    p0 = np.where(np.arange(n) % 2 == 0, 0.0, 2 * math.pi * 0.2)
    grid = np.concatenate([p, p0])
    Z = wl.dressing_table(6)
    kw = dict(T=0.2, freq_max=5.0, statistics=0, n_tail=3)
    desc = frg.make_desc(frg.FRG_FAMILY_TWO_POINT_T, 12, 10.0, n_x=8, **kw)
    tgrid, tZ = _d(torch, grid), _d(torch, Z)
    state = _d(torch, rng.uniform(-1.2, 2.0, n))
    out = torch.empty_like(state)
    for rep in range(2):
        s = state.cpu().numpy()
        ctx.flow_rhs(desc, state, tgrid, out, Z=tZ, m2_floor=-0.5, coef=-0.25)
        torch.cuda.synchronize()
        ref = oracle.integrate_ft(oracle.TWO_POINT_T, 12, 10.0, n_x=8, ext=(p, p0),
                                  m2=np.maximum(s, -0.5), Z=Z, **kw)
        assert _rel(out.cpu().numpy(), -0.25 * ref) <= TOL
        state.mul_(0.9).add_(0.05)


def test_session_serves_finite_temperature_requests(env):
    # finite- and zero-temperature requests through one session: every result bitwise equal to
    # the request evaluated alone and within 1e-12 of the oracle
    frg, ctx, torch = env
    rng = np.random.default_rng(31)
    reqs = []
    for i in range(12):
        n = int(rng.integers(5, 120))
        m2 = rng.uniform(0.05, 2.0, n)
        T = float(rng.uniform(0.05, 0.5))
        stat = int(i % 2)
        if i % 3 == 0:
            desc = frg.make_desc(frg.FRG_FAMILY_LPA_T, int(rng.integers(8, 40)), 6.0, T=T,
                                 freq_max=6.0, statistics=stat, n_tail=int(rng.integers(0, 6)))
            ext, Z = None, None
        elif i % 3 == 1:
            desc = frg.make_desc(frg.FRG_FAMILY_TWO_POINT_T, int(rng.integers(4, 24)), 10.0,
                                 n_x=int(rng.integers(2, 16)), T=T, freq_max=4.0,
                                 statistics=stat, n_tail=int(rng.integers(0, 6)))
            ext = np.concatenate([10 ** rng.uniform(-3, 2, n), rng.uniform(-1, 1, n)])
            Z = wl.dressing_table(60 + i)
        else:
            desc = frg.make_desc(frg.FRG_FAMILY_TWO_POINT, int(rng.integers(8, 40)), 10.0,
                                 n_x=int(rng.integers(4, 24)))
            ext = 10 ** rng.uniform(-3, 2, n)
            Z = wl.dressing_table(60 + i)
        reqs.append(dict(desc=desc, ext=ext, m2=m2, Z=Z, n=n, out=np.full(n, np.nan),
                         err=np.full(n, np.nan)))
    s = frg.frg_session_open(ctx.handle, frg.frg_session_config(3, 256 << 20, 20, 0))
    tickets = []
    for r in reqs:
        zt = frg.frg_log_table(None if r["Z"] is None else r["Z"].ctypes.data,
                               0 if r["Z"] is None else r["Z"].size, wl.Z_XMIN, wl.Z_XMAX)
        b = frg.frg_batch(r["n"], None if r["ext"] is None else r["ext"].ctypes.data,
                          r["m2"].ctypes.data, 0.0, zt, r["out"].ctypes.data, r["err"].ctypes.data)
        tickets.append(frg.frg_session_submit(s, r["desc"], b, -1))
    for t in tickets:
        assert frg.frg_session_wait(s, t, 60000) == frg.FRG_OK
    frg.frg_session_close(s)
    for r in reqs:
        d = r["desc"]
        alone = _run(env, d, r["n"], ext=r["ext"], m2=r["m2"], Z=r["Z"])
        assert np.array_equal(r["out"], alone)
        if d.family == frg.FRG_FAMILY_TWO_POINT:
            ref = oracle.integrate(2, d.n_q, d.q_max, n_x=d.n_x, ext=r["ext"], m2=r["m2"],
                                   Z=r["Z"])
        else:
            fam = oracle.LPA_T if d.family == frg.FRG_FAMILY_LPA_T else oracle.TWO_POINT_T
            ext = None if r["ext"] is None else (r["ext"][:r["n"]], r["ext"][r["n"]:])
            ref = oracle.integrate_ft(fam, d.n_q, d.q_max, n_x=d.n_x, T=d.T, freq_max=d.freq_max,
                                      statistics=d.statistics, n_tail=d.n_tail, ext=ext,
                                      m2=r["m2"], Z=r["Z"])
        assert _rel(r["out"], ref) <= TOL
