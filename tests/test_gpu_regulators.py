"""GPU parity for the regulator variants -- polynomial-exponential s_N (the paper's default, N = 8,
and other orders) and flat (Litim) -- in every family, against the FP64 oracle: 1e-12 relative
per point, bitwise equality across tile shapes and in fused launches mixed with the exponential
regulator, the float32 form of both in fused launches.
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


def _run(env, desc, n, *, ext=None, m2=None, Z=None, ctx=None):
    frg, ctx0, torch = env
    out = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    (ctx or ctx0).integrate(desc, out, ext=None if ext is None else _d(torch, ext),
                            m2=None if m2 is None else _d(torch, m2),
                            Z=None if Z is None else _d(torch, Z), x_min=wl.Z_XMIN,
                            x_max=wl.Z_XMAX)
    torch.cuda.synchronize()
    return out.cpu().numpy()


# GPU regulator code -> (oracle kind, order)
def _okind(reg, n):
    return {0: oracle.REG_EXP, 1: oracle.reg_polyexp(n or 8), 2: oracle.REG_LITIM}[reg]


def _nodes_clear_of_kink(n_q, q_max):
    # the flat regulator's k dR/dk jumps at |q| = k: keep every radial node off it
    x, _ = np.polynomial.legendre.leggauss(n_q)
    q = 0.5 * q_max * (x + 1.0)
    return np.min(np.abs(q - 1.0)) > 1e-6


REGS = [(1, 0), (1, 3), (1, 16), (2, 0)]


@pytest.mark.parametrize("reg,order", REGS)
def test_lpa_regulators(env, reg, order):
    frg = env[0]
    assert _nodes_clear_of_kink(wl.LPA_NQ, wl.LPA_QMAX)
    rho, u, m2 = wl.lpa_potential()
    for d in (3, 4):
        desc = frg.make_desc(frg.FRG_FAMILY_LPA, wl.LPA_NQ, wl.LPA_QMAX, d=d, regulator=reg,
                             reg_order=order)
        got = _run(env, desc, m2.size, m2=m2)
        ref = oracle.integrate(oracle.LPA, wl.LPA_NQ, wl.LPA_QMAX, d=d, m2=m2,
                               regulator=_okind(reg, order))
        assert _rel(got, ref) <= TOL, d


@pytest.mark.parametrize("reg,order", REGS)
@pytest.mark.parametrize("n_ext,n_q,n_x,k", [(37, 13, 6, 1.0), (256, 64, 32, 1.0), (9, 20, 7, 1.9)])
def test_two_point_regulators(env, reg, order, n_ext, n_q, n_x, k):
    frg = env[0]
    q_max = 10.0
    assert _nodes_clear_of_kink(n_q, q_max)
    rng = np.random.default_rng(n_ext + 7 * reg)
    p = k * 10 ** rng.uniform(-3, 2, n_ext)
    m2 = k * k * rng.uniform(-0.5, 2.0, n_ext)
    Z = wl.dressing_table(13)
    desc = frg.make_desc(frg.FRG_FAMILY_TWO_POINT, n_q, q_max, n_x=n_x, k=k, regulator=reg,
                         reg_order=order)
    got = _run(env, desc, n_ext, ext=p, m2=m2, Z=Z)
    ref = oracle.integrate(oracle.TWO_POINT, n_q, q_max, n_x=n_x, k=k, ext=p, m2=m2, Z=Z,
                           regulator=_okind(reg, order))
    assert _rel(got, ref) <= TOL


@pytest.mark.parametrize("reg,order", REGS)
def test_three_point_regulators(env, reg, order):
    frg = env[0]
    rng = np.random.default_rng(50 + reg)
    n = 40
    P = 10 ** rng.uniform(-3, 2, n)
    A = rng.uniform(0, math.pi, n)
    m2 = rng.uniform(0.1, 2.0, n)
    Z = wl.dressing_table(2)
    desc = frg.make_desc(frg.FRG_FAMILY_THREE_POINT, 12, 10.0, n_x=8, n_phi=6, regulator=reg,
                         reg_order=order)
    got = _run(env, desc, n, ext=np.concatenate([P, A]), m2=m2, Z=Z)
    ref = oracle.integrate(oracle.THREE_POINT, 12, 10.0, n_x=8, n_phi=6, ext=(P, A), m2=m2, Z=Z,
                           regulator=_okind(reg, order))
    assert _rel(got, ref) <= TOL


@pytest.mark.parametrize("reg,order", REGS)
def test_finite_temperature_regulators(env, reg, order):
    # the paper's finite-temperature O(N) example uses s_8 on the spatial momentum
    frg = env[0]
    rho, u, m2 = wl.lpa_potential()
    ft = dict(T=0.2, freq_max=6.0, statistics=0, n_tail=4)
    desc = frg.make_desc(frg.FRG_FAMILY_LPA_T, wl.LPA_NQ, wl.LPA_QMAX, regulator=reg,
                         reg_order=order, **ft)
    got = _run(env, desc, m2.size, m2=m2)
    ref = oracle.integrate_ft(oracle.LPA_T, wl.LPA_NQ, wl.LPA_QMAX, m2=m2,
                              regulator=_okind(reg, order), **ft)
    assert _rel(got, ref) <= TOL
    rng = np.random.default_rng(3)
    n = 30
    p, p0 = 10 ** rng.uniform(-3, 2, n), 2 * math.pi * 0.2 * rng.integers(-1, 2, n)
    Z = wl.dressing_table(4)
    desc = frg.make_desc(frg.FRG_FAMILY_TWO_POINT_T, 16, 10.0, n_x=8, regulator=reg,
                         reg_order=order, **ft)
    got = _run(env, desc, n, ext=np.concatenate([p, p0]), m2=m2[:n], Z=Z)
    ref = oracle.integrate_ft(oracle.TWO_POINT_T, 16, 10.0, n_x=8, ext=(p, p0), m2=m2[:n], Z=Z,
                              regulator=_okind(reg, order), **ft)
    assert _rel(got, ref) <= TOL


def test_regulator_tile_shapes_and_fused_mix_bitwise(env, tmp_path, monkeypatch):
    frg, ctx, torch = env
    n_q, n_x, n = 13, 6, 37
    rng = np.random.default_rng(91)
    p = 10 ** rng.uniform(-3, 2, n)
    m2 = rng.uniform(-0.3, 2.0, n)
    Z = wl.dressing_table(7)
    desc = frg.make_desc(frg.FRG_FAMILY_TWO_POINT, n_q, 10.0, n_x=n_x, regulator=1)
    target = 16 * torch.cuda.get_device_properties(0).multi_processor_count
    res = []
    for lq, ch, lx in [(0, 1, 0), (0, 13, 0), (3, 2, 0), (6, 1, 0), (2, 1, 2)]:
        cache = tmp_path / f"reg_{lq}_{ch}_{lx}.txt"
        cache.write_text(f"2 0 {n_q} {n_x} 0 {n} {target} {lq} {ch} {lx}\n")
        monkeypatch.setenv("FRG_AUTOTUNE_CACHE", str(cache))
        c = frg.Context(0)
        try:
            res.append(_run(env, desc, n, ext=p, m2=m2, Z=Z, ctx=c))
        finally:
            torch.cuda.synchronize()
            c.close()
    for r in res[1:]:
        assert np.array_equal(r, res[0])
    # one fused launch mixing regulators and families equals each request alone
    descs = [desc,
             frg.make_desc(frg.FRG_FAMILY_TWO_POINT, n_q, 10.0, n_x=n_x),
             frg.make_desc(frg.FRG_FAMILY_TWO_POINT, n_q, 10.0, n_x=n_x, regulator=2),
             frg.make_desc(frg.FRG_FAMILY_LPA, 32, 6.0, regulator=1, reg_order=4),
             frg.make_desc(frg.FRG_FAMILY_THREE_POINT, 6, 10.0, n_x=4, n_phi=3, regulator=2)]
    exts = [p, p, p, None, np.concatenate([p, rng.uniform(0, math.pi, n)])]
    alone = [_run(env, d, n, ext=e, m2=m2, Z=Z) for d, e in zip(descs, exts)]
    outs = [torch.full((n,), float("nan"), dtype=torch.float64, device="cuda") for _ in descs]
    keep = [None if e is None else _d(torch, e) for e in exts]
    tm, tz = _d(torch, m2), _d(torch, Z)
    bs = [frg.make_batch(n, o, ext=k, m2=tm, Z=tz, x_min=wl.Z_XMIN, x_max=wl.Z_XMAX)
          for o, k in zip(outs, keep)]
    ctx.integrate_multi(descs, bs)
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        assert np.array_equal(o.cpu().numpy(), alone[i]), i


def test_regulator_arguments_checked(env):
    frg, ctx, torch = env
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    ext = torch.ones(4, dtype=torch.float64, device="cuda")
    for kw, status in [(dict(regulator=3), frg.FRG_E_INVAL), (dict(regulator=-1), frg.FRG_E_INVAL),
                       (dict(regulator=1, reg_order=17), frg.FRG_E_INVAL)]:
        desc = frg.make_desc(frg.FRG_FAMILY_TWO_POINT, 8, 6.0, n_x=4, **kw)
        with pytest.raises(frg.FrgError) as ei:
            ctx.integrate(desc, out, ext=ext, m2_scalar=0.5)
        assert ei.value.status == status, kw


def test_fp32_regulators_fused_equal_alone(env):
    # float32 requests with the s_8 and the flat regulator (and one float64 request) in one
    # fused launch (the general kernel): values and stated bounds bitwise those of the requests
    # evaluated alone
    frg, ctx, torch = env
    p, m2, Z = wl.near_pole()
    P, A, m3, Z3 = wl.three_point()
    sel = np.arange(0, 1024, 29)
    reqs = [(frg.make_desc(2, 24, 10.0, n_x=12, precision=1, near_pole_tau=0.1, regulator=1),
             p, m2, Z, True),
            (frg.make_desc(3, 12, 10.0, n_x=6, n_phi=6, precision=1, near_pole_tau=0.1,
                           regulator=2), np.concatenate([P[sel], A[sel]]), m3[sel], Z3, True),
            (frg.make_desc(2, 16, 10.0, n_x=8, regulator=1), p, m2 + 1.5, Z, False)]
    descs, batches, outs, errs, keep, alone = [], [], [], [], [], []
    for d, ext, mm, Zt, f32 in reqs:
        n = mm.size
        te, tm, tZ = _d(torch, ext), _d(torch, mm), _d(torch, Zt)
        o = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        e = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda") if f32 else None
        descs.append(d)
        batches.append(frg.make_batch(n, o, ext=te, m2=tm, Z=tZ, x_min=wl.Z_XMIN,
                                      x_max=wl.Z_XMAX, err_out=e))
        outs.append(o)
        errs.append(e)
        keep += [te, tm, tZ]
        o1 = torch.empty(n, dtype=torch.float64, device="cuda")
        e1 = torch.empty(n, dtype=torch.float64, device="cuda") if f32 else None
        ctx.integrate(d, o1, ext=te, m2=tm, Z=tZ, x_min=wl.Z_XMIN, x_max=wl.Z_XMAX, err_out=e1)
        alone.append((o1, e1))
    ctx.integrate_multi(descs, batches)
    torch.cuda.synchronize()
    for i in range(len(reqs)):
        assert torch.equal(outs[i], alone[i][0]), i
        if errs[i] is not None:
            assert torch.equal(errs[i], alone[i][1]), i
