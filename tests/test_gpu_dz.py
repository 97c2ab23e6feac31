"""GPU derivatives of the vertex integrals (two-point and three-point, in vacuum and at finite
temperature) in their dressing-table entries (dout_dz, dI_e/dZ_i) against the FP64 oracle,
entry by entry.

Every term of an entry's sum has the same sign (W, the weights and G are positive at these
masses), so each entry is compared at 1e-12 relative, plus 1e-12 of its row's largest entry: the
interpolation weights f and 1 - f carry the absolute rounding of the dressing coordinate s (a
few ulp of s, 1e-14 to 1e-13 for tables of hundreds of entries, computed through different
logarithms on the two sides), which an entry reached only through a small weight feels relative
to itself but not relative to its row.
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


def _run(env, n_q, q_max, n_x, p, Z, *, m2=None, m2_scalar=0.0, k=1.0, reg=0, x_min=wl.Z_XMIN,
         x_max=wl.Z_XMAX):
    frg, ctx, torch = env
    n = len(p)
    out = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    jac = torch.full((n * len(Z),), float("nan"), dtype=torch.float64, device="cuda")
    desc = frg.make_desc(frg.FRG_FAMILY_TWO_POINT, n_q, q_max, n_x=n_x, k=k, regulator=reg)
    ctx.integrate(desc, out, ext=_d(torch, p), m2=None if m2 is None else _d(torch, m2),
                  m2_scalar=m2_scalar, Z=_d(torch, Z), x_min=x_min, x_max=x_max, dz=jac)
    torch.cuda.synchronize()
    return out.cpu().numpy(), jac.cpu().numpy().reshape(n, len(Z))


def _check(got, ref):
    assert got.shape == ref.shape
    assert np.all(np.isfinite(got))
    floor = TOL * np.max(np.abs(ref), axis=1, keepdims=True)
    assert np.all(np.abs(got - ref) <= TOL * np.abs(ref) + floor)


def _okind(reg):
    return {0: oracle.REG_EXP, 1: oracle.reg_polyexp(8), 2: oracle.REG_LITIM}[reg]


@pytest.mark.parametrize("reg", [0, 1, 2])
@pytest.mark.parametrize("n_ext,n_q,n_x,nZ,k", [(37, 13, 6, 9, 1.0), (40, 64, 40, 57, 1.0),
                                                 (9, 20, 7, 300, 1.7)])
def test_dz_matches_oracle(env, reg, n_ext, n_q, n_x, nZ, k):
    # n_x = 40: 25 radial nodes per round, three rounds; momenta below and above the table
    rng = np.random.default_rng(n_ext + 3 * reg)
    p = k * np.concatenate([[0.0, 2e-4, 500.0], 10 ** rng.uniform(-3, 2, n_ext - 3)])
    m2 = k * k * rng.uniform(0.1, 2.0, n_ext)
    Z = wl.dressing_table(5 + nZ, nZ)
    got_v, got = _run(env, n_q, 10.0, n_x, p, Z, m2=m2, k=k, reg=reg)
    ref = oracle.integrate_dz(n_q, 10.0, n_x=n_x, ext=p, m2=m2, Z=Z, k=k,
                              regulator=_okind(reg), x_min=wl.Z_XMIN, x_max=wl.Z_XMAX)
    _check(got, ref)
    ref_v = oracle.integrate(oracle.TWO_POINT, n_q, 10.0, n_x=n_x, k=k, ext=p, m2=m2, Z=Z,
                             regulator=_okind(reg))
    assert np.max(np.abs(got_v - ref_v) / np.abs(ref_v)) <= TOL


@pytest.mark.parametrize("stat,reg,scaled", [(0, 0, False), (1, 1, True), (0, 2, False)])
def test_dz_finite_temperature_matches_oracle(env, stat, reg, scaled):
    # the Matsubara sum folded into the radial index; momenta below and above the table
    frg, ctx, torch = env
    rng = np.random.default_rng(60 + stat + reg)
    n, n_q, n_x, nZ = 21, 20, 9, 33
    p = np.concatenate([[0.0, 3e-4, 400.0], 10 ** rng.uniform(-3, 2, n - 3)])
    p0 = rng.uniform(-1.0, 1.0, n)
    m2 = rng.uniform(0.1, 1.5, n)
    Z = wl.dressing_table(70 + nZ, nZ)
    ft = dict(T=0.2, freq_max=4.0, statistics=stat, n_tail=3, freq_scaled=scaled)
    out = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    jac = torch.full((n * nZ,), float("nan"), dtype=torch.float64, device="cuda")
    desc = frg.make_desc(frg.FRG_FAMILY_TWO_POINT_T, n_q, 10.0, n_x=n_x, regulator=reg, **ft)
    ctx.integrate(desc, out, ext=_d(torch, np.concatenate([p, p0])), m2=_d(torch, m2),
                  Z=_d(torch, Z), x_min=wl.Z_XMIN, x_max=wl.Z_XMAX, dz=jac)
    torch.cuda.synchronize()
    ref = oracle.integrate_ft_dz(n_q, 10.0, n_x=n_x, ext=(p, p0), m2=m2, Z=Z,
                                 regulator=_okind(reg), x_min=wl.Z_XMIN, x_max=wl.Z_XMAX, **ft)
    _check(jac.cpu().numpy().reshape(n, nZ), ref)
    ref_v = oracle.integrate_ft(oracle.TWO_POINT_T, n_q, 10.0, n_x=n_x, ext=(p, p0), m2=m2,
                                Z=Z, regulator=_okind(reg), **ft)
    assert np.max(np.abs(out.cpu().numpy() - ref_v) / np.abs(ref_v)) <= TOL


@pytest.mark.parametrize("reg", [0, 1, 2])
@pytest.mark.parametrize("n,n_q,n_x,n_phi,nZ", [(13, 9, 5, 7, 11), (6, 12, 40, 600, 48)])
def test_dz_three_point_matches_oracle(env, reg, n, n_q, n_x, n_phi, nZ):
    # rows of (radial, cos1) pairs over phi; n_phi = 600: one row per round; angles over
    # [0, pi] and beyond it (sin(alpha) < 0 reads |sin(alpha)|)
    frg, ctx, torch = env
    rng = np.random.default_rng(80 + n + reg)
    p = np.concatenate([[0.0, 400.0], 10 ** rng.uniform(-3, 2, n - 2)])
    alpha = np.concatenate([[0.0, math.pi], rng.uniform(0.0, math.pi, n - 3), [4.0]])
    m2 = rng.uniform(0.1, 1.5, n)
    Z = wl.dressing_table(90 + nZ, nZ)
    out = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    jac = torch.full((n * nZ,), float("nan"), dtype=torch.float64, device="cuda")
    desc = frg.make_desc(frg.FRG_FAMILY_THREE_POINT, n_q, 10.0, n_x=n_x, n_phi=n_phi,
                         regulator=reg)
    ctx.integrate(desc, out, ext=_d(torch, np.concatenate([p, alpha])), m2=_d(torch, m2),
                  Z=_d(torch, Z), x_min=wl.Z_XMIN, x_max=wl.Z_XMAX, dz=jac)
    torch.cuda.synchronize()
    ref = oracle.integrate_dz_three(n_q, 10.0, n_x=n_x, n_phi=n_phi, ext=(p, alpha), m2=m2, Z=Z,
                                    regulator=_okind(reg), x_min=wl.Z_XMIN, x_max=wl.Z_XMAX)
    _check(jac.cpu().numpy().reshape(n, nZ), ref)
    ref_v = oracle.integrate(oracle.THREE_POINT, n_q, 10.0, n_x=n_x, n_phi=n_phi,
                             ext=(p, alpha), m2=m2, Z=Z, regulator=_okind(reg))
    assert np.max(np.abs(out.cpu().numpy() - ref_v) / np.abs(ref_v)) <= TOL


@pytest.mark.parametrize("stat,reg", [(0, 0), (1, 1), (0, 2)])
def test_dz_three_point_finite_temperature_matches_oracle(env, stat, reg):
    # family 6: the radial index folds the frequencies in; each inner leg with its own shift
    frg, ctx, torch = env
    rng = np.random.default_rng(120 + stat + reg)
    n, n_q, n_x, n_phi, nZ = 11, 8, 6, 5, 23
    p = np.concatenate([[0.0, 400.0], 10 ** rng.uniform(-3, 2, n - 2)])
    alpha = np.concatenate([[0.0, math.pi], rng.uniform(0.0, math.pi, n - 2)])
    p01, p02 = rng.uniform(-1.0, 1.0, n), rng.uniform(-1.0, 1.0, n)
    m2 = rng.uniform(0.1, 1.5, n)
    Z = wl.dressing_table(130 + nZ, nZ)
    ft = dict(T=0.25, freq_max=3.0, statistics=stat, n_tail=2)
    out = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    jac = torch.full((n * nZ,), float("nan"), dtype=torch.float64, device="cuda")
    desc = frg.make_desc(frg.FRG_FAMILY_THREE_POINT_T, n_q, 10.0, n_x=n_x, n_phi=n_phi,
                         regulator=reg, **ft)
    ext = np.concatenate([p, alpha, p01, p02])
    ctx.integrate(desc, out, ext=_d(torch, ext), m2=_d(torch, m2), Z=_d(torch, Z),
                  x_min=wl.Z_XMIN, x_max=wl.Z_XMAX, dz=jac)
    torch.cuda.synchronize()
    ref = oracle.integrate_ft_three_dz(n_q, 10.0, n_x=n_x, n_phi=n_phi, ext=(p, alpha, p01, p02),
                                       m2=m2, Z=Z, regulator=_okind(reg), x_min=wl.Z_XMIN,
                                       x_max=wl.Z_XMAX, **ft)
    _check(jac.cpu().numpy().reshape(n, nZ), ref)
    ref_v = oracle.integrate_ft(oracle.THREE_POINT_T, n_q, 10.0, n_x=n_x, n_phi=n_phi,
                                ext=(p, alpha, p01, p02), m2=m2, Z=Z, regulator=_okind(reg),
                                **ft)
    assert np.max(np.abs(out.cpu().numpy() - ref_v) / np.abs(ref_v)) <= TOL
    # the same block from a fused launch beside a vacuum three-point request
    out2 = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    jac2 = torch.full((n * nZ,), float("nan"), dtype=torch.float64, device="cuda")
    o3 = torch.empty(n, dtype=torch.float64, device="cuda")
    te, tm, tZ = _d(torch, ext), _d(torch, m2), _d(torch, Z)
    t3 = _d(torch, np.concatenate([p, alpha]))
    ctx.integrate_multi(
        [desc, frg.make_desc(frg.FRG_FAMILY_THREE_POINT, 8, 10.0, n_x=6, n_phi=5)],
        [frg.make_batch(n, out2, ext=te, m2=tm, Z=tZ, x_min=wl.Z_XMIN, x_max=wl.Z_XMAX,
                        dz=jac2),
         frg.make_batch(n, o3, ext=t3, m2=tm, Z=tZ, x_min=wl.Z_XMIN, x_max=wl.Z_XMAX)])
    torch.cuda.synchronize()
    assert torch.equal(out2, out) and torch.equal(jac2, jac)


def test_dz_two_point_workload_full_size(env):
    # one right-hand side of the two-point workload: 256 momenta x 64 x 32, 256-entry table
    p, m2, Z = wl.two_point()
    got_v, got = _run(env, wl.TWO_NQ, wl.TWO_QMAX, wl.TWO_NX, p, Z, m2_scalar=m2)
    ref = oracle.integrate_dz(wl.TWO_NQ, wl.TWO_QMAX, n_x=wl.TWO_NX, ext=p, m2_scalar=m2, Z=Z,
                              x_min=wl.Z_XMIN, x_max=wl.Z_XMAX)
    _check(got, ref)


def test_dz_full_size_three_point_and_finite_temperature_sampled(env):
    # one right-hand side of the three-point workload (1024 points x 64 x 32 x 16) and of the
    # finite-temperature workload (256 momenta x 47 frequencies x 64 x 32), every point on the
    # GPU, a sample of points through the oracle
    frg, ctx, torch = env
    rng = np.random.default_rng(17)
    P, A, m3, Z3 = wl.three_point()
    n = P.size
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    jac = torch.full((n * Z3.size,), float("nan"), dtype=torch.float64, device="cuda")
    d3 = frg.make_desc(frg.FRG_FAMILY_THREE_POINT, wl.THREE_NQ, wl.THREE_QMAX, n_x=wl.THREE_NX,
                       n_phi=wl.THREE_NPHI)
    ctx.integrate(d3, out, ext=_d(torch, np.concatenate([P, A])), m2=_d(torch, m3),
                  Z=_d(torch, Z3), x_min=wl.Z_XMIN, x_max=wl.Z_XMAX, dz=jac)
    torch.cuda.synchronize()
    J = jac.cpu().numpy().reshape(n, Z3.size)
    idx = np.sort(rng.choice(n, 24, replace=False))
    ref = oracle.integrate_dz_three(wl.THREE_NQ, wl.THREE_QMAX, n_x=wl.THREE_NX,
                                    n_phi=wl.THREE_NPHI, ext=(P[idx], A[idx]), m2=m3[idx], Z=Z3,
                                    x_min=wl.Z_XMIN, x_max=wl.Z_XMAX)
    _check(J[idx], ref)
    p = wl.momenta_log()
    p0 = np.where(np.arange(p.size) % 2 == 0, 0.0, 2 * math.pi * wl.FT_T)
    Z = wl.dressing_table(1000)
    ft = dict(T=wl.FT_T, freq_max=wl.FT_FREQ_MAX, statistics=0, n_tail=wl.FT_N_TAIL)
    dft = frg.make_desc(frg.FRG_FAMILY_TWO_POINT_T, wl.FT_NQ, wl.FT_QMAX, n_x=wl.FT_NX, **ft)
    out = torch.empty(p.size, dtype=torch.float64, device="cuda")
    jac = torch.full((p.size * Z.size,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.integrate(dft, out, ext=_d(torch, np.concatenate([p, p0])), m2_scalar=0.5,
                  Z=_d(torch, Z), x_min=wl.Z_XMIN, x_max=wl.Z_XMAX, dz=jac)
    torch.cuda.synchronize()
    J = jac.cpu().numpy().reshape(p.size, Z.size)
    idx = np.sort(rng.choice(p.size, 16, replace=False))
    ref = oracle.integrate_ft_dz(wl.FT_NQ, wl.FT_QMAX, n_x=wl.FT_NX, ext=(p[idx], p0[idx]),
                                 m2_scalar=0.5, Z=Z, x_min=wl.Z_XMIN, x_max=wl.Z_XMAX, **ft)
    _check(J[idx], ref)


def test_dz_largest_table_and_rule(env):
    # the largest dressing table (4096 entries, 135 KB of LDS) and the largest cos1 rule (1024
    # nodes: one radial node per round)
    Z = 0.8 + 0.7 * (0.5 + 0.5 * np.sin(np.linspace(0, 40, 4096)))
    p = np.array([0.01, 0.7, 3.0])
    for n_q, n_x, nz in ((16, 64, 4096), (4, 1024, 64)):
        got_v, got = _run(env, n_q, 10.0, n_x, p, Z[:nz], m2_scalar=0.3)
        ref = oracle.integrate_dz(n_q, 10.0, n_x=n_x, ext=p, m2_scalar=0.3, Z=Z[:nz],
                                  x_min=wl.Z_XMIN, x_max=wl.Z_XMAX)
        _check(got, ref)


def test_dz_reproducible_and_value_unchanged(env):
    frg, ctx, torch = env
    p, m2, Z = wl.two_point()
    v1, j1 = _run(env, 24, 10.0, 12, p, Z, m2_scalar=m2)
    v2, j2 = _run(env, 24, 10.0, 12, p, Z, m2_scalar=m2)
    assert np.array_equal(j1, j2)
    out = torch.empty(p.size, dtype=torch.float64, device="cuda")
    desc = frg.make_desc(frg.FRG_FAMILY_TWO_POINT, 24, 10.0, n_x=12)
    ctx.integrate(desc, out, ext=_d(torch, p), m2_scalar=m2, Z=_d(torch, Z), x_min=wl.Z_XMIN,
                  x_max=wl.Z_XMAX)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), v1)


def test_dz_same_bits_alone_and_in_a_batch(env):
    """The block is summed exactly across lanes (integer accumulation), so a point's entries
    are the same bits whether it is launched alone (a workgroup of 16 wavefronts) or among
    1024 points (4 wavefronts per workgroup)."""
    frg, ctx, torch = env
    P, A, m3, Z3 = wl.three_point()
    d3 = frg.make_desc(frg.FRG_FAMILY_THREE_POINT, 24, wl.THREE_QMAX, n_x=12, n_phi=8)

    def block(idx):
        n = idx.size
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        jac = torch.full((n * Z3.size,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.integrate(d3, out, ext=_d(torch, np.concatenate([P[idx], A[idx]])),
                      m2=_d(torch, m3[idx]), Z=_d(torch, Z3), x_min=wl.Z_XMIN, x_max=wl.Z_XMAX,
                      dz=jac)
        torch.cuda.synchronize()
        return jac.cpu().numpy().reshape(n, Z3.size)

    every = block(np.arange(P.size))
    for i in (0, 517, P.size - 1):
        assert np.array_equal(block(np.array([i])), every[i:i + 1]), i


def test_dz_through_fused_launches(env):
    """frg_integrate_multi computes each request's block after the fused launch: the same bits
    as frg_integrate_batch per request, requests without it untouched, and again when the same
    call is repeated (the plan cache relaunches the blocks too)."""
    frg, ctx, torch = env
    P, A, m3, Z3 = wl.three_point()
    p, m2, Z2 = wl.two_point()
    sel = np.arange(0, P.size, 7)
    reqs = [
        (frg.make_desc(frg.FRG_FAMILY_THREE_POINT, 24, wl.THREE_QMAX, n_x=12, n_phi=8),
         np.concatenate([P[sel], A[sel]]), m3[sel], Z3, True),
        (frg.make_desc(frg.FRG_FAMILY_TWO_POINT, 32, wl.TWO_QMAX, n_x=16), p,
         np.full(p.size, m2), Z2, True),
        (frg.make_desc(frg.FRG_FAMILY_TWO_POINT, 16, wl.TWO_QMAX, n_x=8), p,
         np.full(p.size, m2), Z2, False),
    ]
    descs, batches, outs, jacs, keep, alone = [], [], [], [], [], []
    for desc, ext, mm, Z, want in reqs:
        n = mm.size
        te, tm, tZ = _d(torch, ext), _d(torch, mm), _d(torch, Z)
        out = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        jac = torch.full((n * Z.size,), float("nan"), dtype=torch.float64, device="cuda") \
            if want else None
        descs.append(desc)
        batches.append(frg.make_batch(n, out, ext=te, m2=tm, Z=tZ, x_min=wl.Z_XMIN,
                                      x_max=wl.Z_XMAX, dz=jac))
        outs.append(out)
        jacs.append(jac)
        keep += [te, tm, tZ]
        o1 = torch.empty(n, dtype=torch.float64, device="cuda")
        j1 = torch.empty(n * Z.size, dtype=torch.float64, device="cuda") if want else None
        ctx.integrate(desc, o1, ext=te, m2=tm, Z=tZ, x_min=wl.Z_XMIN, x_max=wl.Z_XMAX, dz=j1)
        alone.append((o1, j1))
    for rep in range(2):
        for j in jacs:
            if j is not None:
                j.fill_(float("nan"))
        ctx.integrate_multi(descs, batches)
        torch.cuda.synchronize()
        for i in range(len(reqs)):
            assert torch.equal(outs[i], alone[i][0]), (rep, i)
            if jacs[i] is not None:
                assert torch.equal(jacs[i], alone[i][1]), (rep, i)


def test_dz_unsupported_and_invalid(env):
    frg, ctx, torch = env
    n = 4
    out = torch.zeros(n, dtype=torch.float64, device="cuda")
    ext = torch.ones(2 * n, dtype=torch.float64, device="cuda")
    Z = _d(torch, wl.dressing_table(1, 16))
    jac = torch.zeros(n * 16, dtype=torch.float64, device="cuda")
    cases = [(frg.make_desc(frg.FRG_FAMILY_LPA_T, 8, 6.0, T=0.2, freq_max=3.0),
              frg.FRG_E_UNSUPPORTED),
             (frg.make_desc(frg.FRG_FAMILY_TWO_POINT, 8, 6.0, n_x=4, precision=1),
              frg.FRG_E_UNSUPPORTED),
             (frg.make_desc(frg.FRG_FAMILY_LPA, 8, 6.0), frg.FRG_E_UNSUPPORTED),
             (frg.make_desc(frg.FRG_FAMILY_TWO_POINT_T, 8, 6.0, n_x=4, T=0.2, freq_max=3.0,
                            complex_freq=True), frg.FRG_E_UNSUPPORTED)]
    for desc, status in cases:
        # complex frequencies: out holds Re and Im of the n points
        o = torch.zeros(2 * n, dtype=torch.float64, device="cuda") if desc.complex_freq else out
        e = torch.ones(3 * n, dtype=torch.float64, device="cuda") if desc.complex_freq else ext
        with pytest.raises(frg.FrgError) as ei:
            ctx.integrate(desc, o, ext=e, m2_scalar=0.5, Z=Z, dz=jac)
        assert ei.value.status == status
    d2 = frg.make_desc(frg.FRG_FAMILY_TWO_POINT, 8, 6.0, n_x=4)
    # no table: a batch built by hand (the binding checks the size against the table)
    b = frg.make_batch(n, out, ext=ext, m2_scalar=0.5)
    b.dout_dz = jac.data_ptr()
    with pytest.raises(frg.FrgError) as ei:
        frg.frg_integrate_batch(ctx.handle, d2, b, 0)
    assert ei.value.status == frg.FRG_E_INVAL
    with pytest.raises(ValueError):
        frg.make_batch(n, out, ext=ext, m2_scalar=0.5, Z=Z, dz=jac[:-1])
    torch.cuda.synchronize()


def test_dz_through_sessions(env):
    """Sessions return dI_e/dZ_i in host buffers: a two-point request with its own table, a
    three-point one on a resident table, a finite-temperature three-point request above one
    launch's node budget (split into parts, each part's rows after its outputs) and requests
    without it beside them; values and blocks the bits frg_integrate_batch gives alone."""
    frg, ctx, torch = env
    rng = np.random.default_rng(321)
    p = wl.momenta_log(200)
    Z2, Z3 = wl.dressing_table(40, 64), wl.dressing_table(41, 48)
    P, A, p01, p02, m2b, Zb = wl.three_point_ft_batch(1)
    reqs = [
        dict(desc=frg.make_desc(2, 24, 10.0, n_x=12), ext=p, m2=rng.uniform(0.1, 2.0, p.size),
             Z=Z2, resident=False, dz=True),
        dict(desc=frg.make_desc(3, 10, 10.0, n_x=6, n_phi=5),
             ext=np.concatenate([p[:90], rng.uniform(0, math.pi, 90)]),
             m2=rng.uniform(0.1, 2.0, 90), Z=Z3, resident=True, dz=True),
        dict(desc=frg.make_desc(2, 16, 10.0, n_x=8), ext=p, m2=rng.uniform(0.1, 2.0, p.size),
             Z=Z2, resident=False, dz=False),
        # 1024 pairs x 32 radial x 47 frequencies x 16 x 16 = 3.9e8 nodes: in parts
        dict(desc=frg.make_desc(6, 32, wl.THREE_QMAX, n_x=16, n_phi=16, T=wl.FT_T,
                                freq_max=wl.FT_FREQ_MAX, n_tail=wl.FT_N_TAIL),
             ext=np.concatenate([P, A, p01, p02]), m2=m2b[0], Z=Zb[0], resident=False, dz=True),
    ]
    s = frg.frg_session_open(ctx.handle, frg.frg_session_config(3, 1 << 30, 20, 0))
    tickets = []
    for r in reqs:
        n = r["m2"].size
        r["n"] = n
        r["out"] = np.full(n, np.nan)
        r["jac"] = np.full(n * r["Z"].size, np.nan) if r["dz"] else None
        if r["resident"]:
            tid = frg.frg_session_register_table(s, r["Z"].ctypes.data, r["Z"].size, wl.Z_XMIN,
                                                 wl.Z_XMAX)
            zt = frg.frg_log_table(None, 0, wl.Z_XMIN, wl.Z_XMAX)
        else:
            tid = -1
            zt = frg.frg_log_table(r["Z"].ctypes.data, r["Z"].size, wl.Z_XMIN, wl.Z_XMAX)
        b = frg.frg_batch(n, r["ext"].ctypes.data, r["m2"].ctypes.data, 0.0, zt,
                          r["out"].ctypes.data, None, None,
                          None if r["jac"] is None else r["jac"].ctypes.data)
        tickets.append(frg.frg_session_submit(s, r["desc"], b, tid))
    for t in tickets:
        assert frg.frg_session_wait(s, t, 120000) == frg.FRG_OK
    frg.frg_session_close(s)
    for i, r in enumerate(reqs):
        n, nz = r["n"], r["Z"].size
        out = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        jac = torch.full((n * nz,), float("nan"), dtype=torch.float64, device="cuda") \
            if r["dz"] else None
        ctx.integrate(r["desc"], out, ext=_d(torch, r["ext"]), m2=_d(torch, r["m2"]),
                      Z=_d(torch, r["Z"]), x_min=wl.Z_XMIN, x_max=wl.Z_XMAX, dz=jac)
        torch.cuda.synchronize()
        assert np.array_equal(r["out"], out.cpu().numpy()), i
        if r["dz"]:
            assert np.array_equal(r["jac"], jac.cpu().numpy()), i
