"""frg_integrate_batch_noalloc against frg_integrate_batch, through the C ABI.

The no-allocation entry point keeps its scratch (quadrature rules not yet cached, radial
contributions of chunked requests, float32 amplification slots) in one static device array; its
results must be bitwise those of frg_integrate_batch on the same inputs.  Every case makes two
calls in a row, the second with a smaller input, so the second runs on whatever the first left
in the shared array.
"""
import numpy as np
import pytest

from paper_2412_13043_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2412_13043_amd import frg

    yield frg, torch
    torch.cuda.synchronize()


def _d(torch, a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), dtype=torch.float64,
                        device="cuda")


def _both(env, ctx, desc, n_ext, *, ext=None, m2=None, m2_scalar=0.0, Z=None, err=False,
          dm2=False, dz=False, order=("noalloc", "batch")):
    """Run the request through both entry points (in `order`); returns {entry: [arrays]}."""
    frg, torch = env
    te = None if ext is None else _d(torch, ext)
    tm = None if m2 is None else _d(torch, m2)
    tz = None if Z is None else _d(torch, Z)
    res = {}
    for entry in order:
        out = torch.full((n_ext,), float("nan"), dtype=torch.float64, device="cuda")
        eo = torch.full((n_ext,), float("nan"), dtype=torch.float64, device="cuda") \
            if err else None
        do = torch.full((n_ext,), float("nan"), dtype=torch.float64, device="cuda") \
            if dm2 else None
        jz = torch.full((n_ext * len(Z),), float("nan"), dtype=torch.float64, device="cuda") \
            if dz else None
        fn = ctx.integrate_noalloc if entry == "noalloc" else ctx.integrate
        fn(desc, out, ext=te, m2=tm, m2_scalar=m2_scalar, Z=tz, x_min=wl.Z_XMIN,
           x_max=wl.Z_XMAX, err_out=eo, dout=do, dz=jz)
        torch.cuda.synchronize()
        res[entry] = [t.cpu().numpy() for t in (out, eo, do, jz) if t is not None]
    return res


def _same_bits(res):
    a, b = res["noalloc"], res["batch"]
    assert len(a) == len(b)
    for x, y in zip(a, b):
        assert np.all(np.isfinite(x)), "unwritten or non-finite output"
        assert np.array_equal(x.view(np.uint64), y.view(np.uint64))


def test_three_point_chunked_then_smaller(env):
    frg, torch = env
    # a fresh context: the first call finds no cached rules and builds them in the scratch
    with frg.Context(0) as ctx:
        P, A, m3, Z = wl.three_point()
        desc = frg.make_desc(3, wl.THREE_NQ, wl.THREE_QMAX, n_x=wl.THREE_NX,
                             n_phi=wl.THREE_NPHI)
        # 1024 pairs x 32768 nodes: radially chunked, contributions in the scratch
        _same_bits(_both(env, ctx, desc, P.size, ext=np.concatenate([P, A]), m2=m3, Z=Z))
        # second call, smaller, new rule sizes (not cached before this call)
        rng = np.random.default_rng(7)
        n = 200
        p = 10.0 ** rng.uniform(-3, 2, n)
        a = rng.uniform(0.0, np.pi, n)
        m2 = rng.uniform(0.1, 2.0, n)
        d2 = frg.make_desc(3, 24, 8.0, n_x=12, n_phi=8)
        _same_bits(_both(env, ctx, d2, n, ext=np.concatenate([p, a]), m2=m2, Z=Z))


def test_fp32_chunked_slots_then_smaller(env):
    frg, torch = env
    with frg.Context(0) as ctx:
        rng = np.random.default_rng(11)
        Z = wl.dressing_table(5)
        # 64 momenta x 512 x 256 nodes: 8 radial chunks, one amplification slot per point
        n = 64
        p = 10.0 ** rng.uniform(-3, 2, n)
        m2 = rng.uniform(-0.95, -0.5, n)
        desc = frg.make_desc(2, 512, 10.0, n_x=256, precision=1, near_pole_tau=0.1)
        _same_bits(_both(env, ctx, desc, n, ext=p, m2=m2, Z=Z, err=True))
        # the batch entry point first this time (rules cached), then the smaller one
        n2 = 40
        d2 = frg.make_desc(2, 48, 10.0, n_x=16, precision=1, near_pole_tau=0.1)
        _same_bits(_both(env, ctx, d2, n2, ext=p[:n2], m2=m2[:n2], Z=Z, err=True,
                         order=("batch", "noalloc")))


@pytest.mark.parametrize("case", ["lpa", "two_point_dm2_dz", "finite_T", "lpa_T",
                                  "three_point_T_dm2_dz"])
def test_families_two_calls(env, case):
    frg, torch = env
    rng = np.random.default_rng(3)
    Z = wl.dressing_table(2)
    with frg.Context(0) as ctx:
        for n, nq, nx in ((300, 64, 32), (37, 20, 9)):
            p = 10.0 ** rng.uniform(-3, 2, n)
            m2 = rng.uniform(0.1, 2.0, n)
            if case == "lpa":
                desc = frg.make_desc(1, nq, 6.0)
                res = _both(env, ctx, desc, n, m2=m2, dm2=True)
            elif case == "two_point_dm2_dz":
                desc = frg.make_desc(2, nq, 10.0, n_x=nx)
                res = _both(env, ctx, desc, n, ext=p, m2=m2, Z=Z, dm2=True, dz=True)
            elif case == "finite_T":
                desc = frg.make_desc(5, nq, 10.0, n_x=nx, T=0.2, freq_max=10.0, n_tail=4,
                                     statistics=1)
                p0 = np.pi * 0.2 * np.exp(-1.0 / (np.pi * 0.2)) * np.ones(n)
                res = _both(env, ctx, desc, n, ext=np.concatenate([p, p0]), m2=m2, Z=Z)
            elif case == "three_point_T_dm2_dz":
                desc = frg.make_desc(6, nq // 4, 10.0, n_x=nx // 2, n_phi=6, T=0.2,
                                     freq_max=6.0, n_tail=3)
                al = rng.uniform(0.0, np.pi, n)
                p01 = 2 * np.pi * 0.2 * rng.integers(-1, 2, n)
                p02 = 2 * np.pi * 0.2 * rng.integers(-1, 2, n)
                res = _both(env, ctx, desc, n, ext=np.concatenate([p, al, p01, p02]), m2=m2,
                            Z=Z, dm2=True, dz=True)
            else:
                desc = frg.make_desc(4, nq, 6.0, T=0.1, freq_max=8.0, freq_scaled=True)
                res = _both(env, ctx, desc, n, m2=m2)
            _same_bits(res)


def test_rejects_requests_beyond_the_scratch(env):
    frg, torch = env
    with frg.Context(0) as ctx:
        # finite temperature, T = 0.005 k and |w| <= 10 k: 637 frequencies x 64 radial nodes =
        # 40768 radial indices; 100 momenta are radially chunked, so their contributions alone
        # take 100 x 40768 doubles = 32.6 MB > 16 MiB
        n = 100
        desc = frg.make_desc(5, 64, 10.0, n_x=8, T=0.005, freq_max=10.0)
        te = _d(torch, np.concatenate([np.linspace(0.1, 5.0, n), np.zeros(n)]))
        out = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        with pytest.raises(frg.FrgError) as ei:
            ctx.integrate_noalloc(desc, out, ext=te, m2_scalar=0.5)
        assert ei.value.status == frg.FRG_E_NOMEM
        assert "static scratch" in str(ei.value)
        torch.cuda.synchronize()
        assert bool(torch.isnan(out).all().item())  # nothing was enqueued
