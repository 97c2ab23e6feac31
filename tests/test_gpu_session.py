"""Serving loop on the GPU: every request's result matches the FP64 oracle, is bitwise identical
to the same request evaluated alone (frg_integrate_batch), and admission under a small HBM budget
delays requests without failing them."""
import math
import threading

import numpy as np
import pytest

import oracle
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


def _request(i, frg, small=False):
    """Host buffers of a mixed request (families, sizes, precisions)."""
    rng = np.random.default_rng(900 + i)
    fam = 1 + i % 3
    prec = (i // 3) % 2
    n_ext = int(rng.integers(5, 40 if small else 300))
    if fam == 1:
        desc = frg.make_desc(1, int(rng.integers(8, 64)), 6.0, precision=prec, near_pole_tau=0.1)
        ext = None
    elif fam == 2:
        desc = frg.make_desc(2, int(rng.integers(8, 40)), 10.0, n_x=int(rng.integers(4, 24)),
                             precision=prec, near_pole_tau=0.1)
        ext = 10 ** rng.uniform(-3, 2, n_ext)
    else:
        desc = frg.make_desc(3, int(rng.integers(4, 16)), 10.0, n_x=int(rng.integers(4, 12)),
                             n_phi=int(rng.integers(2, 9)), precision=prec, near_pole_tau=0.1)
        ext = np.concatenate([10 ** rng.uniform(-3, 2, n_ext), rng.uniform(0, math.pi, n_ext)])
    m2 = rng.uniform(0.05, 2.0, n_ext)
    Z = wl.dressing_table(50 + i) if fam > 1 else None
    return dict(desc=desc, ext=ext, m2=m2, Z=Z, n=n_ext, fam=fam, prec=prec,
                out=np.full(n_ext, np.nan), err=np.full(n_ext, np.nan))


def _host_batch(frg, r):
    zt = frg.frg_log_table(None if r["Z"] is None else r["Z"].ctypes.data,
                           0 if r["Z"] is None else r["Z"].size, wl.Z_XMIN, wl.Z_XMAX)
    return frg.frg_batch(r["n"], None if r["ext"] is None else r["ext"].ctypes.data,
                         r["m2"].ctypes.data, 0.0, zt, r["out"].ctypes.data, r["err"].ctypes.data)


def _alone(env, r):
    frg, ctx, torch = env
    d = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    out = torch.empty(r["n"], dtype=torch.float64, device="cuda")
    ctx.integrate(r["desc"], out, ext=None if r["ext"] is None else d(r["ext"]), m2=d(r["m2"]),
                  Z=None if r["Z"] is None else d(r["Z"]), x_min=wl.Z_XMIN, x_max=wl.Z_XMAX)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_session_mix_equals_alone_and_oracle(env):
    frg, ctx, torch = env
    cfg = frg.frg_session_config(3, 256 << 20, 20, 0)
    s = frg.frg_session_open(ctx.handle, cfg)
    reqs = [_request(i, frg) for i in range(24)]
    tickets = [frg.frg_session_submit(s, r["desc"], _host_batch(frg, r), -1) for r in reqs]
    for t in tickets:
        assert frg.frg_session_wait(s, t, 60000) == frg.FRG_OK
    st = frg.frg_session_stats(s)
    frg.frg_session_close(s)
    assert st.completed == 24 and st.failed == 0
    for r in reqs:
        alone = _alone(env, r)
        assert np.array_equal(r["out"], alone), "result differs between the mix and alone"
        if r["prec"] == 0:
            d = r["desc"]
            kw = dict(n_x=d.n_x, n_phi=d.n_phi, m2=r["m2"], Z=r["Z"])
            ext = None if r["fam"] == 1 else (r["ext"] if r["fam"] == 2 else
                                              (r["ext"][:r["n"]], r["ext"][r["n"]:]))
            ref = oracle.integrate(r["fam"], d.n_q, d.q_max, ext=ext, **kw)
            assert np.max(np.abs(r["out"] - ref) / ref) <= 1e-12
        else:
            assert np.all(np.isfinite(r["err"])) and np.all(r["err"] > 0)


def test_session_admission_small_budget_and_threads(env):
    frg, ctx, torch = env
    reqs = [_request(100 + i, frg, small=True) for i in range(40)]
    biggest = max(r["n"] * r["desc"].n_q * 8 + 4 * 256 + r["n"] * 32 for r in reqs)
    cfg = frg.frg_session_config(4, 4 * biggest, 20, 0)  # only a few requests fit at once
    s = frg.frg_session_open(ctx.handle, cfg)
    errs = []

    def client(chunk):
        try:
            for r in chunk:
                t = frg.frg_session_submit(s, r["desc"], _host_batch(frg, r), -1)
                assert frg.frg_session_wait(s, t, 60000) == frg.FRG_OK
        except Exception as e:  # pragma: no cover
            errs.append(e)

    th = [threading.Thread(target=client, args=(reqs[i::8],)) for i in range(8)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    st = frg.frg_session_stats(s)
    frg.frg_session_close(s)
    assert not errs and st.completed == 40 and st.failed == 0 and st.rejected == 0
    for r in reqs:
        assert np.array_equal(r["out"], _alone(env, r))


def test_session_resident_table(env):
    frg, ctx, torch = env
    s = frg.frg_session_open(ctx.handle, frg.frg_session_config(2, 64 << 20, 20, 0))
    Z = wl.dressing_table(77)
    tid = frg.frg_session_register_table(s, Z.ctypes.data, Z.size, wl.Z_XMIN, wl.Z_XMAX)
    p = wl.momenta_log(33)
    out = np.full(p.size, np.nan)
    desc = frg.make_desc(2, 24, 10.0, n_x=12)
    b = frg.frg_batch(p.size, p.ctypes.data, None, 0.7, frg.frg_log_table(None, 0, 0, 0),
                      out.ctypes.data, None)
    t = frg.frg_session_submit(s, desc, b, tid)
    assert frg.frg_session_wait(s, t, 30000) == frg.FRG_OK
    frg.frg_session_close(s)
    ref = oracle.integrate(2, 24, 10.0, n_x=12, ext=p, m2_scalar=0.7, Z=Z)
    assert np.max(np.abs(out - ref) / ref) <= 1e-12
