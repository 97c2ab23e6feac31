"""Benchmark of the batched loop-integral hot path on one MI355X.

Step (default workload) = one flow right-hand-side batch of the three-point vertex workload: 8
right-hand sides, each 1024 external (|p|, alpha) pairs x (64 radial x 32 cos1 x 16 phi
Gauss-Legendre nodes) with its own tabulated dressing Z (256-point log grid) and masses m^2 in
U[0.1, 2], float64 -- evaluated by one fused frg_integrate_multi launch (268,435,456 integrand
nodes), the largest configuration that fits one GPU.  Inputs are resident in HBM before the
timed region.  Before the warmup steps the step runs untimed for --warm-seconds, long enough for
the GPU's clocks to settle under load; the timed steps then measure the sustained rate.

Printed (one JSON line): Gnodes/s, ms per step, the roofline of the dominant kernel (algorithmic
FP64 FLOPs per node x nodes per launch / average kernel time from HIP events on the launch
stream, against the MI355X FP64 vector peak, next to the hardware-counted FLOPs of the committed
profile), the FP64 oracle timed on the host cores on a bounded sample of the same workload, and
secondary figures for the other workloads (LPA batch, two-point batch, finite temperature, the
float32 precision form, derivatives, right-hand-side latency, the flow steppers and the serving
loop against the plain per-batch path).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# The serving measurement keeps up to six launches in flight on six streams; they overlap on
# the device only on separate hardware queues, and HIP gives a process four by default (shared
# with torch's and the library's other streams).  Set before anything initialises HIP.
os.environ.setdefault("GPU_MAX_HW_QUEUES", "12")

FP64_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
FP32_PEAK_TFLOPS = 157.3  # packed FP32 (v_pk_fma_f32); unpacked float32 tops out at half
# Algorithmic FP64 work per integrand node, in FLOPs as the hardware counts them (FMA = 2).
# The elementary sequences are the counted values of the FLOP-count probe (frg_flop_probe: the
# FP64 FLOP counter of one dispatch per sequence, less the bare loop, per call; summary and
# command in profiles/flop_probe.md): table log 12, expm1(-y) 29, Newton reciprocal 5.  Around
# them each family's node term adds plain arithmetic, counted from its code:
#   LPA:         the denominator (1: the rule holds q^2 + R per node, the mass enters in units
#                of k^2), the reciprocal, its square (1), accumulate (2);
#   two-point:   l^2 (2), the log, the dressing coordinate (2) and lerp (3), expm1, l^2 e (2),
#                the single-reciprocal denominator (4), the reciprocal, -E x (1), accumulate
#                (2) -- 16 + log + expm1 + reciprocal;
#   three-point: the second leg's l^2 (2), its propagator (the two-point term without l^2 and
#                accumulation), the product into the sum (2); the first leg (l^2 and a
#                propagator, 2 + 58) once per (radial, cos1) pair, i.e. 60/n_phi per node plus
#                4/n_phi of per-pair geometry.
SEQ_FLOP = {"log": 12.0, "expm1": 29.0, "rcp": 5.0}
_PROP = SEQ_FLOP["log"] + 2.0 + 3.0 + SEQ_FLOP["expm1"] + 2.0 + 4.0 + SEQ_FLOP["rcp"] + 1.0
FLOP_LPA = 1.0 + SEQ_FLOP["rcp"] + 1.0 + 2.0
FLOP_TWO = 2.0 + _PROP + 2.0


def flop_three(n_phi):
    return 2.0 + _PROP + 2.0 + (2.0 + _PROP + 4.0) / n_phi


# the standard workloads' three-point rule has 16 phi nodes
FLOP_PER_NODE = {1: FLOP_LPA, 2: FLOP_TWO, 3: flop_three(16), 5: FLOP_TWO, 6: flop_three(16)}
# an earlier FLOP-equivalent estimate (transcendentals as 25/25/10), kept for comparison
FLOP_PER_NODE_SURVEY = {1: 15.0, 2: 74.0, 3: 147.0, 5: 74.0, 6: 147.0}
# Two-point nodes with y = l2/k^2 >= 38 have an exponential below double precision: their exact
# value needs no expm1 and a plain reciprocal of Z l2 + m2 instead of the single-reciprocal form
# (l^2 e, the outer FMA's extra term and -E x): expm1 + 5 FLOPs fewer.  The kernel takes that
# path per wavefront when all its lanes are in that far field.
FAR_Y = 38.0
FAR_FLOP_SAVED = SEQ_FLOP["expm1"] + 5.0


def two_point_far_fraction(p, n_q, q_max, n_x):
    """Fraction of two-point nodes (k = 1) whose exponential is below double precision."""
    xq, _ = np.polynomial.legendre.leggauss(n_q)
    q = 0.5 * q_max * (xq + 1.0)
    x, _ = np.polynomial.legendre.leggauss(n_x)
    P = np.asarray(p, dtype=np.float64)
    l2 = q[None, :, None] ** 2 + P[:, None, None] ** 2 + 2.0 * q[None, :, None] * P[:, None, None] \
        * x[None, None, :]
    return float(np.mean(l2 >= FAR_Y))


def three_point_far_fractions(P, A, n_q, q_max, n_x, n_phi):
    """Fractions of three-point second-leg nodes and first-leg (radial, cos1) pairs (k = 1)
    whose exponential is below double precision (y = l2/k^2 >= FAR_Y)."""
    xq, _ = np.polynomial.legendre.leggauss(n_q)
    q = 0.5 * q_max * (xq + 1.0)
    x, _ = np.polynomial.legendre.leggauss(n_x)
    sx = np.sqrt(1.0 - x * x)
    xp, _ = np.polynomial.legendre.leggauss(n_phi)
    cph = np.cos(0.5 * np.pi * (xp + 1.0))
    far2 = far1 = 0.0
    for i in range(0, P.size, 64):
        p = P[i:i + 64, None, None, None]
        a = A[i:i + 64, None, None, None]
        Q = q[None, :, None, None]
        c0 = Q * Q + p * p
        l1 = c0 + 2.0 * Q * p * x[None, None, :, None]
        l2 = c0 - 2.0 * Q * p * (x[None, None, :, None] * np.cos(a)
                                 + sx[None, None, :, None] * cph[None, None, None, :] * np.sin(a))
        far2 += float(np.count_nonzero(l2 >= FAR_Y))
        far1 += float(np.count_nonzero(l1 >= FAR_Y))
    return far2 / (P.size * n_q * n_x * n_phi), far1 / (P.size * n_q * n_x)


def ft_frequency_count(T, lam, n_tail, fermionic=False):
    """Nodes of the Matsubara frequency rule: every |2 pi T (n + eta)| <= lam plus the tail nodes
    of both sides."""
    import math

    eta = 0.5 if fermionic else 0.0
    n_hi = math.floor(lam / (2.0 * math.pi * T) - eta)
    return 2 * n_hi + (2 if fermionic else 1) + 2 * n_tail


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_sha():
    """Hash of the device sources with line comments and blank lines removed (comment edits do
    not change the kernels the traffic counters were taken on)."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in ("frg_kernels.hip", "frg_math.hpp", "frg_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2412_13043_amd", "csrc", f)) as fh:
            for line in fh:
                code = re.sub(r"//.*", "", line).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_counters(workload):
    """Per-launch counter figures of the workload's dominant kernel from the committed rocprofv3
    summaries (profiles/kernel_counters.json: HBM bytes from FETCH_SIZE + WRITE_SIZE scaled by a
    plain copy of known size, and the FP64 FLOP counter x 64 lanes), or {} when the kernel
    sources have changed since those counters were taken."""
    path = os.path.join(ROOT, "profiles", "kernel_counters.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return {}
    if d.get("source_sha256_16") != kernel_source_sha():
        return {}
    return d.get("workloads", {}).get(workload, {})


def _dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), dtype=torch.float64,
                        device="cuda")


def warm_clocks(torch, fn, seconds):
    """Untimed calls of fn until `seconds` of wall time have passed; returns their number.  The
    GPU raises its clocks over the first few tens of milliseconds of sustained load (the
    two-point batch launch takes 0.25 ms cold and 0.193 ms from about the 150th launch on, then
    holds that rate for seconds), so a timed region that starts cold measures the ramp."""
    n = 0
    t0 = time.perf_counter()
    while True:
        fn()
        n += 1
        if n % 4 == 0:
            torch.cuda.synchronize()
            if time.perf_counter() - t0 >= seconds:
                return n


def time_kernel(torch, fn, steps, warmup):
    """Run fn warmup + steps times; return (wall seconds for the timed steps, average ms per step
    from one pair of HIP events around them on the launch stream).  Events between steps would
    put their own markers into the stream, so the timed region is bracketed only once."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record(stream)
    for _ in range(steps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return t1 - t0, [a.elapsed_time(b) / steps]


def two_point_batch_setup(torch, frg, B=256, precision=0, seed_m2=None, tau=0.1, regulator=0,
                          dm2=False):
    from paper_2412_13043_amd import workloads as wl

    if seed_m2 is None:
        p, m2, Zs = wl.two_point_batch(B)
        m2a = None
    else:
        p, m2a, Zs = wl.near_pole_batch(B)
        m2 = 0.0
    tp = _dev(torch, p)
    tZ = _dev(torch, Zs)
    tm = _dev(torch, m2a) if m2a is not None else None
    out = torch.empty((B, p.size), dtype=torch.float64, device="cuda")
    err = torch.empty((B, p.size), dtype=torch.float64, device="cuda") if precision else None
    dout = torch.empty((B, p.size), dtype=torch.float64, device="cuda") if dm2 else None
    desc = frg.make_desc(2, wl.TWO_NQ, wl.TWO_QMAX, n_x=wl.TWO_NX, precision=precision,
                         near_pole_tau=tau if precision else 0.0, regulator=regulator)
    batches = [frg.make_batch(p.size, out[b], ext=tp, m2=None if tm is None else tm[b],
                              m2_scalar=m2, Z=tZ[b], x_min=wl.Z_XMIN, x_max=wl.Z_XMAX,
                              err_out=None if err is None else err[b],
                              dout=None if dout is None else dout[b]) for b in range(B)]
    keep = (tp, tZ, tm, out, err, dout)
    nodes = B * p.size * wl.TWO_NQ * wl.TWO_NX
    return [desc] * B, batches, out, err, nodes, keep


def host_description():
    """The host CPU as the oracle timings see it: model, sockets, physical cores, logical CPUs,
    the CPUs this process may use, and the clock (lscpu's maximum MHz where it reports one,
    else /proc/cpuinfo's current MHz)."""
    import platform
    import subprocess

    d = {"cpu_model": platform.processor() or "unknown", "logical_cpus": os.cpu_count()}
    try:
        d["cpus_available"] = len(os.sched_getaffinity(0))
    except AttributeError:
        d["cpus_available"] = os.cpu_count()
    phys, sockets, mhz = set(), set(), []
    try:
        cur = {}
        with open("/proc/cpuinfo") as f:
            for line in list(f) + [""]:
                if not line.strip():
                    if "physical id" in cur:
                        sockets.add(cur["physical id"])
                        phys.add((cur["physical id"], cur.get("core id", "")))
                    cur = {}
                    continue
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                cur[k] = v
                if k == "model name":
                    d["cpu_model"] = v
                elif k == "cpu MHz":
                    mhz.append(float(v))
    except OSError:
        pass
    d["sockets"] = len(sockets) or None
    d["physical_cores"] = len(phys) or None
    d["mhz_current_mean"] = round(float(np.mean(mhz)), 1) if mhz else None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k == "CPU max MHz":
                d["mhz_max"] = float(v)
            elif k == "Socket(s)" and v.isdigit():
                d["sockets"] = int(v)
            elif k == "Core(s) per socket" and v.isdigit():
                d["cores_per_socket"] = int(v)
            elif k == "Thread(s) per core" and v.isdigit():
                d["threads_per_core"] = int(v)
    except (OSError, subprocess.SubprocessError):
        pass
    return d


def cpu_baseline(target_seconds=12.0):
    """FP64 oracle on the host cores, on a bounded sample of the timed workload (the three-point
    batch): (p, alpha) pairs of its right-hand sides in order, each with its right-hand side's
    masses and dressing table, disjoint pair ranges in parallel threads."""
    import oracle
    from paper_2412_13043_amd import workloads as wl

    P, A, m3, Z3 = wl.three_point_batch()
    threads = min(len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                  else (os.cpu_count() or 1), 16)
    per_pair = wl.THREE_NQ * wl.THREE_NX * wl.THREE_NPHI
    block = 8 * threads  # pairs per round: 8 per thread
    nodes_done = pairs_done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < target_seconds:
        b = (pairs_done // P.size) % m3.shape[0]
        lo = pairs_done % P.size
        idx = np.arange(lo, min(lo + block, P.size))
        chunks = np.array_split(idx, threads)
        ths = [threading.Thread(target=oracle.integrate,
                                args=(oracle.THREE_POINT, wl.THREE_NQ, wl.THREE_QMAX),
                                kwargs=dict(n_x=wl.THREE_NX, n_phi=wl.THREE_NPHI,
                                            ext=(P[c], A[c]), m2=m3[b][c], Z=Z3[b]))
               for c in chunks if c.size]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        pairs_done += idx.size
        nodes_done += idx.size * per_pair
    el = time.perf_counter() - t0
    host = host_description()
    return {"value": round(nodes_done / el / 1e9, 6), "unit": "Gnodes/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{pairs_done} (p, alpha) pairs of the three-point batch (64x32x16 nodes "
                      f"each, float64, C -O2 libm), {threads} threads over disjoint pair ranges, "
                      f"{el:.1f} s",
            "host": host}


def oracle_timings(threads_max=16, seconds=1.5):
    """The FP64 oracle per workload on the host: seconds per right-hand side with one thread and
    with `threads_max` threads over disjoint external-point ranges, plus the host description."""
    import platform

    import oracle
    from paper_2412_13043_amd import workloads as wl

    host = host_description()
    avail = host.get("cpus_available") or 1
    threads = min(avail, threads_max)

    def rate(call, n_points, nodes_per_point, n_threads):
        """Repeat `call(lo, hi)` over point ranges split across n_threads for >= `seconds`."""
        chunks = np.array_split(np.arange(n_points), n_threads)
        done = 0
        t0 = time.perf_counter()
        while True:
            ths = [threading.Thread(target=call, args=(c[0], c[-1] + 1)) for c in chunks if c.size]
            for t in ths:
                t.start()
            for t in ths:
                t.join()
            done += n_points
            el = time.perf_counter() - t0
            if el >= seconds:
                return done * nodes_per_point / el  # nodes per second

    res = {"host": dict(host, threads_used=threads)}
    # LPA: 64 rho points x GL32 per right-hand side; the 4096-RHS batch, one point = one integral
    rho, u, m2 = wl.lpa_batch()
    m2f = m2.reshape(-1)
    lpa = lambda lo, hi: oracle.integrate(oracle.LPA, wl.LPA_NQ, wl.LPA_QMAX, m2=m2f[lo:hi])
    # two-point: 256 momenta x 64x32 per right-hand side
    p, m2s, Z = wl.two_point()
    two = lambda lo, hi: oracle.integrate(oracle.TWO_POINT, wl.TWO_NQ, wl.TWO_QMAX,
                                          n_x=wl.TWO_NX, ext=p[lo:hi], m2_scalar=m2s, Z=Z)
    # three-point: 1024 (p, alpha) pairs x 64x32x16 per right-hand side
    P, A, m3, Z3 = wl.three_point()
    three = lambda lo, hi: oracle.integrate(oracle.THREE_POINT, wl.THREE_NQ, wl.THREE_QMAX,
                                            n_x=wl.THREE_NX, n_phi=wl.THREE_NPHI,
                                            ext=(P[lo:hi], A[lo:hi]), m2=m3[lo:hi], Z=Z3)
    # finite-temperature three-point: 1024 pairs x 47 frequencies x 64x32x16 per right-hand
    # side (its first 256 pairs timed; one thread: 16 of them)
    Pf, Af, f1, f2, mf, Zf = wl.three_point_ft_batch(1)
    n_f = ft_frequency_count(wl.FT_T, wl.FT_FREQ_MAX, wl.FT_N_TAIL)
    three_ft = lambda lo, hi: oracle.integrate_ft(
        oracle.THREE_POINT_T, wl.THREE_NQ, wl.THREE_QMAX, n_x=wl.THREE_NX, n_phi=wl.THREE_NPHI,
        T=wl.FT_T, freq_max=wl.FT_FREQ_MAX, n_tail=wl.FT_N_TAIL,
        ext=(Pf[lo:hi], Af[lo:hi], f1[lo:hi], f2[lo:hi]), m2=mf[0][lo:hi], Z=Zf[0])
    npp_ft = n_f * wl.THREE_NQ * wl.THREE_NX * wl.THREE_NPHI
    cases = {
        "lpa": (lpa, m2f.size, wl.LPA_NQ, wl.LPA_N_RHO * wl.LPA_NQ, 1.0),
        "two_point": (two, p.size, wl.TWO_NQ * wl.TWO_NX, p.size * wl.TWO_NQ * wl.TWO_NX, 1.0),
        # one thread: a 64-pair sample of the right-hand side
        "three_point": (three, P.size, wl.THREE_NQ * wl.THREE_NX * wl.THREE_NPHI,
                        P.size * wl.THREE_NQ * wl.THREE_NX * wl.THREE_NPHI, 64 / P.size),
        "three_point_finite_T": (three_ft, 256, npp_ft, Pf.size * npp_ft, 16 / 256),
    }
    # the O(4) LPA flow of the stepper benchmark, integrated by the oracle's stepper
    import math

    from oracle import stepper as rk

    rho_s = wl.lpa_rho_grid()

    def flow(t, u):
        k = math.exp(-t)
        return oracle.lpa_flow_rhs(rho_s, u, wl.LPA_NQ, wl.LPA_QMAX, k=k, n_comp=4,
                                   m2_floor=-0.9 * k * k)

    st = rk.Dopri5(flow, 0.3 + rho_s, **STEPPER_CFG)
    t0 = time.perf_counter()
    st.advance(STEPPER_T_END["lpa"])
    res["lpa_flow_stepper"] = {"wall_ms": round((time.perf_counter() - t0) * 1e3, 2),
                               "accepted": st.accepted, "rejected": st.rejected,
                               "rhs_evals": st.evals, "threads": 1}
    for name, (call, n_pts, npp, nodes_rhs, single_frac) in cases.items():
        out = {"nodes_per_rhs": nodes_rhs}
        for nt in (1, threads):
            n_use = max(int(n_pts * single_frac), nt) if nt == 1 else n_pts
            r = rate(call, n_use, npp, nt)
            out[f"threads_{nt}"] = {"gnodes_per_s": round(r / 1e9, 5),
                                    "seconds_per_rhs": round(nodes_rhs / r, 6)}
        res[name] = out
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--warm-seconds", type=float, default=0.3,
                    help="untimed calls for this long before the warmup steps (clock ramp)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the secondary workloads")
    ap.add_argument("--serving-seconds", type=float, default=15.0,
                    help="measured seconds of the serving replay per offered load and path")
    ap.add_argument("--serving-warm", type=float, default=2.0,
                    help="seconds of arrivals excluded at the start of each serving replay")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving measurement (after the timed line)")
    ap.add_argument("--serving-slots", type=int, default=6,
                    help="launch slots (max_inflight) of the served session")
    ap.add_argument("--serving-poll-us", type=int, default=2,
                    help="how often a slot checks its launch for completion (microseconds)")
    ap.add_argument("--serving-paths", default="both", choices=["both", "session"],
                    help="serve the traces through the session and the plain path, or the "
                         "session only")
    ap.add_argument("--workload", default="three_point_8",
                    choices=["two_point_256", "three_point_8", "lpa_4096", "two_point_ft_16",
                             "three_point_ft_2", "two_point_256_near_pole",
                             "two_point_256_near_pole_fp32"],
                    help="workload of the timed line (default: the three-point batch, the "
                         "largest single-GPU configuration); the others exist so that each "
                         "family's kernel can be timed and profiled on its own")
    ap.add_argument("--flop-probe", action="store_true",
                    help="only run the FLOP-count probe kernels (one dispatch per elementary "
                         "sequence, for a profiler's FP64 FLOP counters)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (the "
                         "reference kernel for scaling FETCH_SIZE/WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the loop-integral "
              "path is measured on a single MI355X", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.flop_probe:
        from paper_2412_13043_amd import frg

        blocks, iters = 1024, 4096
        out = torch.empty(blocks * 64, dtype=torch.float64, device="cuda")
        for seq in range(5):
            frg.frg_flop_probe(seq, blocks, iters, out)
        torch.cuda.synchronize()
        print(json.dumps({"flop_probe": {"sequences": ["loop", "log_tab", "expm1_neg", "exp_neg",
                                                       "rcp_nr"],
                                         "evaluations_per_dispatch": blocks * 64 * iters}}))
        return
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8}))
        return

    from paper_2412_13043_amd import frg
    from paper_2412_13043_amd import workloads as wl

    ctx = frg.Context(0)
    log(f"bench: {args.workload} setup")
    step, nodes, family, kernel, config, keep = workload_setup(torch, frg, wl, ctx,
                                                                args.workload)

    clock_calls = warm_clocks(torch, step, args.warm_seconds) if args.warm_seconds > 0 else 0
    log(f"bench: timing {args.steps} steps after {clock_calls} clock-warming calls and "
        f"{args.warmup} warmup")
    wall, ev_ms = time_kernel(torch, step, args.steps, args.warmup)
    ms_per_step = wall / args.steps * 1e3
    value = nodes * args.steps / wall / 1e9
    avg_ms = float(np.mean(ev_ms))
    flops = FLOP_PER_NODE[family] * nodes
    achieved = flops / (avg_ms * 1e-3) / 1e12
    # the finite-temperature workload has the two-point workload's spatial nodes and momenta
    far = two_point_far_fraction(wl.two_point()[0], wl.TWO_NQ, wl.TWO_QMAX, wl.TWO_NX) \
        if family in (2, 5) else 0.0
    required = FLOP_PER_NODE[family] - FAR_FLOP_SAVED * far
    if family == 3:
        # the second leg per node and the first leg per (radial, cos1) pair, each skipping the
        # exponential in the far field
        P3, A3 = wl.three_point()[:2]
        far, far1 = three_point_far_fractions(P3, A3, wl.THREE_NQ, wl.THREE_QMAX, wl.THREE_NX,
                                              wl.THREE_NPHI)
        required = FLOP_PER_NODE[3] - FAR_FLOP_SAVED * (far + far1 / wl.THREE_NPHI)
    counters = measured_counters(args.workload)
    per_s = 1.0 / (avg_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS
    counted = counters.get("counted_fp64_flop_per_launch")
    res = {
        "metric": "integrand Gnodes/s + % FP64/FP32 vector peak; p50/p99 RHS latency",
        "value": round(value, 3),
        "unit": "Gnodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "clock_warmup": {"seconds": args.warm_seconds, "calls": clock_calls},
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": config.get("precision", "f64"),
        "data": "synthetic",
        "config": config,
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                     "traffic": counters.get("traffic_bytes"),
                     "kernel": kernel, "avg_kernel_ms": round(avg_ms, 4),
                     "flop_per_node": FLOP_PER_NODE[family],
                     "flop_per_node_basis": "counted elementary sequences (profiles/"
                                            "flop_probe.md) + the node term's arithmetic",
                     # the hardware FP64 FLOP counter of this kernel (committed profile) over
                     # the time measured here
                     "frac_counted": round(counted * per_s, 4) if counted else None,
                     "counted_flop_per_node": round(counted / nodes, 2) if counted else None,
                     # the work the nodes strictly need (the far-field ones skip expm1)
                     "far_field_fraction": round(far, 4),
                     "flop_per_node_required": round(required, 2),
                     "frac_required": round(required * nodes * per_s, 4),
                     # the earlier FLOP-equivalent estimate, for comparison
                     "flop_per_node_survey": FLOP_PER_NODE_SURVEY[family],
                     "frac_survey": round(FLOP_PER_NODE_SURVEY[family] * nodes * per_s, 4)},
    }
    extra = {}
    if not args.no_extra:
        if args.serving_only:
            extra = {"serving": serving(torch, frg, wl, ctx, seconds=args.serving_seconds,
                                        warm=args.serving_warm,
                                        plain=args.serving_paths == "both",
                                        max_inflight=args.serving_slots,
                                        poll_us=args.serving_poll_us)}
        else:
            extra = secondary(torch, frg, wl, ctx, serving_seconds=args.serving_seconds,
                              serving_warm=args.serving_warm)
    if extra:
        res["extra"] = extra
    if not args.no_cpu:
        log("bench: CPU oracle baseline")
        res["cpu_baseline"] = cpu_baseline()
        if not args.no_extra:
            log("bench: oracle per workload, one thread and all threads")
            res.setdefault("extra", {})["oracle_cpu"] = oracle_timings()
    torch.cuda.synchronize()
    ctx.close()
    print(json.dumps(res), flush=True)


def workload_setup(torch, frg, wl, ctx, name):
    """Inputs resident in HBM and a step function for one timed workload."""
    if name == "two_point_256":
        descs, batches, out, _, nodes, keep = two_point_batch_setup(torch, frg)
        config = {"workload": "two-point vertex flow d=4: 256 right-hand sides x 256 momenta x "
                              "64x32 GL nodes, per-RHS tabulated Z, m2=0.5, float64, one fused "
                              "frg_integrate_multi launch",
                  "nodes_per_step": nodes, "rhs_per_step": 256}
        return (lambda: ctx.integrate_multi(descs, batches), nodes, 2, "frg::multi_kernel<2, 0, 0, false>",
                config, keep)
    if name in ("two_point_256_near_pole", "two_point_256_near_pole_fp32"):
        prec = 1 if name.endswith("fp32") else 0
        descs, batches, out, _, nodes, keep = two_point_batch_setup(torch, frg, precision=prec,
                                                                    seed_m2=4, tau=0.1)
        config = {"workload": "two-point vertex flow d=4 near the pole: 256 right-hand sides x "
                              "256 momenta x 64x32 GL nodes, per-RHS tabulated Z, m2 in "
                              "U[-0.95,-0.5], " + ("float32 form (tau = 0.1)" if prec else
                                                   "float64") +
                              ", one fused frg_integrate_multi launch",
                  "nodes_per_step": nodes, "rhs_per_step": 256,
                  "precision": "f32" if prec else "f64"}
        return (lambda: ctx.integrate_multi(descs, batches), nodes, 2,
                f"frg::multi_kernel<2, {prec}, 0, false>", config, keep)
    if name == "three_point_8":
        P, A, m3, Z3 = wl.three_point_batch()
        text = _dev(torch, np.concatenate([P, A]))
        tm3, tZ3 = _dev(torch, m3), _dev(torch, Z3)
        o3 = torch.empty((8, P.size), dtype=torch.float64, device="cuda")
        d3 = frg.make_desc(3, wl.THREE_NQ, wl.THREE_QMAX, n_x=wl.THREE_NX, n_phi=wl.THREE_NPHI)
        b3 = [frg.make_batch(P.size, o3[b], ext=text, m2=tm3[b], Z=tZ3[b], x_min=wl.Z_XMIN,
                             x_max=wl.Z_XMAX) for b in range(8)]
        nodes = 8 * P.size * wl.THREE_NQ * wl.THREE_NX * wl.THREE_NPHI
        config = {"workload": "three-point vertex flow d=4: 8 right-hand sides x 1024 external "
                              "pairs x 64x32x16 GL nodes, per-RHS tabulated Z, m2 in U[0.1,2], "
                              "float64, one fused frg_integrate_multi launch",
                  "nodes_per_step": nodes, "rhs_per_step": 8}
        return (lambda: ctx.integrate_multi([d3] * 8, b3), nodes, 3, "frg::multi_kernel<3, 0, 0, false>",
                config, (text, tm3, tZ3, o3))
    if name == "two_point_ft_16":
        descs, batches, nodes, keep = two_point_ft_setup(torch, frg, wl)
        config = {"workload": "two-point vertex flow at finite temperature d=3+1: 16 right-hand "
                              "sides x 256 momenta x (47 Matsubara frequencies (T = 0.1 k, "
                              "|w| <= 10 k, 8 tail nodes per side) x 64 radial x 32 cos1 GL "
                              "nodes), per-RHS tabulated Z, m2=0.5, float64, one fused "
                              "frg_integrate_multi launch",
                  "nodes_per_step": nodes, "rhs_per_step": 16}
        return (lambda: ctx.integrate_multi(descs, batches), nodes, 5, "frg::multi_kernel<5, 0, 0, false>",
                config, keep)
    if name == "three_point_ft_2":
        descs, batches, nodes, keep = three_point_ft_setup(torch, frg, wl)
        config = {"workload": "three-point vertex flow at finite temperature d=3+1: 2 right-hand "
                              "sides x 1024 external pairs x (47 Matsubara frequencies (T = 0.1 "
                              "k, |w| <= 10 k, 8 tail nodes per side) x 64 radial x 32 cos1 x "
                              "16 phi GL nodes), leg frequencies 0 or +-2 pi T, per-RHS "
                              "tabulated Z and m2 in U[0.1,2], float64, one fused "
                              "frg_integrate_multi launch",
                  "nodes_per_step": nodes, "rhs_per_step": len(descs)}
        return (lambda: ctx.integrate_multi(descs, batches), nodes, 6, "frg::multi_kernel<6, 0, 0, false>",
                config, keep)
    rho, u, m2 = wl.lpa_batch()
    tm = _dev(torch, m2.reshape(-1))
    o1 = torch.empty(tm.numel(), dtype=torch.float64, device="cuda")
    d1 = frg.make_desc(1, wl.LPA_NQ, wl.LPA_QMAX)
    nodes = tm.numel() * wl.LPA_NQ
    config = {"workload": "LPA O(4) d=3: 4096 right-hand sides x 64 rho points x 32 GL nodes, "
                          "float64, one frg_integrate_batch launch",
              "nodes_per_step": nodes, "rhs_per_step": 4096}
    return (lambda: ctx.integrate(d1, o1, m2=tm), nodes, 1, "frg::batch_kernel<1, 0, 0, false>", config,
            (tm, o1))


def two_point_ft_setup(torch, frg, wl, B=16, mu=None):
    """The finite-temperature two-point batch, inputs resident in HBM; mu: the inner leg's
    frequency p0 - i mu (complex results, Re and Im per point)."""
    p, p0, m2, Z = wl.two_point_ft_batch(B)
    desc = frg.make_desc(frg.FRG_FAMILY_TWO_POINT_T, wl.FT_NQ, wl.FT_QMAX, n_x=wl.FT_NX,
                         T=wl.FT_T, freq_max=wl.FT_FREQ_MAX, n_tail=wl.FT_N_TAIL,
                         complex_freq=mu is not None)
    ext = [p, p0] if mu is None else [p, p0, np.full(p.size, -mu)]
    te, tZ = _dev(torch, np.concatenate(ext)), _dev(torch, Z)
    out = torch.empty((B, p.size * (1 if mu is None else 2)), dtype=torch.float64, device="cuda")
    batches = [frg.make_batch(p.size, out[b], ext=te, m2_scalar=m2, Z=tZ[b], x_min=wl.Z_XMIN,
                              x_max=wl.Z_XMAX) for b in range(B)]
    n_f = ft_frequency_count(wl.FT_T, wl.FT_FREQ_MAX, wl.FT_N_TAIL)
    nodes = B * p.size * n_f * wl.FT_NQ * wl.FT_NX
    return [desc] * B, batches, nodes, (te, tZ, out)


def three_point_ft_setup(torch, frg, wl, B=2):
    """The finite-temperature three-point batch, inputs resident in HBM."""
    P, A, p01, p02, m2, Z = wl.three_point_ft_batch(B)
    desc = frg.make_desc(frg.FRG_FAMILY_THREE_POINT_T, wl.THREE_NQ, wl.THREE_QMAX,
                         n_x=wl.THREE_NX, n_phi=wl.THREE_NPHI, T=wl.FT_T,
                         freq_max=wl.FT_FREQ_MAX, n_tail=wl.FT_N_TAIL)
    te, tm, tZ = _dev(torch, np.concatenate([P, A, p01, p02])), _dev(torch, m2), _dev(torch, Z)
    out = torch.empty((B, P.size), dtype=torch.float64, device="cuda")
    batches = [frg.make_batch(P.size, out[b], ext=te, m2=tm[b], Z=tZ[b], x_min=wl.Z_XMIN,
                              x_max=wl.Z_XMAX) for b in range(B)]
    n_f = ft_frequency_count(wl.FT_T, wl.FT_FREQ_MAX, wl.FT_N_TAIL)
    nodes = B * P.size * n_f * wl.THREE_NQ * wl.THREE_NX * wl.THREE_NPHI
    return [desc] * B, batches, nodes, (te, tm, tZ, out)


STEPPER_CFG = dict(rtol=1e-8, atol=1e-10, h0=0.05, h_min=1e-8, h_max=0.5, max_steps=100000)
STEPPER_T_END = {"lpa": 3.0, "lpa_abm4": 3.0, "lpa_rkf78": 3.0, "lpa_abm4_variable": 3.0,
                 "two_point": 1.0}


def stepper_bench(torch, frg, wl, ctx):
    """Whole flows integrated by the device stepper: the O(4) LPA flow (64 rho points, GL32) from
    k = Lambda to k = Lambda e^-3 (adaptive Dormand-Prince; fixed-step ABM4 with h = 0.05; the
    adaptive Fehlberg 7(8) pair; variable-step ABM4), and a two-point vertex flow (256 momenta,
    64x32 nodes, state m2 per momentum, dstate/dt = -I) from k = Lambda to Lambda e^-1."""
    res = {}
    rho = wl.lpa_rho_grid()
    grid = _dev(torch, rho)
    d1 = frg.make_desc(frg.FRG_FAMILY_LPA, wl.LPA_NQ, wl.LPA_QMAX)
    p, m2, Z = wl.two_point()
    tp, tZ = _dev(torch, p), _dev(torch, Z)
    d2 = frg.make_desc(frg.FRG_FAMILY_TWO_POINT, wl.TWO_NQ, wl.TWO_QMAX, n_x=wl.TWO_NX)

    def run(kind):
        if kind == "lpa":
            state = _dev(torch, 0.3 + rho)
            st = ctx.stepper(d1, state, grid, n_comp=4, m2_floor=-0.9, **STEPPER_CFG)
        elif kind == "lpa_abm4":
            # the fixed-step Adams-Bashforth-Moulton 4 PECE over the same flow, h = 0.05
            state = _dev(torch, 0.3 + rho)
            st = ctx.stepper(d1, state, grid, n_comp=4, m2_floor=-0.9, h0=0.05, max_steps=10000,
                             method=1)
        elif kind == "lpa_rkf78":
            state = _dev(torch, 0.3 + rho)
            st = ctx.stepper(d1, state, grid, n_comp=4, m2_floor=-0.9, method=2, **STEPPER_CFG)
        elif kind == "lpa_abm4_variable":
            state = _dev(torch, 0.3 + rho)
            st = ctx.stepper(d1, state, grid, n_comp=4, m2_floor=-0.9, method=3,
                             **dict(STEPPER_CFG, h0=0.01))
        else:
            state = torch.full((p.size,), m2, dtype=torch.float64, device="cuda")
            st = ctx.stepper(d2, state, tp, Z=tZ, x_min=wl.Z_XMIN, x_max=wl.Z_XMAX,
                             m2_floor=-0.9, coef=-1.0, **STEPPER_CFG)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, s = st.advance(STEPPER_T_END[kind])
        el = time.perf_counter() - t0
        st.close()
        return el, s

    for kind in ("lpa", "lpa_abm4", "lpa_rkf78", "lpa_abm4_variable", "two_point"):
        run(kind)  # plans and rules
        el, s = run(kind)
        attempts = s.accepted + s.rejected
        res[kind] = {"t_end": STEPPER_T_END[kind], "accepted": int(s.accepted),
                     "rejected": int(s.rejected), "rhs_evals": int(s.rhs_evals),
                     "wall_ms": round(el * 1e3, 3),
                     "us_per_step": round(el / max(attempts, 1) * 1e6, 2),
                     "us_per_rhs": round(el / max(int(s.rhs_evals), 1) * 1e6, 2)}
    return res


EXTRA_WARM_S = 0.1  # clock warming before each secondary timing


def secondary(torch, frg, wl, ctx, serving_seconds=15.0, serving_warm=2.0):
    """Other workloads, timed the same way (fewer steps, shorter clock warming)."""
    ex = {}
    # LPA batch: 4096 right-hand sides x 64 rho points x GL32
    log("bench: LPA batch")
    rho, u, m2 = wl.lpa_batch()
    tm = _dev(torch, m2.reshape(-1))
    o1 = torch.empty(tm.numel(), dtype=torch.float64, device="cuda")
    d1 = frg.make_desc(1, wl.LPA_NQ, wl.LPA_QMAX)
    f1 = lambda: ctx.integrate(d1, o1, m2=tm)
    warm_clocks(torch, f1, EXTRA_WARM_S)
    wall, ev = time_kernel(torch, f1, 500, 20)
    n1 = tm.numel() * wl.LPA_NQ
    ex["lpa_batch_4096"] = {"gnodes_per_s": round(n1 / (np.mean(ev) * 1e-3) / 1e9, 2),
                            "avg_kernel_ms": round(float(np.mean(ev)), 4)}
    # two-point batch: 256 right-hand sides x 256 momenta x 64x32 (one fused launch)
    log("bench: two-point batch")
    descs2, batches2, _, _, n2, keep2 = two_point_batch_setup(torch, frg)
    f2 = lambda: ctx.integrate_multi(descs2, batches2)
    warm_clocks(torch, f2, EXTRA_WARM_S)
    wall, ev = time_kernel(torch, f2, 200, 5)
    ms2 = float(np.mean(ev))
    far2 = two_point_far_fraction(wl.two_point()[0], wl.TWO_NQ, wl.TWO_QMAX, wl.TWO_NX)
    ex["two_point_batch_256"] = {
        "gnodes_per_s": round(n2 / (ms2 * 1e-3) / 1e9, 2), "avg_kernel_ms": round(ms2, 4),
        "frac_fp64_peak": round(FLOP_PER_NODE[2] * n2 / (ms2 * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                                4),
        "frac_required": round((FLOP_PER_NODE[2] - FAR_FLOP_SAVED * far2) * n2 / (ms2 * 1e-3)
                               / 1e12 / FP64_PEAK_TFLOPS, 4),
        "far_field_fraction": round(far2, 4)}
    del keep2
    # three-point batch: 8 right-hand sides x 1024 external pairs x 64x32x16
    log("bench: three-point batch")
    P, A, m3, Z3 = wl.three_point_batch()
    text = _dev(torch, np.concatenate([P, A]))
    tm3 = _dev(torch, m3)
    tZ3 = _dev(torch, Z3)
    o3 = torch.empty((8, P.size), dtype=torch.float64, device="cuda")
    d3 = frg.make_desc(3, wl.THREE_NQ, wl.THREE_QMAX, n_x=wl.THREE_NX, n_phi=wl.THREE_NPHI)
    b3 = [frg.make_batch(P.size, o3[b], ext=text, m2=tm3[b], Z=tZ3[b], x_min=wl.Z_XMIN,
                         x_max=wl.Z_XMAX) for b in range(8)]
    f3 = lambda: ctx.integrate_multi([d3] * 8, b3)
    warm_clocks(torch, f3, EXTRA_WARM_S)
    wall, ev = time_kernel(torch, f3, 40, 2)
    n3 = 8 * P.size * wl.THREE_NQ * wl.THREE_NX * wl.THREE_NPHI
    ms3 = float(np.mean(ev))
    ex["three_point_batch_8"] = {
        "gnodes_per_s": round(n3 / (ms3 * 1e-3) / 1e9, 2), "avg_kernel_ms": round(ms3, 3),
        "fp64_tflops": round(FLOP_PER_NODE[3] * n3 / (ms3 * 1e-3) / 1e12, 3),
        "frac_fp64_peak": round(FLOP_PER_NODE[3] * n3 / (ms3 * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                                4)}
    # finite temperature: the two-point workload with a Matsubara sum (same kernel body, the
    # frequency folded into the radial index)
    log("bench: finite-temperature two-point batch")
    dft, bft, nft, keep_ft = two_point_ft_setup(torch, frg, wl)
    fft = lambda: ctx.integrate_multi(dft, bft)
    warm_clocks(torch, fft, EXTRA_WARM_S)
    wall, ev = time_kernel(torch, fft, 100, 5)
    msft = float(np.mean(ev))
    ex["two_point_finite_T_batch_16"] = {
        "gnodes_per_s": round(nft / (msft * 1e-3) / 1e9, 2), "avg_kernel_ms": round(msft, 3),
        "nodes": nft,
        "frac_fp64_peak": round(FLOP_PER_NODE[5] * nft / (msft * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                                4)}
    del keep_ft
    # the same with the inner leg's frequency p0 - i mu (chemical potential mu = 0.5 k)
    log("bench: finite-temperature two-point batch at mu = 0.5")
    dmu, bmu, nmu, keep_mu = two_point_ft_setup(torch, frg, wl, mu=0.5)
    fmu = lambda: ctx.integrate_multi(dmu, bmu)
    warm_clocks(torch, fmu, EXTRA_WARM_S)
    wall, ev = time_kernel(torch, fmu, 100, 5)
    msmu = float(np.mean(ev))
    ex["two_point_finite_T_mu_batch_16"] = {
        "gnodes_per_s": round(nmu / (msmu * 1e-3) / 1e9, 2), "avg_kernel_ms": round(msmu, 3),
        "nodes": nmu, "mu": 0.5, "vs_real_frequencies": round(msft / msmu, 3)}
    del keep_mu
    log("bench: finite-temperature three-point batch")
    d6, b6, n6, keep6 = three_point_ft_setup(torch, frg, wl)
    f6 = lambda: ctx.integrate_multi(d6, b6)
    warm_clocks(torch, f6, EXTRA_WARM_S)
    wall, ev = time_kernel(torch, f6, 20, 2)
    ms6 = float(np.mean(ev))
    ex["three_point_finite_T_batch_2"] = {
        "gnodes_per_s": round(n6 / (ms6 * 1e-3) / 1e9, 2), "avg_kernel_ms": round(ms6, 3),
        "nodes": n6,
        "frac_fp64_peak": round(FLOP_PER_NODE[6] * n6 / (ms6 * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                                4)}
    del keep6
    # the same two-point batch with the paper's default regulator (polynomial-exponential s_8)
    # and with the flat one
    for name, reg, dm2 in (("two_point_poly_exp_s8_256", 1, False), ("two_point_flat_256", 2, False),
                           ("two_point_with_dI_dm2_256", 0, True)):
        log(f"bench: {name}")
        dr, br, _, _, nr, keep_r = two_point_batch_setup(torch, frg, regulator=reg, dm2=dm2)
        fr = lambda: ctx.integrate_multi(dr, br)
        warm_clocks(torch, fr, EXTRA_WARM_S)
        wall, ev = time_kernel(torch, fr, 100, 5)
        msr = float(np.mean(ev))
        ex[name] = {"gnodes_per_s": round(nr / (msr * 1e-3) / 1e9, 2),
                    "avg_kernel_ms": round(msr, 4)}
        del keep_r
    # the derivatives in the dressing-table entries (dout_dz) for one right-hand side of the
    # two-point workload: 256 momenta x 256 entries, after the integral on the same stream
    log("bench: dressing derivatives")
    pz, m2z, Zz = wl.two_point()
    tpz, tZz = _dev(torch, pz), _dev(torch, Zz)
    oz = torch.empty(pz.size, dtype=torch.float64, device="cuda")
    jz = torch.empty(pz.size * Zz.size, dtype=torch.float64, device="cuda")
    dzd = frg.make_desc(2, wl.TWO_NQ, wl.TWO_QMAX, n_x=wl.TWO_NX)
    res_z = {}
    for name, dz in (("value_only", None), ("value_and_dI_dZ", jz)):
        fz = lambda: ctx.integrate(dzd, oz, ext=tpz, m2_scalar=m2z, Z=tZz, x_min=wl.Z_XMIN,
                                   x_max=wl.Z_XMAX, dz=dz)
        warm_clocks(torch, fz, EXTRA_WARM_S)
        wall, ev = time_kernel(torch, fz, 200, 5)
        res_z[name + "_us"] = round(float(np.mean(ev)) * 1e3, 2)
    res_z["jacobian_entries"] = int(pz.size * Zz.size)
    res_z["nodes"] = int(pz.size * wl.TWO_NQ * wl.TWO_NX)
    ex["two_point_dI_dZ_one_rhs"] = res_z
    # the same for one right-hand side of the three-point workload (1024 points x 256 entries)
    P3, A3, m3z, Z3z = wl.three_point()
    te3, tm3z, tZ3z = _dev(torch, np.concatenate([P3, A3])), _dev(torch, m3z), _dev(torch, Z3z)
    o3z = torch.empty(P3.size, dtype=torch.float64, device="cuda")
    j3z = torch.empty(P3.size * Z3z.size, dtype=torch.float64, device="cuda")
    d3z = frg.make_desc(3, wl.THREE_NQ, wl.THREE_QMAX, n_x=wl.THREE_NX, n_phi=wl.THREE_NPHI)
    res_z3 = {}
    for name, dz in (("value_only", None), ("value_and_dI_dZ", j3z)):
        fz = lambda: ctx.integrate(d3z, o3z, ext=te3, m2=tm3z, Z=tZ3z, x_min=wl.Z_XMIN,
                                   x_max=wl.Z_XMAX, dz=dz)
        warm_clocks(torch, fz, EXTRA_WARM_S)
        wall, ev = time_kernel(torch, fz, 20, 2)
        res_z3[name + "_us"] = round(float(np.mean(ev)) * 1e3, 1)
    res_z3["jacobian_entries"] = int(P3.size * Z3z.size)
    res_z3["nodes"] = int(P3.size * wl.THREE_NQ * wl.THREE_NX * wl.THREE_NPHI)
    ex["three_point_dI_dZ_one_rhs"] = res_z3
    # precision form on the near-pole workload vs float64 on identical inputs
    log("bench: float32 precision form")

    def fp32_vs_fp64(seed_m2, tau, regulator=0):
        res = {}
        for prec in (0, 1):
            descs, batches, out, err, nodes, keep = two_point_batch_setup(
                torch, frg, precision=prec, seed_m2=seed_m2, tau=tau, regulator=regulator)
            fp = lambda: ctx.integrate_multi(descs, batches)
            warm_clocks(torch, fp, EXTRA_WARM_S)
            wall, ev = time_kernel(torch, fp, 100, 5)
            res[prec] = (float(np.mean(ev)), out.clone(),
                         None if err is None else err.clone(), nodes)
        ms64, o64, _, nodes = res[0]
        ms32, o32, e32, _ = res[1]
        rel = ((o32 - o64).abs() / o64.abs()).cpu().numpy()
        within = bool(((o32 - o64).abs() / o64.abs() <= e32).all().item())
        gn = nodes / (ms32 * 1e-3) / 1e9
        return {"speedup_vs_fp64": round(ms64 / ms32, 3),
                "gnodes_per_s": round(gn, 2),
                # nominal work per node against the packed float32 peak (the form issues no
                # packed instructions, so half of it is its own ceiling)
                "frac_fp32_peak": round(FLOP_PER_NODE[2] * gn / 1e3 / FP32_PEAK_TFLOPS, 4),
                "max_rel_err_vs_fp64": float(rel.max()),
                "median_rel_err_vs_fp64": float(np.median(rel)),
                "max_stated_bound": float(e32.max().item()), "all_within_bound": within,
                "near_pole_tau": tau}

    # near-pole workload (m2 in U[-0.95, -0.5]) at the default threshold, then swept
    ex["fp32_form_near_pole"] = fp32_vs_fp64(4, 0.1)
    ex["fp32_form_near_pole_tau_sweep"] = {str(t): fp32_vs_fp64(4, t) for t in (0.0, 0.25)}
    # the two-point workload itself (m2 = 0.5): no propagator falls back to float64
    ex["fp32_form_two_point"] = fp32_vs_fp64(None, 0.1)
    # the polynomial-exponential s_8 regulator (the paper's default) in both forms
    ex["fp32_form_two_point_s8"] = fp32_vs_fp64(None, 0.1, regulator=1)
    # right-hand-side latency: one LPA, two-point and three-point RHS per call, the plan's kernels
    # launched directly (default) and replayed as a captured HIP graph (FRG_FLOW_GRAPH=1)
    log("bench: RHS latency")
    lat = {}
    rho = wl.lpa_rho_grid()
    trho = _dev(torch, rho)
    st = _dev(torch, -0.3 + rho)
    du = torch.empty_like(st)
    dl = frg.make_desc(1, wl.LPA_NQ, wl.LPA_QMAX)
    p, m2, Z = wl.two_point()
    tp, tZ = _dev(torch, p), _dev(torch, Z)
    s2 = torch.full((p.size,), m2, dtype=torch.float64, device="cuda")
    d2 = torch.empty_like(s2)
    dd = frg.make_desc(2, wl.TWO_NQ, wl.TWO_QMAX, n_x=wl.TWO_NX)
    P, A, m3, Z3 = wl.three_point()
    tg3, tZ3 = _dev(torch, np.concatenate([P, A])), _dev(torch, Z3)
    s3 = _dev(torch, m3)
    d3o = torch.empty_like(s3)
    d3 = frg.make_desc(3, wl.THREE_NQ, wl.THREE_QMAX, n_x=wl.THREE_NX, n_phi=wl.THREE_NPHI)
    os.environ["FRG_FLOW_GRAPH"] = "1"
    gctx = frg.Context(0)
    del os.environ["FRG_FLOW_GRAPH"]
    for mode, c in (("", ctx), ("_graph", gctx)):
        lat["lpa_rhs" + mode] = _latency(torch, lambda: c.flow_rhs(dl, st, trho, du, n_comp=4,
                                                                   m2_floor=-0.9), n=10000)
        lat["two_point_rhs" + mode] = _latency(torch, lambda: c.flow_rhs(dd, s2, tp, d2, Z=tZ,
                                                                         m2_floor=-0.9, coef=1.0),
                                               n=10000)
        lat["three_point_rhs" + mode] = _latency(
            torch, lambda: c.flow_rhs(d3, s3, tg3, d3o, Z=tZ3, m2_floor=-0.9, coef=1.0), n=2000)
    torch.cuda.synchronize()
    gctx.close()
    ex["rhs_latency_us"] = lat
    log("bench: flow stepper")
    ex["flow_stepper"] = stepper_bench(torch, frg, wl, ctx)
    log("bench: serving")
    ex["serving"] = serving(torch, frg, wl, ctx, seconds=serving_seconds, warm=serving_warm)
    return ex


def serving(torch, frg, wl, ctx, n_steppers=200, seconds=15.0, warm=2.0,
            loads=(0.5, 0.8, 0.95), seed=12345, max_inflight=6, plain=True, poll_us=2):
    """Workload 5: right-hand-side requests of 200 synthetic RK4 time-steppers, served by a
    session and, for comparison, by the plain per-batch float64 path, with one client harness.

    Each stepper (workloads.stepper_spec) owns a request shape (family, n_ext, nodes per
    dimension, float64 or float32), a dressing table (resident in the session; on the device for
    the plain path) and four RK4 stage inputs.  The C++ replay harness (frg_serving_replay)
    takes an open-loop arrival trace: Poisson arrivals, each the next stage request of a
    uniformly drawn stepper, at a rate set for an offered load of `load` times the session's
    measured saturation capacity.  The same trace is replayed (a) through the session (submit at
    the arrival time; completions stamped by waiter threads blocked on the tickets) and (b)
    through the plain path: first in, first out on one stream, each request's inputs copied to
    the device, one frg_integrate_batch in float64, the result copied back.  The first `warm`
    seconds of arrivals are excluded; `seconds` are measured.  Every session result is compared
    bit for bit with the same request computed alone through frg_integrate_batch (float32
    requests with the float32 form), every plain-path float64 result as well.
    """
    import ctypes

    specs = [wl.stepper_spec(i) for i in range(n_steppers)]
    fam_name = {1: "lpa", 2: "two_point", 3: "three_point"}

    def stage_inputs(sp, stage):
        u = sp.state0 * (1.0 + 0.01 * stage)
        if sp.family == 1:
            g = np.gradient(u, sp.ext)
            m2 = np.maximum(u + 2.0 * sp.ext * g, -0.9)
            ext = None
        else:
            m2 = np.clip(u, 0.05, 4.0)
            ext = np.ascontiguousarray(sp.ext)
        return ext, np.ascontiguousarray(m2)

    def desc_of(sp):
        prec = 1 if sp.fp32 else 0
        return frg.make_desc(sp.family, sp.n_q, sp.q_max, n_x=sp.n_x, n_phi=sp.n_phi,
                             precision=prec, near_pole_tau=0.1 if prec else 0.0)

    cfg = frg.frg_session_config(max_inflight, 4 << 30, poll_us, 0)  # 4 GiB arena
    sess = frg.frg_session_open(ctx.handle, cfg)
    keep = []
    kinds, kind_spec, kind_nodes = [], [], []
    for sp in specs:
        tid, zdev = -1, None
        if sp.Z is not None:
            tid = frg.frg_session_register_table(sess, sp.Z.ctypes.data, sp.Z.size, wl.Z_XMIN,
                                                 wl.Z_XMAX)
            zdev = _dev(torch, sp.Z)
            keep.append(zdev)
        d = desc_of(sp)
        tz = zdev
        for stage in range(4):
            ext, m2 = stage_inputs(sp, stage)
            # the request alone, as the session must reproduce it
            out = torch.empty(sp.n_ext, dtype=torch.float64, device="cuda")
            err = torch.empty(sp.n_ext, dtype=torch.float64, device="cuda") if sp.fp32 else None
            ctx.integrate(d, out, ext=None if ext is None else _dev(torch, ext),
                          m2=_dev(torch, m2), Z=tz, x_min=wl.Z_XMIN, x_max=wl.Z_XMAX,
                          err_out=err)
            expect = np.ascontiguousarray(out.cpu().numpy())
            keep += [ext, m2, expect]
            kinds.append(frg.frg_replay_kind(
                d, sp.n_ext, None if ext is None else ext.ctypes.data, m2.ctypes.data, tid,
                None if zdev is None else zdev.data_ptr(), 0 if sp.Z is None else sp.Z.size,
                wl.Z_XMIN, wl.Z_XMAX, expect.ctypes.data))
            kind_spec.append(sp)
            kind_nodes.append(wl.request_nodes(sp))
    torch.cuda.synchronize()
    kind_nodes = np.array(kind_nodes, dtype=np.float64)
    kfam = np.array([sp.family for sp in kind_spec])
    k32 = np.array([sp.fp32 for sp in kind_spec])
    rng = np.random.default_rng(seed)

    def draw_kinds(n):
        st = rng.integers(0, n_steppers, n)
        counter = np.zeros(n_steppers, dtype=np.int64)
        out = np.empty(n, dtype=np.int64)
        for i, j in enumerate(st):
            out[i] = 4 * j + counter[j] % 4
            counter[j] += 1
        return out

    def pct(x, q):
        return round(float(np.percentile(x, q)), 1) if len(x) else None

    def summary(lat, status, mism, idx, sel, wall):
        ok = sel & (status == 0)
        nodes = kind_nodes[idx]
        res = {"requests": int(sel.sum()), "failed": int((sel & (status != 0)).sum()),
               "mismatches": int((sel & (mism != 0)).sum()),
               "p50_us": pct(lat[ok], 50), "p99_us": pct(lat[ok], 99),
               "gnodes_per_s_served": round(float(nodes[ok].sum()) / (wall * 1e-6) / 1e9, 2)
               if wall > 0 else None}
        classes = {}
        for f in (1, 2, 3):
            for p32 in (False, True):
                m = ok & (kfam[idx] == f) & (k32[idx] == p32)
                if m.any():
                    classes[f"{fam_name[f]}_{'fp32' if p32 else 'fp64'}"] = {
                        "requests": int(m.sum()), "mean_nodes": round(float(nodes[m].mean())),
                        "p50_us": pct(lat[m], 50), "p99_us": pct(lat[m], 99)}
        res["per_class"] = classes
        return res

    res = {"steppers": n_steppers, "max_inflight": max_inflight, "poll_us": poll_us,
           "warm_seconds": warm,
           "seconds_per_load": seconds, "kinds": len(kinds),
           "mean_request_nodes": round(float(kind_nodes.mean()))}
    # saturation capacity: a burst of requests all arriving at once, through both paths
    n_burst = 1500
    bidx = draw_kinds(n_burst)
    btimes = np.zeros(n_burst)
    cap = {}
    paths = (("session", 0), ("plain_fp64_per_batch", 1)) if plain else (("session", 0),)
    for name, mode in paths:
        log(f"bench: serving capacity, {name}")
        lat, status, mism, wall = frg.frg_serving_replay(
            ctx.handle, sess if mode == 0 else None, mode, kinds, btimes, bidx, n_waiters=64)
        cap[name] = {"gnodes_per_s": round(float(kind_nodes[bidx].sum()) / (wall * 1e-6) / 1e9,
                                           2),
                     "requests": n_burst, "wall_ms": round(wall / 1e3, 1),
                     "failed": int((status != 0).sum()), "mismatches": int((mism != 0).sum())}
    res["capacity"] = cap
    c_nodes = cap["session"]["gnodes_per_s"] * 1e9
    for load in (loads if seconds > 0 else ()):
        rate = load * c_nodes / float(kind_nodes.mean())  # requests per second
        n = int(rate * (warm + seconds) * 1.02) + 1
        gaps = rng.exponential(1.0 / rate, n)
        times = np.cumsum(gaps) * 1e6
        times = times[times < (warm + seconds) * 1e6]
        idx = draw_kinds(times.size)
        sel = times >= warm * 1e6
        entry = {"offered_load": load, "arrival_rate_per_s": round(rate, 1),
                 "offered_gnodes_per_s": round(load * c_nodes / 1e9, 2)}
        for name, mode in paths:
            log(f"bench: serving at offered load {load}, {name}")
            s0 = frg.frg_session_stats(sess)
            lat, status, mism, wall = frg.frg_serving_replay(
                ctx.handle, sess if mode == 0 else None, mode, kinds, times, idx, n_waiters=64)
            # served rate over the measured arrivals: their nodes over first measured arrival
            # to last completion
            t_first = float(times[sel].min()) if sel.any() else 0.0
            span = float((times[sel] + np.where(status[sel] == 0, lat[sel], 0.0)).max()
                         - t_first) if sel.any() else 0.0
            entry[name] = summary(lat, status, mism, idx, sel, span)
            if mode == 0:
                s1 = frg.frg_session_stats(sess)
                entry[name]["launches"] = int(s1.launches - s0.launches)
                dc = max(int(s1.completed - s0.completed), 1)
                entry[name]["mean_phase_us"] = {
                    ph: round((getattr(s1, f"mean_{ph}_us") * s1.completed
                               - getattr(s0, f"mean_{ph}_us") * s0.completed) / dc, 1)
                    for ph in ("queue", "launch", "device", "finish")}
        res[f"load_{load}"] = entry
    st = frg.frg_session_stats(sess)
    res["session_stats"] = {"p50_us": round(st.p50_us, 1), "p99_us": round(st.p99_us, 1),
                            "completed": int(st.completed), "failed": int(st.failed),
                            "launches": int(st.launches), "tickets_held": int(st.tickets_held)}
    frg.frg_session_close(sess)
    del keep
    return res


def _latency(torch, fn, n=2000):
    for _ in range(20):
        fn()
    torch.cuda.synchronize()
    ts = np.empty(n)
    for i in range(n):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts[i] = time.perf_counter() - t0
    return {"p50": round(float(np.percentile(ts, 50)) * 1e6, 2),
            "p99": round(float(np.percentile(ts, 99)) * 1e6, 2), "calls": n}


if __name__ == "__main__":
    main()
