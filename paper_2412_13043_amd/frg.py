"""Thin ctypes binding of the C ABI in include/frg.h (argument marshalling only).

Every computation runs in libfrg.so's HIP kernels.  torch is used for device memory (tensors
whose data_ptr() are handed to the library) and for streams.  There is no CPU fallback: if the
built library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int, c_size_t, c_uint64, c_void_p

# torch ships its own HIP and HSA runtimes (same sonames as the system ROCm ones).  Importing it
# before libfrg.so makes the loader bind libfrg's libamdhip64.so.7 dependency to the copy torch
# already loaded, so the process has one HIP runtime; loading libfrg.so first would bring in a
# second runtime, and whichever initialises second finds no device.
import torch  # noqa: F401  (load order matters, see above)

_HERE = os.path.dirname(os.path.abspath(__file__))
# FRG_LIBRARY selects another build of the same library (for example one compiled with different
# tuning macros); the default is the in-tree build.
LIB_PATH = os.environ.get("FRG_LIBRARY") or os.path.join(_HERE, "libfrg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it first (python -m paper_2412_13043_amd.build, or "
        "__graft_entry__.build()); there is no fallback path")

_lib = ctypes.CDLL(LIB_PATH)

# ---- enums (frg.h) --------------------------------------------------------------------------
FRG_OK, FRG_E_INVAL, FRG_E_NOMEM, FRG_E_DEVICE, FRG_E_NOTREADY, FRG_E_TIMEOUT, \
    FRG_E_CANCELLED, FRG_E_UNSUPPORTED = range(8)
FRG_FP64, FRG_FP32_KAHAN = 0, 1
FRG_FAMILY_LPA, FRG_FAMILY_TWO_POINT, FRG_FAMILY_THREE_POINT = 1, 2, 3
FRG_FAMILY_LPA_T, FRG_FAMILY_TWO_POINT_T, FRG_FAMILY_THREE_POINT_T = 4, 5, 6
FRG_BOSONIC, FRG_FERMIONIC = 0, 1
FRG_REG_EXPONENTIAL, FRG_REG_POLY_EXP, FRG_REG_FLAT = 0, 1, 2
FRG_MAX_NODES = 1024
FRG_MAX_FT_NODES = 65536
FRG_MAX_TABLE = 4096

STATUS_NAMES = {0: "FRG_OK", 1: "FRG_E_INVAL", 2: "FRG_E_NOMEM", 3: "FRG_E_DEVICE",
                4: "FRG_E_NOTREADY", 5: "FRG_E_TIMEOUT", 6: "FRG_E_CANCELLED",
                7: "FRG_E_UNSUPPORTED"}


class FrgError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


# ---- structs (frg.h) ------------------------------------------------------------------------
class frg_integral_desc(ctypes.Structure):
    _fields_ = [("family", c_int), ("d", c_int), ("n_q", c_int), ("n_x", c_int),
                ("n_phi", c_int), ("precision", c_int), ("q_max", c_double), ("k", c_double),
                ("near_pole_tau", c_double), ("T", c_double), ("freq_max", c_double),
                ("statistics", c_int), ("n_tail", c_int), ("freq_scaled", c_int),
                ("regulator", c_int), ("reg_order", c_int), ("complex_freq", c_int)]


class frg_log_table(ctypes.Structure):
    _fields_ = [("values", c_void_p), ("n", c_int), ("x_min", c_double), ("x_max", c_double)]


class frg_batch(ctypes.Structure):
    _fields_ = [("n_ext", c_int), ("ext", c_void_p), ("m2", c_void_p), ("m2_scalar", c_double),
                ("Z", frg_log_table), ("out", c_void_p), ("err_out", c_void_p),
                ("dout_dm2", c_void_p), ("dout_dz", c_void_p)]


class frg_flow_state(ctypes.Structure):
    _fields_ = [("family", c_int), ("n_ext", c_int), ("state", c_void_p), ("grid", c_void_p),
                ("Z", frg_log_table), ("n_comp", c_int), ("m2_floor", c_double),
                ("coef", c_double)]


class frg_session_config(ctypes.Structure):
    _fields_ = [("max_inflight", c_int), ("hbm_budget_bytes", c_size_t), ("poll_us", c_int),
                ("watchdog_ms", c_int)]


class frg_stats(ctypes.Structure):
    _fields_ = [("p50_us", c_double), ("p99_us", c_double), ("gnodes_per_s", c_double),
                ("admitted", c_uint64), ("queued", c_uint64), ("rejected", c_uint64),
                ("completed", c_uint64), ("failed", c_uint64), ("cancelled", c_uint64),
                ("nodes", c_uint64), ("launches", c_uint64), ("tickets_held", c_uint64),
                ("mean_queue_us", c_double), ("mean_launch_us", c_double),
                ("mean_device_us", c_double), ("mean_finish_us", c_double)]


class frg_stepper_config(ctypes.Structure):
    _fields_ = [("rtol", c_double), ("atol", c_double), ("h0", c_double), ("h_min", c_double),
                ("h_max", c_double), ("max_steps", c_int), ("fixed_step", c_int), ("method", c_int)]


class frg_stepper_stats(ctypes.Structure):
    _fields_ = [("t", c_double), ("h", c_double), ("last_err", c_double),
                ("accepted", c_uint64), ("rejected", c_uint64), ("rhs_evals", c_uint64)]


_P = c_void_p
_sig = {
    "frg_context_create": ([c_int, c_size_t, POINTER(c_void_p)], c_int),
    "frg_context_destroy": ([_P], c_int),
    "frg_last_error": ([], c_char_p),
    "frg_integrate_batch": ([_P, POINTER(frg_integral_desc), POINTER(frg_batch), _P], c_int),
    "frg_integrate_batch_noalloc": ([_P, POINTER(frg_integral_desc), POINTER(frg_batch), _P],
                                    c_int),
    "frg_integrate_multi": ([_P, c_int, POINTER(frg_integral_desc), POINTER(frg_batch), _P],
                            c_int),
    "frg_flow_rhs": ([_P, POINTER(frg_integral_desc), POINTER(frg_flow_state), _P, _P], c_int),
    "frg_autotune": ([_P, POINTER(frg_integral_desc), POINTER(frg_batch), _P, c_int,
                      POINTER(c_double)], c_int),
    "frg_session_open": ([_P, POINTER(frg_session_config), POINTER(c_void_p)], c_int),
    "frg_session_register_table": ([_P, _P, c_int, c_double, c_double, POINTER(c_int)], c_int),
    "frg_session_submit": ([_P, POINTER(frg_integral_desc), POINTER(frg_batch), c_int,
                            POINTER(c_uint64)], c_int),
    "frg_session_poll": ([_P, c_uint64, POINTER(c_int)], c_int),
    "frg_session_wait": ([_P, c_uint64, c_int], c_int),
    "frg_session_cancel": ([_P, c_uint64], c_int),
    "frg_session_stats": ([_P, POINTER(frg_stats)], c_int),
    "frg_session_close": ([_P], c_int),
    "frg_stepper_create": ([_P, POINTER(frg_integral_desc), POINTER(frg_flow_state),
                            POINTER(frg_stepper_config), POINTER(c_void_p)], c_int),
    "frg_stepper_advance": ([_P, c_double, _P, POINTER(frg_stepper_stats)], c_int),
    "frg_stepper_destroy": ([_P], c_int),
    "frg_litim_threshold": ([c_int, c_int, _P, _P, c_int, _P], c_int),
}
EXPORTED = tuple(_sig)
for _name, (_args, _res) in _sig.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res
# test double of the serving loop (include/frg_testing.h)
_lib.frg_session_open_fake.argtypes = [POINTER(frg_session_config), c_double, c_double,
                                       POINTER(c_void_p)]
_lib.frg_session_open_fake.restype = c_int
class frg_replay_kind(ctypes.Structure):
    _fields_ = [("desc", frg_integral_desc), ("n_ext", c_int), ("ext", c_void_p),
                ("m2", c_void_p), ("table_id", c_int), ("Z_dev", c_void_p), ("nZ", c_int),
                ("x_min", c_double), ("x_max", c_double), ("expect", c_void_p)]


class frg_replay_arrival(ctypes.Structure):
    _fields_ = [("t_us", c_double), ("kind", c_int)]


class frg_replay_result(ctypes.Structure):
    _fields_ = [("latency_us", c_double), ("status", c_int), ("mismatch", c_int)]


_lib.frg_serving_replay.argtypes = [c_void_p, c_void_p, c_int, c_int, POINTER(frg_replay_kind),
                                    c_int, POINTER(frg_replay_arrival), c_int,
                                    POINTER(frg_replay_result), POINTER(c_double)]
_lib.frg_serving_replay.restype = c_int
_lib.frg_flop_probe.argtypes = [c_int, c_int, c_int, c_void_p, c_void_p]
_lib.frg_flop_probe.restype = c_int
_lib.frg_math_probe.argtypes = [c_int, POINTER(c_double), c_void_p]
_lib.frg_math_probe.restype = c_int
_lib.frg_fp32_error_constants.argtypes = [POINTER(c_double)]
_lib.frg_fp32_error_constants.restype = None
_lib.frg_session_fake_fail_launches.argtypes = [c_void_p, c_int]
_lib.frg_session_fake_fail_launches.restype = c_int
TESTING_EXPORTED = ("frg_session_open_fake", "frg_session_fake_fail_launches",
                    "frg_serving_replay", "frg_flop_probe", "frg_math_probe",
                    "frg_fp32_error_constants")


def frg_last_error() -> str:
    m = _lib.frg_last_error()
    return m.decode() if m else ""


def _check(status: int, where: str, ok=(FRG_OK,)) -> int:
    if status not in ok:
        raise FrgError(status, where, frg_last_error())
    return status


# ---- direct wrappers with the ABI's names -----------------------------------------------------
def frg_context_create(device: int = 0, hbm_budget_bytes: int = 0) -> int:
    h = c_void_p()
    _check(_lib.frg_context_create(device, hbm_budget_bytes, byref(h)), "frg_context_create")
    return h.value


def frg_context_destroy(ctx: int) -> None:
    _check(_lib.frg_context_destroy(ctx), "frg_context_destroy")


def frg_litim_threshold(d: int, n: int, w: int, out: int, count: int, stream: int) -> None:
    _check(_lib.frg_litim_threshold(d, n, w, out, count, stream), "frg_litim_threshold")


def litim_threshold(d: int, n: int, w, out, stream=None):
    """out[i] = l_n^d(w[i]) (float64 device tensors of equal size); returns out."""
    if w.numel() != out.numel():
        raise ValueError("w and out must have the same number of values")
    frg_litim_threshold(d, n, _dptr(w), _dptr(out), int(w.numel()), _stream(stream))
    return out


def frg_integrate_batch(ctx: int, desc: frg_integral_desc, batch: frg_batch, stream: int) -> None:
    _check(_lib.frg_integrate_batch(ctx, byref(desc), byref(batch), stream), "frg_integrate_batch")


def frg_integrate_batch_noalloc(ctx: int, desc: frg_integral_desc, batch: frg_batch,
                                stream: int) -> None:
    _check(_lib.frg_integrate_batch_noalloc(ctx, byref(desc), byref(batch), stream),
           "frg_integrate_batch_noalloc")


def frg_integrate_multi(ctx: int, descs, batches, stream: int) -> None:
    n = len(descs)
    D = (frg_integral_desc * n)(*descs)
    B = (frg_batch * n)(*batches)
    _check(_lib.frg_integrate_multi(ctx, n, D, B, stream), "frg_integrate_multi")


def frg_autotune(ctx: int, desc: frg_integral_desc, batch: frg_batch, stream: int,
                 reps: int = 3) -> float:
    best = c_double()
    _check(_lib.frg_autotune(ctx, byref(desc), byref(batch), stream, reps, byref(best)),
           "frg_autotune")
    return best.value


def frg_flow_rhs(ctx: int, desc: frg_integral_desc, state: frg_flow_state, dstate_dt: int,
                 stream: int) -> None:
    _check(_lib.frg_flow_rhs(ctx, byref(desc), byref(state), dstate_dt, stream), "frg_flow_rhs")


def frg_stepper_create(ctx: int, desc: frg_integral_desc, state: frg_flow_state,
                       cfg: frg_stepper_config) -> int:
    h = c_void_p()
    _check(_lib.frg_stepper_create(ctx, byref(desc), byref(state), byref(cfg), byref(h)),
           "frg_stepper_create")
    return h.value


def frg_stepper_advance(st: int, t_end: float, stream: int, ok=(FRG_OK,)):
    """Returns (status, stats); statuses outside `ok` raise."""
    stats = frg_stepper_stats()
    rc = _check(_lib.frg_stepper_advance(st, t_end, stream, byref(stats)), "frg_stepper_advance",
                ok)
    return rc, stats


def frg_stepper_destroy(st: int) -> None:
    _check(_lib.frg_stepper_destroy(st), "frg_stepper_destroy")


def frg_session_open(ctx: int, cfg: frg_session_config) -> int:
    h = c_void_p()
    _check(_lib.frg_session_open(ctx, byref(cfg), byref(h)), "frg_session_open")
    return h.value


def frg_session_open_fake(cfg: frg_session_config, ns_per_node: float, base_us: float) -> int:
    h = c_void_p()
    _check(_lib.frg_session_open_fake(byref(cfg), ns_per_node, base_us, byref(h)),
           "frg_session_open_fake")
    return h.value


def frg_serving_replay(ctx, session, mode: int, kinds, times_us, kind_idx, n_waiters: int = 64):
    """Open-loop replay (include/frg_testing.h): kinds is a list of frg_replay_kind, times_us
    and kind_idx the arrivals (ascending times).  Returns (latency_us, status, mismatch) numpy
    arrays and the wall time in microseconds."""
    import numpy as np

    n = len(times_us)
    K = (frg_replay_kind * len(kinds))(*kinds)
    A = (frg_replay_arrival * max(n, 1))()
    for i in range(n):
        A[i].t_us = float(times_us[i])
        A[i].kind = int(kind_idx[i])
    R = (frg_replay_result * max(n, 1))()
    wall = c_double()
    _check(_lib.frg_serving_replay(ctx, session, mode, len(kinds), K, n, A, n_waiters, R,
                                   byref(wall)), "frg_serving_replay")
    lat = np.array([R[i].latency_us for i in range(n)])
    status = np.array([R[i].status for i in range(n)], dtype=np.int32)
    mism = np.array([R[i].mismatch for i in range(n)], dtype=np.int32)
    return lat, status, mism, wall.value


def frg_flop_probe(seq: int, blocks: int, iters: int, out, stream=None) -> None:
    """One dispatch of the FLOP-count probe kernel for sequence `seq` (include/frg_testing.h);
    out: float64 device tensor of blocks * 64 values."""
    if out.numel() < blocks * 64:
        raise ValueError("out needs blocks * 64 values")
    _check(_lib.frg_flop_probe(seq, blocks, iters, _dptr(out), _stream(stream)), "frg_flop_probe")


def frg_math_probe(which: int, stream=None) -> float:
    """Largest error of one float32 elementary operation over its whole input range
    (include/frg_testing.h): 0 log2 (absolute, on [1/2, 1)), 1 expm1(-y), 2 reciprocal,
    3 2^x."""
    v = c_double()
    _check(_lib.frg_math_probe(which, byref(v), _stream(stream)), "frg_math_probe")
    return v.value


def frg_fp32_error_constants() -> tuple:
    """(u, log2 error, expm1 error, reciprocal error, 2^x error) the float32 form's bound
    uses."""
    a = (c_double * 5)()
    _lib.frg_fp32_error_constants(a)
    return tuple(a)


def frg_session_fake_fail_launches(s: int, n: int) -> None:
    _check(_lib.frg_session_fake_fail_launches(s, n), "frg_session_fake_fail_launches")


def frg_session_register_table(s: int, Z_host_ptr: int, n: int, x_min: float,
                               x_max: float) -> int:
    tid = c_int()
    _check(_lib.frg_session_register_table(s, Z_host_ptr, n, x_min, x_max, byref(tid)),
           "frg_session_register_table")
    return tid.value


def frg_session_submit(s: int, desc: frg_integral_desc, batch: frg_batch, table_id: int) -> int:
    t = c_uint64()
    _check(_lib.frg_session_submit(s, byref(desc), byref(batch), table_id, byref(t)),
           "frg_session_submit")
    return t.value


def frg_session_poll(s: int, ticket: int) -> bool:
    done = c_int()
    _check(_lib.frg_session_poll(s, ticket, byref(done)), "frg_session_poll")
    return bool(done.value)


def frg_session_wait(s: int, ticket: int, timeout_ms: int = -1) -> int:
    return _check(_lib.frg_session_wait(s, ticket, timeout_ms), "frg_session_wait",
                  ok=(FRG_OK, FRG_E_TIMEOUT))


def frg_session_cancel(s: int, ticket: int) -> int:
    return _check(_lib.frg_session_cancel(s, ticket), "frg_session_cancel",
                  ok=(FRG_OK, FRG_E_NOTREADY))


def frg_session_stats(s: int) -> frg_stats:
    st = frg_stats()
    _check(_lib.frg_session_stats(s, byref(st)), "frg_session_stats")
    return st


def frg_session_close(s: int) -> None:
    _check(_lib.frg_session_close(s), "frg_session_close")


def raw_status(name: str, *args) -> int:
    """Call an ABI function and return its status without raising (for error-path tests)."""
    return getattr(_lib, name)(*args)


# ---- torch-tensor conveniences (marshalling only) ---------------------------------------------
def _dptr(t) -> int | None:
    if t is None:
        return None
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.dtype != torch.float64 or not t.is_contiguous() or t.device.type != "cuda":
        raise ValueError("expected a contiguous float64 tensor on a HIP (cuda) device")
    return t.data_ptr()


def _stream(stream) -> int:
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def make_desc(family: int, n_q: int, q_max: float, *, n_x: int = 0, n_phi: int = 0, d: int = 0,
              k: float = 1.0, precision: int = FRG_FP64, near_pole_tau: float = 0.0,
              T: float = 0.0, freq_max: float = 0.0, statistics: int = FRG_BOSONIC,
              n_tail: int = 0, freq_scaled: bool = False, regulator: int = FRG_REG_EXPONENTIAL,
              reg_order: int = 0, complex_freq: bool = False):
    """Descriptor; T, freq_max, statistics, n_tail and freq_scaled apply to the finite-temperature
    families (4, 5, 6) only, complex_freq to families 5 and 6; regulator and reg_order to every
    family."""
    if d == 0:
        d = 3 if family == FRG_FAMILY_LPA else 4
    return frg_integral_desc(family, d, n_q, n_x, n_phi, precision, q_max, k, near_pole_tau,
                             T, freq_max, statistics, n_tail, 1 if freq_scaled else 0, regulator,
                             reg_order, 1 if complex_freq else 0)


def make_batch(n_ext: int, out, *, ext=None, m2=None, m2_scalar: float = 0.0, Z=None,
               x_min: float = 1e-3, x_max: float = 1e3, err_out=None, dout=None,
               dz=None) -> frg_batch:
    """dout: optional device tensor receiving dI/dm2 per point (float64 descriptors).
    dz: optional contiguous float64 device tensor of n_ext * len(Z) values receiving dI_e/dZ_i
    row-major (vertex families, frg_integrate_batch only)."""
    if dz is not None:
        nz = 0 if Z is None else int(Z.numel())
        if (dz.numel() != n_ext * nz or not dz.is_contiguous() or not dz.is_cuda or
                str(dz.dtype) != "torch.float64"):
            raise ValueError(f"dz must be a contiguous float64 device tensor of n_ext * len(Z) = "
                             f"{n_ext * nz} values")
    zt = frg_log_table(_dptr(Z), 0 if Z is None else int(Z.numel()), x_min, x_max)
    return frg_batch(n_ext, _dptr(ext), _dptr(m2), m2_scalar, zt, _dptr(out), _dptr(err_out),
                     _dptr(dout), _dptr(dz))


def _n_points(desc, out) -> int:
    """External points of a call whose results go to `out`: with complex external frequencies
    out holds the real parts followed by the imaginary parts (2 values per point)."""
    n = int(out.numel())
    if desc.complex_freq:
        if n % 2:
            raise ValueError("with complex frequencies out holds 2 values per point (Re, Im)")
        return n // 2
    return n


class Context:
    """Owns one frg_context on a HIP device."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.device = device
        self.handle = frg_context_create(device, hbm_budget_bytes)

    def close(self):
        if self.handle:
            frg_context_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):  # pragma: no cover - best effort
        try:
            self.close()
        except Exception:
            pass

    def integrate(self, desc, out, *, ext=None, m2=None, m2_scalar=0.0, Z=None, x_min=1e-3,
                  x_max=1e3, err_out=None, dout=None, dz=None, stream=None):
        n_ext = _n_points(desc, out)
        b = make_batch(n_ext, out, ext=ext, m2=m2, m2_scalar=m2_scalar, Z=Z,
                       x_min=x_min, x_max=x_max, err_out=err_out, dout=dout, dz=dz)
        frg_integrate_batch(self.handle, desc, b, _stream(stream))
        return out

    def integrate_noalloc(self, desc, out, *, ext=None, m2=None, m2_scalar=0.0, Z=None,
                          x_min=1e-3, x_max=1e3, err_out=None, dout=None, dz=None, stream=None):
        """frg_integrate_batch_noalloc: as integrate, scratch in the library's static array."""
        n_ext = _n_points(desc, out)
        b = make_batch(n_ext, out, ext=ext, m2=m2, m2_scalar=m2_scalar, Z=Z,
                       x_min=x_min, x_max=x_max, err_out=err_out, dout=dout, dz=dz)
        frg_integrate_batch_noalloc(self.handle, desc, b, _stream(stream))
        return out

    def autotune(self, desc, out, *, ext=None, m2=None, m2_scalar=0.0, Z=None, x_min=1e-3,
                 x_max=1e3, reps=3, stream=None):
        b = make_batch(_n_points(desc, out), out, ext=ext, m2=m2, m2_scalar=m2_scalar, Z=Z,
                       x_min=x_min, x_max=x_max)
        return frg_autotune(self.handle, desc, b, _stream(stream), reps)

    def integrate_multi(self, descs, batches, stream=None):
        frg_integrate_multi(self.handle, list(descs), list(batches), _stream(stream))

    def flow_rhs(self, desc, state, grid, dstate_dt, *, Z=None, x_min=1e-3, x_max=1e3,
                 n_comp=4, m2_floor=-0.9, coef=1.0, stream=None):
        zt = frg_log_table(_dptr(Z), 0 if Z is None else int(Z.numel()), x_min, x_max)
        st = frg_flow_state(desc.family, int(dstate_dt.numel()), _dptr(state), _dptr(grid), zt,
                            n_comp, m2_floor, coef)
        frg_flow_rhs(self.handle, desc, st, _dptr(dstate_dt), _stream(stream))
        return dstate_dt

    def stepper(self, desc, state, grid, *, Z=None, x_min=1e-3, x_max=1e3, n_comp=4,
                m2_floor=-0.9, coef=1.0, rtol=1e-8, atol=1e-10, h0=1e-2, h_min=1e-10,
                h_max=1.0, max_steps=100000, fixed_step=False, method=0):
        """A flow stepper evolving `state` (device tensor) in place: method 0 the adaptive
        Dormand-Prince 5(4) (or fixed steps), method 1 the fixed-step Adams-Bashforth-Moulton 4
        PECE, method 2 the adaptive Runge-Kutta-Fehlberg 7(8) (or fixed steps), method 3 the
        variable-step Adams-Bashforth-Moulton 4 PECE.  state, grid and Z must stay alive while
        the stepper is used."""
        return Stepper(self, desc, state, grid, Z=Z, x_min=x_min, x_max=x_max, n_comp=n_comp,
                       m2_floor=m2_floor, coef=coef, rtol=rtol, atol=atol, h0=h0, h_min=h_min,
                       h_max=h_max, max_steps=max_steps, fixed_step=fixed_step, method=method)


class Stepper:
    """frg_stepper: integrates the flow of frg_flow_rhs in RG time t = log(Lambda/k)."""

    def __init__(self, ctx, desc, state, grid, *, Z, x_min, x_max, n_comp, m2_floor, coef, rtol,
                 atol, h0, h_min, h_max, max_steps, fixed_step, method=0):
        zt = frg_log_table(_dptr(Z), 0 if Z is None else int(Z.numel()), x_min, x_max)
        fs = frg_flow_state(desc.family, int(state.numel()), _dptr(state), _dptr(grid), zt,
                            n_comp, m2_floor, coef)
        cfg = frg_stepper_config(rtol, atol, h0, h_min, h_max, max_steps, 1 if fixed_step else 0,
                                 method)
        self._keep = (state, grid, Z)
        self.handle = frg_stepper_create(ctx.handle, desc, fs, cfg)

    def advance(self, t_end, stream=None, ok=(FRG_OK,)):
        """Advance to t_end; returns (status, frg_stepper_stats)."""
        return frg_stepper_advance(self.handle, t_end, _stream(stream), ok)

    def close(self):
        if self.handle:
            frg_stepper_destroy(self.handle)
            self.handle = None

    def __del__(self):  # pragma: no cover - best effort
        try:
            self.close()
        except Exception:
            pass


class Session:
    """A serving session (frg_session_*) with host buffers: submit() queues one request and
    returns a ticket; its results are in the given numpy arrays once wait() returns FRG_OK.
    The arrays of a request must stay alive until its ticket has ended.  `fake=(ns_per_node,
    base_us)` opens the scheduling test double instead (no context, no device work)."""

    def __init__(self, ctx=None, *, max_inflight=4, hbm_budget_bytes=0, poll_us=0,
                 watchdog_ms=0, fake=None):
        cfg = frg_session_config(max_inflight, hbm_budget_bytes, poll_us, watchdog_ms)
        if fake is not None:
            self.handle = frg_session_open_fake(cfg, float(fake[0]), float(fake[1]))
        else:
            self.handle = frg_session_open(ctx.handle, cfg)
        self._keep = {}

    def register_table(self, Z, x_min, x_max) -> int:
        """Copies a dressing table (float64 numpy array) to the device for the session's
        lifetime; returns its id for submit(table_id=...)."""
        import numpy as np

        z = np.ascontiguousarray(Z, dtype=np.float64)
        return frg_session_register_table(self.handle, z.ctypes.data, int(z.size), x_min, x_max)

    def submit(self, desc, out, *, ext=None, m2=None, m2_scalar=0.0, Z=None, x_min=1e-3,
               x_max=1e3, table_id=-1, err_out=None, dout=None, dz=None) -> int:
        """Queues one request on host arrays (contiguous float64 numpy arrays; out holds the
        results, 2 values per point with complex frequencies)."""
        arrs = [a for a in (ext, m2, Z, out, err_out, dout, dz) if a is not None]
        for a in arrs:
            if str(a.dtype) != "float64" or not a.flags["C_CONTIGUOUS"]:
                raise ValueError("session buffers must be contiguous float64 numpy arrays")
        n = int(out.size) // (2 if desc.complex_freq else 1)
        ptr = lambda a: None if a is None else a.ctypes.data
        zt = frg_log_table(ptr(Z), 0 if Z is None else int(Z.size), x_min, x_max)
        b = frg_batch(n, ptr(ext), ptr(m2), m2_scalar, zt, ptr(out), ptr(err_out), ptr(dout),
                      ptr(dz))
        t = frg_session_submit(self.handle, desc, b, table_id)
        self._keep[t] = arrs
        return t

    def wait(self, ticket, timeout_ms=-1) -> int:
        st = frg_session_wait(self.handle, ticket, timeout_ms)
        if st == FRG_OK:
            self._keep.pop(ticket, None)
        return st

    def poll(self, ticket) -> bool:
        done = frg_session_poll(self.handle, ticket)
        if done:
            self._keep.pop(ticket, None)
        return done

    def stats(self):
        return frg_session_stats(self.handle)

    def close(self):
        if self.handle:
            frg_session_close(self.handle)
            self.handle = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
