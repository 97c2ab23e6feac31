"""FP64 CPU oracle for the batched fRG loop integrals -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import this package.  The product library (``paper_2412_13043_amd``) never imports, links or
calls it, and the two share no code: the oracle is plain C (``frg_oracle.c``: long-double
Newton Gauss-Legendre, libm transcendentals, Neumaier sums), wrapped here with ctypes.

What each function computes, and the passage of arXiv 2412.13043 it follows, is documented
in ``frg_oracle.h``.  Every function here is pinned by ``tests/test_oracle_*.py`` to closed
forms, library routines, high-precision (mpmath) evaluations, brute-force Cartesian sums and
invariances; none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "frg_oracle.c")
_LIB = os.path.join(_HERE, "libfrg_oracle.so")

REG_EXP = 0
REG_LITIM = 1
REG_POLYEXP = 100  # + N: the polynomial-exponential regulator of order N


def reg_polyexp(n: int = 8) -> int:
    return REG_POLYEXP + n
LPA = 1
TWO_POINT = 2
THREE_POINT = 3
LPA_T = 4
TWO_POINT_T = 5
THREE_POINT_T = 6
BOSONIC = 0
FERMIONIC = 1

_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math) into oracle/libfrg_oracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build()
            lib = ctypes.CDLL(_LIB)
            D, I, P = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
            lib.frgo_gauss_legendre.argtypes = [I, D, D, P, P]
            lib.frgo_regulator.argtypes = [I, D, D]
            lib.frgo_regulator.restype = D
            lib.frgo_regulator_dot.argtypes = [I, D, D]
            lib.frgo_regulator_dot.restype = D
            lib.frgo_dressing.argtypes = [P, I, D, D, D]
            lib.frgo_dressing.restype = D
            lib.frgo_propagator.argtypes = [I, P, I, D, D, D, D, D]
            lib.frgo_propagator.restype = D
            lib.frgo_integrate.argtypes = [I, I, I, I, I, D, D, I, P, P, D, P, I, D, D, I, P]
            lib.frgo_vertex_hyperspherical.argtypes = [I, I, I, I, I, D, D, I, P, P, D, P, I, D, D, P]
            lib.frgo_lpa_flow_rhs.argtypes = [I, I, D, D, I, I, D, P, P, I, P]
            lib.frgo_fd_derivatives.argtypes = [P, P, I, P, P]
            lib.frgo_matsubara_rule.argtypes = [I, D, D, I, I, P, P]
            lib.frgo_integrate_ft.argtypes = [I, I, I, D, D, I, I, D, D, I, I, P, P, D, P, I, D, D,
                                              I, P]
            lib.frgo_integrate_dm2.argtypes = lib.frgo_integrate.argtypes
            lib.frgo_integrate_ft_dm2.argtypes = lib.frgo_integrate_ft.argtypes
            lib.frgo_integrate_dz.argtypes = [I, I, I, D, D, I, P, P, D, P, I, D, D, I, P]
            lib.frgo_litim_threshold.argtypes = [I, I, D]
            lib.frgo_litim_threshold.restype = D
            lib.frgo_integrate_dz_three.argtypes = [I, I, I, D, D, I, P, P, D, P, I, D, D, I, P]
            lib.frgo_integrate_ft_dz.argtypes = [I, I, D, D, I, I, D, D, I, I, P, P, D, P, I, D,
                                                 D, I, P]
            lib.frgo_integrate_ft_three.argtypes = [I, I, I, D, D, I, I, D, D, I, I, P, P, D, P,
                                                    I, D, D, I, I, P]
            lib.frgo_vertex_ft_spherical.argtypes = [I, I, I, D, D, I, I, D, D, I, I, P, P, D, D,
                                                     D, P, I, D, D, P]
            lib.frgo_integrate_ft_three_dz.argtypes = [I, I, I, D, D, I, I, D, D, I, I, P, P, D,
                                                       P, I, D, D, I, P]
            lib.frgo_integrate_ft_complex.argtypes = [I, I, I, I, D, D, I, I, D, D, I, I, P, P,
                                                      D, P, I, D, D, I, P]
            _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def gauss_legendre(n: int, a: float, b: float):
    lib = _load()
    x = np.empty(n)
    w = np.empty(n)
    if lib.frgo_gauss_legendre(n, a, b, _ptr(x), _ptr(w)) != 0:
        raise ValueError("invalid Gauss-Legendre request")
    return x, w


def regulator(l2: float, k: float = 1.0, kind: int = REG_EXP) -> float:
    return _load().frgo_regulator(kind, l2, k)


def regulator_dot(l2: float, k: float = 1.0, kind: int = REG_EXP) -> float:
    return _load().frgo_regulator_dot(kind, l2, k)


def dressing(Z, x_min: float, x_max: float, l2: float) -> float:
    Z = _f64(Z)
    return _load().frgo_dressing(_ptr(Z), 0 if Z is None else len(Z), x_min, x_max, l2)


def propagator(l2, m2, k=1.0, Z=None, x_min=1e-3, x_max=1e3, kind=REG_EXP) -> float:
    Z = _f64(Z)
    return _load().frgo_propagator(kind, _ptr(Z), 0 if Z is None else len(Z), x_min, x_max, l2, m2, k)


def integrate(family, n_q, q_max, *, d=None, n_x=0, n_phi=0, k=1.0, regulator=REG_EXP, ext=None,
              m2=None, m2_scalar=0.0, Z=None, x_min=1e-3, x_max=1e3, n_ext=None, dm2=False):
    """Loop integrals I_e (see frg_oracle.h).  ext: None | p[n] | (p[n], alpha[n])."""
    if d is None:
        d = 3 if family == LPA else 4
    if family == THREE_POINT and ext is not None:
        p, alpha = ext
        ext_arr = np.concatenate([_f64(p), _f64(alpha)])
        n = len(p)
    elif ext is not None:
        ext_arr = _f64(ext)
        n = len(ext_arr)
    else:
        ext_arr = None
        n = None
    m2a = _f64(m2)
    if n is None:
        n = len(m2a) if m2a is not None else int(n_ext)
    Za = _f64(Z)
    out = np.empty(n)
    fn = _load().frgo_integrate_dm2 if dm2 else _load().frgo_integrate
    rc = fn(family, d, n_q, n_x, n_phi, q_max, k, regulator, _ptr(ext_arr), _ptr(m2a), m2_scalar,
            _ptr(Za), 0 if Za is None else len(Za), x_min, x_max, n, _ptr(out))
    if rc != 0:
        raise ValueError(f"frgo_integrate rejected the arguments (rc={rc})")
    return out


def integrate_dz(n_q, q_max, *, n_x, ext, Z, k=1.0, regulator=REG_EXP, m2=None, m2_scalar=0.0,
                 x_min=1e-3, x_max=1e3):
    """dI_e/dZ_i of the two-point integral (see frg_oracle.h): array [n_ext, len(Z)]."""
    ext_arr, Za, m2a = _f64(ext), _f64(Z), _f64(m2)
    n = len(ext_arr)
    out = np.empty((n, len(Za)))
    rc = _load().frgo_integrate_dz(4, n_q, n_x, q_max, k, regulator, _ptr(ext_arr), _ptr(m2a),
                                   m2_scalar, _ptr(Za), len(Za), x_min, x_max, n, _ptr(out))
    if rc != 0:
        raise ValueError(f"frgo_integrate_dz rejected the arguments (rc={rc})")
    return out


def litim_threshold(d: int, n: int, w) -> np.ndarray:
    """l_n^d(w) of the flat regulator, elementwise over w (see frg_oracle.h)."""
    lib = _load()
    return np.array([lib.frgo_litim_threshold(d, n, float(x)) for x in np.atleast_1d(w)])


def integrate_dz_three(n_q, q_max, *, n_x, n_phi, ext, Z, k=1.0, regulator=REG_EXP, m2=None,
                       m2_scalar=0.0, x_min=1e-3, x_max=1e3):
    """dI_e/dZ_i of the three-point integral: array [n_ext, len(Z)]; ext = (p[n], alpha[n])."""
    p, alpha = ext
    ext_arr = np.concatenate([_f64(p), _f64(alpha)])
    Za, m2a = _f64(Z), _f64(m2)
    n = len(p)
    out = np.empty((n, len(Za)))
    rc = _load().frgo_integrate_dz_three(n_q, n_x, n_phi, q_max, k, regulator, _ptr(ext_arr),
                                         _ptr(m2a), m2_scalar, _ptr(Za), len(Za), x_min, x_max,
                                         n, _ptr(out))
    if rc != 0:
        raise ValueError(f"frgo_integrate_dz_three rejected the arguments (rc={rc})")
    return out


def integrate_ft_dz(n_q, q_max, *, n_x, ext, Z, T, freq_max, statistics=BOSONIC, n_tail=0,
                    freq_scaled=False, k=1.0, regulator=REG_EXP, m2=None, m2_scalar=0.0,
                    x_min=1e-3, x_max=1e3):
    """dI_e/dZ_i of the finite-temperature two-point integral: array [n_ext, len(Z)];
    ext = (p[n], p0[n])."""
    p, p0 = ext
    ext_arr = np.concatenate([_f64(p), _f64(p0)])
    Za, m2a = _f64(Z), _f64(m2)
    n = len(p)
    out = np.empty((n, len(Za)))
    rc = _load().frgo_integrate_ft_dz(n_q, n_x, q_max, k, regulator, statistics, T, freq_max,
                                      1 if freq_scaled else 0, n_tail, _ptr(ext_arr), _ptr(m2a),
                                      m2_scalar, _ptr(Za), len(Za), x_min, x_max, n, _ptr(out))
    if rc != 0:
        raise ValueError(f"frgo_integrate_ft_dz rejected the arguments (rc={rc})")
    return out


def integrate_ft_three_dz(n_q, q_max, *, n_x, n_phi, T, statistics=BOSONIC, freq_max,
                          freq_scaled=False, n_tail=0, k=1.0, regulator=REG_EXP, ext, m2=None,
                          m2_scalar=0.0, Z, x_min=1e-3, x_max=1e3):
    """dI_e/dZ_i of the finite-temperature three-point integral: array [n_ext, len(Z)];
    ext = (p, alpha, p01, p02)."""
    ext_arr = np.concatenate([_f64(e) for e in ext])
    n = len(ext[0])
    Za, m2a = _f64(Z), _f64(m2)
    out = np.empty((n, len(Za)))
    rc = _load().frgo_integrate_ft_three_dz(n_q, n_x, n_phi, q_max, k, regulator, statistics, T,
                                            freq_max, 1 if freq_scaled else 0, n_tail,
                                            _ptr(ext_arr), _ptr(m2a), m2_scalar, _ptr(Za),
                                            len(Za), x_min, x_max, n, _ptr(out))
    if rc != 0:
        raise ValueError(f"frgo_integrate_ft_three_dz rejected the arguments (rc={rc})")
    return out


def integrate_ft_complex(family, n_q, q_max, *, T, statistics=BOSONIC, freq_max,
                         freq_scaled=False, n_tail=0, n_x, n_phi=0, k=1.0, regulator=REG_EXP,
                         ext, m2=None, m2_scalar=0.0, Z=None, x_min=1e-3, x_max=1e3):
    """Finite-temperature two- and three-point integrals with complex external frequencies of
    the inner legs; returns complex I_e.  ext: family TWO_POINT_T (p, p0r, p0i); THREE_POINT_T
    (p, alpha, p01r, p02r, p01i, p02i), each an array of n_ext values."""
    ext_arr = np.concatenate([_f64(e) for e in ext])
    n = len(ext[0])
    m2a, Za = _f64(m2), _f64(Z)
    out = np.empty(2 * n)
    rc = _load().frgo_integrate_ft_complex(
        family, n_q, n_x, n_phi, q_max, k, regulator, statistics, T, freq_max,
        1 if freq_scaled else 0, n_tail, _ptr(ext_arr), _ptr(m2a), m2_scalar, _ptr(Za),
        0 if Za is None else len(Za), x_min, x_max, n, _ptr(out))
    if rc != 0:
        raise ValueError(f"frgo_integrate_ft_complex rejected the arguments (rc={rc})")
    return out[:n] + 1j * out[n:]


def vertex_hyperspherical(n_legs, n_q, n_t1, n_t2, n_t3, q_max, p1, p2, m2, *, k=1.0,
                          regulator=REG_EXP, Z=None, x_min=1e-3, x_max=1e3) -> float:
    p1a = _f64(p1)
    p2a = _f64(p2)
    Za = _f64(Z)
    out = np.empty(1)
    rc = _load().frgo_vertex_hyperspherical(n_legs, n_q, n_t1, n_t2, n_t3, q_max, k, regulator,
                                            _ptr(p1a), _ptr(p2a), m2, _ptr(Za),
                                            0 if Za is None else len(Za), x_min, x_max, _ptr(out))
    if rc != 0:
        raise ValueError("frgo_vertex_hyperspherical rejected the arguments")
    return float(out[0])


def fd_derivatives(x, f):
    xa, fa = _f64(x), _f64(f)
    d1 = np.empty(len(xa))
    d2 = np.empty(len(xa))
    if _load().frgo_fd_derivatives(_ptr(xa), _ptr(fa), len(xa), _ptr(d1), _ptr(d2)) != 0:
        raise ValueError("fd_derivatives needs n >= 3")
    return d1, d2


def lpa_flow_rhs(rho, u, n_q, q_max, *, d=3, k=1.0, regulator=REG_EXP, n_comp=4, m2_floor=-0.9):
    rho_a, u_a = _f64(rho), _f64(u)
    out = np.empty(len(rho_a))
    rc = _load().frgo_lpa_flow_rhs(d, n_q, q_max, k, regulator, n_comp, m2_floor, _ptr(rho_a),
                                   _ptr(u_a), len(rho_a), _ptr(out))
    if rc != 0:
        raise ValueError("frgo_lpa_flow_rhs rejected the arguments")
    return out


def matsubara_rule(statistics, T, lam, n_tail=0, cap=1 << 16):
    """Frequency nodes w_j and weights c_j replacing T sum_n f(w_n) (see frg_oracle.h)."""
    w = np.empty(cap)
    c = np.empty(cap)
    n = _load().frgo_matsubara_rule(statistics, T, lam, n_tail, cap, _ptr(w), _ptr(c))
    if n < 0:
        raise ValueError(f"frgo_matsubara_rule rejected the arguments (rc={n})")
    return w[:n].copy(), c[:n].copy()


def integrate_ft(family, n_q, q_max, *, T, statistics=BOSONIC, freq_max, freq_scaled=False,
                 n_tail=0, n_x=0, n_phi=0, k=1.0, regulator=REG_EXP, ext=None, m2=None,
                 m2_scalar=0.0, Z=None, x_min=1e-3, x_max=1e3, n_ext=None, dm2=False):
    """Finite-temperature integrals I_e, families LPA_T, TWO_POINT_T and THREE_POINT_T.
    ext: family TWO_POINT_T (p[n], p0[n]); THREE_POINT_T (p[n], alpha[n], p01[n], p02[n])."""
    if family == THREE_POINT_T:
        ext_arr = np.concatenate([_f64(e) for e in ext])
        n = len(ext[0])
        m2a = _f64(m2)
        Za = _f64(Z)
        out = np.empty(n)
        rc = _load().frgo_integrate_ft_three(
            n_q, n_x, n_phi, q_max, k, regulator, statistics, T, freq_max,
            1 if freq_scaled else 0, n_tail, _ptr(ext_arr), _ptr(m2a), m2_scalar, _ptr(Za),
            0 if Za is None else len(Za), x_min, x_max, n, 1 if dm2 else 0, _ptr(out))
        if rc != 0:
            raise ValueError(f"frgo_integrate_ft_three rejected the arguments (rc={rc})")
        return out
    if family == TWO_POINT_T:
        p, p0 = ext
        ext_arr = np.concatenate([_f64(p), _f64(p0)])
        n = len(p)
    else:
        ext_arr = None
        n = None
    m2a = _f64(m2)
    if n is None:
        n = len(m2a) if m2a is not None else int(n_ext)
    Za = _f64(Z)
    out = np.empty(n)
    fn = _load().frgo_integrate_ft_dm2 if dm2 else _load().frgo_integrate_ft
    rc = fn(family, n_q, n_x, q_max, k, regulator, statistics, T, freq_max,
            1 if freq_scaled else 0, n_tail, _ptr(ext_arr), _ptr(m2a), m2_scalar, _ptr(Za),
            0 if Za is None else len(Za), x_min, x_max, n, _ptr(out))
    if rc != 0:
        raise ValueError(f"frgo_integrate_ft rejected the arguments (rc={rc})")
    return out


def vertex_ft_spherical(n_q, n_t1, n_t2, q_max, p1, p2, p01, p02, m2, *, T, statistics=BOSONIC,
                        freq_max, freq_scaled=False, n_tail=0, k=1.0, regulator=REG_EXP, Z=None,
                        x_min=1e-3, x_max=1e3) -> float:
    """The finite-temperature three-point integral of one point with explicit spatial 3-vectors
    p1, p2 (frgo_vertex_ft_spherical)."""
    p1a, p2a, Za = _f64(p1), _f64(p2), _f64(Z)
    out = np.empty(1)
    rc = _load().frgo_vertex_ft_spherical(n_q, n_t1, n_t2, q_max, k, regulator, statistics, T,
                                          freq_max, 1 if freq_scaled else 0, n_tail, _ptr(p1a),
                                          _ptr(p2a), p01, p02, m2, _ptr(Za),
                                          0 if Za is None else len(Za), x_min, x_max, _ptr(out))
    if rc != 0:
        raise ValueError("frgo_vertex_ft_spherical rejected the arguments")
    return float(out[0])
