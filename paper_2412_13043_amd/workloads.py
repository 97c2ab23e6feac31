"""Seeded synthetic inputs for the loop-integral workloads.

This module only draws and lays out inputs (grids, masses, dressing tables, request mixes); it
holds none of the method's arithmetic (no regulator, propagator, quadrature or reduction).  Both
the GPU path's tests/benchmark and the FP64 oracle's tests take their inputs from here.

The workloads mirror the paper's setting (arXiv 2412.13043): logarithmic external-momentum
grids (Sec. 3.3, Yang-Mills momentum grids), dressing functions tabulated on logarithmic
coordinates (App. F, FunctionTex1D) and tensor-product quadrature rules of a few dozen nodes per
dimension (Sec. 3.3 performance table, Sec. 5.3).  Every array is float64 and host (numpy).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Dressing-table grid: 256 points, log-uniform in |l| over [1e-3 k, 1e3 k].
Z_POINTS = 256
Z_XMIN = 1e-3
Z_XMAX = 1e3


def dressing_table(seed: int, n: int = Z_POINTS) -> np.ndarray:
    """Smooth random dressing values in [0.8, 1.5] on an n-point grid.

    S_j = sum_{m=1..6} (a_m/m) sin(pi m s_j + phi_m), s_j = j/(n-1), a_m ~ U(-1,1),
    phi_m ~ U(0, 2pi); then Z_j = 0.8 + 0.7 (S_j - min S)/(max S - min S).
    """
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, 6)
    ph = rng.uniform(0.0, 2.0 * math.pi, 6)
    s = np.arange(n, dtype=np.float64) / (n - 1)
    S = np.zeros(n)
    for m in range(1, 7):
        S += (a[m - 1] / m) * np.sin(math.pi * m * s + ph[m - 1])
    return 0.8 + 0.7 * (S - S.min()) / (S.max() - S.min())


# ------------------------------------------------------------------------------------------
# Workload 1: LPA O(4) model, d = 3, 64 rho points, GL32 on [0, 6k]
# ------------------------------------------------------------------------------------------
LPA_N_RHO = 64
LPA_NQ = 32
LPA_QMAX = 6.0
LPA_M2_FLOOR = -0.9


def lpa_rho_grid(n: int = LPA_N_RHO) -> np.ndarray:
    """rho_i = i/(n-1), i = 0..n-1 (rho in [0, 1])."""
    return np.arange(n, dtype=np.float64) / (n - 1)


def lpa_potential(a: float = 0.3, b: float = 1.0, n: int = LPA_N_RHO):
    """U(rho) = -a rho + b rho^2/2 on the rho grid: returns rho, u = U', m2 = U' + 2 rho U''.

    m2 is floored at -0.9 as the workload prescribes.  With a = 0.3, b = 1 this is the single
    right-hand side U = -0.3 rho + 0.5 rho^2.
    """
    rho = lpa_rho_grid(n)
    u = -a + b * rho
    m2 = np.maximum(u + 2.0 * rho * b, LPA_M2_FLOOR)
    return rho, u, m2


def lpa_batch(B: int = 4096, seed: int = 11, n: int = LPA_N_RHO):
    """B potentials U = -a rho + b rho^2/2 with a ~ U[0.1, 0.5], b ~ U[0.5, 1.5]."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.1, 0.5, B)
    b = rng.uniform(0.5, 1.5, B)
    rho = lpa_rho_grid(n)
    u = -a[:, None] + b[:, None] * rho[None, :]
    m2 = np.maximum(u + 2.0 * rho[None, :] * b[:, None], LPA_M2_FLOOR)
    return rho, u, m2


# ------------------------------------------------------------------------------------------
# Workload 2: two-point vertex flow, d = 4, 256 log-spaced momenta, GL64 [0,10k] x GL32
# ------------------------------------------------------------------------------------------
TWO_N_EXT = 256
TWO_NQ = 64
TWO_NX = 32
TWO_QMAX = 10.0
TWO_M2 = 0.5


def momenta_log(n: int = TWO_N_EXT, lo: float = -3.0, hi: float = 2.0) -> np.ndarray:
    """p_j = 10^(lo + (hi-lo) j/(n-1)), endpoints included."""
    return 10.0 ** (lo + (hi - lo) * np.arange(n, dtype=np.float64) / (n - 1))


def two_point(seed_z: int = 1):
    """One right-hand side: p (256,), scalar m2 = 0.5, Z table (seed 1)."""
    return momenta_log(), TWO_M2, dressing_table(seed_z)


def two_point_batch(B: int = 256, seed_base: int = 1000):
    """B right-hand sides sharing p and m2 = 0.5, each with its own Z table (seeds 1000+b)."""
    Z = np.stack([dressing_table(seed_base + b) for b in range(B)])
    return momenta_log(), TWO_M2, Z


# ------------------------------------------------------------------------------------------
# Workload 3: three-point vertex flow, d = 4, 64 |p| x 16 angles, GL 64 x 32 x 16
# ------------------------------------------------------------------------------------------
THREE_NP = 64
THREE_NA = 16
THREE_NQ = 64
THREE_NX = 32
THREE_NPHI = 16
THREE_QMAX = 10.0


def three_point_ext(n_p: int = THREE_NP, n_a: int = THREE_NA):
    """|p1| = |p2| = 10^(-3 + 5a/(n_p-1)), alpha_b = pi b/(n_a-1); flat index e = n_a*a + b."""
    p = momenta_log(n_p)
    alpha = math.pi * np.arange(n_a, dtype=np.float64) / (n_a - 1)
    P = np.repeat(p, n_a)
    A = np.tile(alpha, n_p)
    return P, A


def three_point(seed_m2: int = 3, seed_z: int = 1):
    """One right-hand side: (p, alpha) (1024 each), m2 ~ U[0.1, 2] (seed 3), Z (seed 1)."""
    P, A = three_point_ext()
    m2 = np.random.default_rng(seed_m2).uniform(0.1, 2.0, P.shape[0])
    return P, A, m2, dressing_table(seed_z)


def three_point_batch(B: int = 8, seed_m2_base: int = 300, seed_z_base: int = 1000):
    P, A = three_point_ext()
    m2 = np.stack([np.random.default_rng(seed_m2_base + b).uniform(0.1, 2.0, P.shape[0])
                   for b in range(B)])
    Z = np.stack([dressing_table(seed_z_base + b) for b in range(B)])
    return P, A, m2, Z


# ------------------------------------------------------------------------------------------
# Workload 4: precision form of workload 2, masses near the pole m2 ~ U[-0.95, -0.5]
# ------------------------------------------------------------------------------------------
def near_pole(seed_m2: int = 4, seed_z: int = 1):
    p = momenta_log()
    m2 = np.random.default_rng(seed_m2).uniform(-0.95, -0.5, p.shape[0])
    return p, m2, dressing_table(seed_z)


def near_pole_batch(B: int = 256, seed_m2_base: int = 400, seed_z_base: int = 1000):
    p = momenta_log()
    m2 = np.stack([np.random.default_rng(seed_m2_base + b).uniform(-0.95, -0.5, p.shape[0])
                   for b in range(B)])
    Z = np.stack([dressing_table(seed_z_base + b) for b in range(B)])
    return p, m2, Z


# ------------------------------------------------------------------------------------------
# Finite temperature (d = 3 + 1, Matsubara sum): the two-point workload's shapes at T = 0.1 k,
# bosonic frequencies |w| <= 10 k ("q0": fixed domain, the radial range's scale) plus 8 tail
# nodes per side, GL64 on [0, 10k] x GL32 in cos1; external frequency 0 (bosonic lowest) for
# half the points and 2 pi T for the other half; per-RHS Z tables; the LPA on the rho grid.
# ------------------------------------------------------------------------------------------
FT_T = 0.1
FT_FREQ_MAX = 10.0
FT_N_TAIL = 8
FT_NQ = 64
FT_NX = 32
FT_QMAX = 10.0


def two_point_ft_batch(B: int = 16, seed_base: int = 1000):
    """B right-hand sides: p (256 log-spaced) and p0 (0 for even, 2 pi T for odd points),
    m2 = 0.5, Z tables (seeds 1000+b)."""
    p = momenta_log()
    p0 = np.where(np.arange(p.size) % 2 == 1, 2.0 * math.pi * FT_T, 0.0)
    Z = np.stack([dressing_table(seed_base + b) for b in range(B)])
    return p, p0, TWO_M2, Z


def three_point_ft_batch(B: int = 2, seed_m2_base: int = 500, seed_z_base: int = 1000):
    """The three-point workload's external pairs at the finite-temperature settings: (p, alpha)
    as three_point_ext (1024 pairs), leg frequencies p01 = 2 pi T for odd e and 0 otherwise, p02 =
    -2 pi T for e = 2, 3 mod 4 and 0 otherwise (l1 = q + p1 and l2 = q - p2 with bosonic
    external frequencies 0 or 2 pi T: every combination), m2 ~ U[0.1, 2] and Z per right-hand
    side (seeds 500+b, 1000+b)."""
    P, A = three_point_ext()
    e = np.arange(P.size)
    p01 = np.where(e % 2 == 1, 2.0 * math.pi * FT_T, 0.0)
    p02 = np.where((e // 2) % 2 == 1, -2.0 * math.pi * FT_T, 0.0)
    m2 = np.stack([np.random.default_rng(seed_m2_base + b).uniform(0.1, 2.0, P.size)
                   for b in range(B)])
    Z = np.stack([dressing_table(seed_z_base + b) for b in range(B)])
    return P, A, p01, p02, m2, Z


# ------------------------------------------------------------------------------------------
# Workload 5: serving mix of many concurrent time-steppers
# ------------------------------------------------------------------------------------------
@dataclasses.dataclass
class StepperSpec:
    index: int
    family: int          # 1 LPA, 2 two-point, 3 three-point
    n_ext: int
    n_q: int
    n_x: int
    n_phi: int
    fp32: bool
    q_max: float
    ext: np.ndarray | None       # family 2: p; family 3: concat(p, alpha); family 1: rho grid
    state0: np.ndarray           # family 1: u = U'(rho); families 2/3: m2 per point
    Z: np.ndarray | None


def _log_uniform_int(rng, lo: int, hi: int) -> int:
    return int(min(hi, max(lo, round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))))


def stepper_spec(i: int, *, n_ext_range=(16, 4096), n_range=(16, 128)) -> StepperSpec:
    """Stepper i (seed 5+i): family ~ U{1,2,3}; n_ext and per-dimension node counts log-uniform
    integers; FP64 or FP32 with probability 1/2; its own dressing table and initial state."""
    rng = np.random.default_rng(5 + i)
    family = int(rng.integers(1, 4))
    n_ext = _log_uniform_int(rng, *n_ext_range)
    n_q = _log_uniform_int(rng, *n_range)
    n_x = _log_uniform_int(rng, *n_range)
    n_phi = _log_uniform_int(rng, *n_range)
    fp32 = bool(rng.integers(0, 2))
    zseed = 100000 + i
    if family == 1:
        n_ext = max(n_ext, 3)
        rho = np.arange(n_ext, dtype=np.float64) / (n_ext - 1)
        a = rng.uniform(0.1, 0.5)
        b = rng.uniform(0.5, 1.5)
        return StepperSpec(i, 1, n_ext, n_q, 0, 0, fp32, LPA_QMAX, rho, -a + b * rho, None)
    if family == 2:
        p = momenta_log(n_ext)
        m2 = rng.uniform(0.1, 2.0, n_ext)
        return StepperSpec(i, 2, n_ext, n_q, n_x, 0, fp32, TWO_QMAX, p, m2, dressing_table(zseed))
    n_p = max(1, int(round(math.sqrt(n_ext))))
    n_a = max(1, n_ext // n_p)
    n_ext = n_p * n_a
    p = momenta_log(n_p)
    alpha = math.pi * np.arange(n_a, dtype=np.float64) / max(1, n_a - 1)
    ext = np.concatenate([np.repeat(p, n_a), np.tile(alpha, n_p)])
    m2 = rng.uniform(0.1, 2.0, n_ext)
    return StepperSpec(i, 3, n_ext, n_q, n_x, n_phi, fp32, THREE_QMAX, ext, m2, dressing_table(zseed))


def request_nodes(spec: StepperSpec) -> int:
    """Integrand evaluations (nodes) one right-hand side of this stepper costs."""
    if spec.family == 1:
        return spec.n_ext * spec.n_q
    if spec.family == 2:
        return spec.n_ext * spec.n_q * spec.n_x
    return spec.n_ext * spec.n_q * spec.n_x * spec.n_phi
