"""Adaptive explicit Runge-Kutta stepper of the oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may use
this module; the product library never does.  Plain numpy, one stage at a time.

What it computes: the flow dstate/dt = f(t, state) in RG time t = log(Lambda/k) (paper Sec. 2.1)
advanced by the embedded Runge-Kutta pair of Dormand and Prince, order 5(4), with the last stage
reused as the next step's first ("first same as last") -- the RK45 class of explicit steppers the
paper lists for vertex expansions (Sec. 5.2, "Time-stepping").  The tableau is the published one
(J. R. Dormand, P. J. Prince, J. Comput. Appl. Math. 6 (1980) 19, RK5(4)7M); error norm and
step-size rule are the standard ones of Hairer, Norsett & Wanner, Solving ODEs I, Sec. II.4:

    sc_i = atol + rtol max(|y_i|, |ynew_i|),  err = sqrt(mean_i ((ynew_i - yhat_i)/sc_i)^2),
    accept if err <= 1,  h_next = h min(facmax, max(0.2, 0.9 err^(-1/5))),
    facmax = 5, or 1 right after a rejected step; h_next clipped to [h_min, h_max].

A step that would pass t_end ends exactly there.  fixed_step: steps of exactly h0, no control.

Abm4 (below) is the fixed-step Adams-Bashforth-Moulton 4 PECE stepper with an RK4 start.

Abm4Var (below) is the same PECE pair with a variable step: Milne's estimate of the corrector's
local error, (19/270)(y_c - y_p) (the AB4 and AM4 error constants 251/720 and -19/720), in the
norm above; on a change of step the history is moved onto the new spacing by the cubic through
its four points.

Rkf78 (below) is the Runge-Kutta-Fehlberg 7(8) pair (the RK78 class the paper lists next to
RK45, Sec. 5.2): E. Fehlberg, "Classical fifth-, sixth-, seventh-, and eighth-order Runge-Kutta
formulas with stepsize control", NASA TR R-287 (1968), the 13-stage 7(8) formulas.  The
eighth-order solution is kept (local extrapolation); the error estimate is the difference of
the two solutions, 41/840 h (k_1 + k_11 - k_12 - k_13); the norm and the step rule are those
above with the exponent -1/8 (the lower order plus one).
"""
from __future__ import annotations

import math
from fractions import Fraction as F

import numpy as np

# Dormand-Prince RK5(4)7M, exact fractions
C = [F(0), F(1, 5), F(3, 10), F(4, 5), F(8, 9), F(1), F(1)]
A = [
    [],
    [F(1, 5)],
    [F(3, 40), F(9, 40)],
    [F(44, 45), F(-56, 15), F(32, 9)],
    [F(19372, 6561), F(-25360, 2187), F(64448, 6561), F(-212, 729)],
    [F(9017, 3168), F(-355, 33), F(46732, 5247), F(49, 176), F(-5103, 18656)],
    [F(35, 384), F(0), F(500, 1113), F(125, 192), F(-2187, 6784), F(11, 84)],
]
B = A[6] + [F(0)]  # fifth order
BHAT = [F(5179, 57600), F(0), F(7571, 16695), F(393, 640), F(-92097, 339200), F(187, 2100),
        F(1, 40)]  # fourth order (embedded)


class Dopri5:
    """State: t, y, the next step size h, the first stage of the next step (if known)."""

    def __init__(self, f, y0, *, rtol, atol, h0, h_min, h_max, max_steps, fixed_step=False,
                 t0=0.0):
        self.f = f
        self.y = np.array(y0, dtype=np.float64)
        self.t = float(t0)
        self.rtol, self.atol = rtol, atol
        self.h0, self.h_min, self.h_max = h0, h_min, h_max
        self.h = min(max(h0, h_min), h_max)
        self.max_steps = max_steps
        self.fixed = fixed_step
        self.k0 = None
        self.rejected_last = False
        self.accepted = 0
        self.rejected = 0
        self.evals = 0
        self.last_err = 0.0

    def _f(self, t, y):
        self.evals += 1
        return np.asarray(self.f(t, y), dtype=np.float64)

    def advance(self, t_end):
        """Advance to t_end; returns "ok", "max_steps" or "h_min"."""
        attempts = 0
        while self.t < t_end:
            if attempts >= self.max_steps:
                return "max_steps"
            attempts += 1
            h = self.h0 if self.fixed else self.h
            last = self.t + h >= t_end * (1.0 - 1e-14) - 1e-300
            if last:
                h = t_end - self.t
            if self.k0 is None:
                self.k0 = self._f(self.t, self.y)
            K = [self.k0]
            for s in range(1, 7):
                incr = sum(float(A[s][j]) * K[j] for j in range(s))
                K.append(self._f(self.t + float(C[s]) * h, self.y + h * incr))
            ynew = self.y + h * sum(float(B[j]) * K[j] for j in range(6))
            if self.fixed:
                err = 0.0
            else:
                est = h * sum(float(B[j] - BHAT[j]) * K[j] for j in range(7))
                sc = self.atol + self.rtol * np.maximum(np.abs(self.y), np.abs(ynew))
                err = math.sqrt(float(np.mean((est / sc) ** 2)))
            self.last_err = err
            if self.fixed or err <= 1.0:
                self.y = ynew
                self.k0 = K[6]
                self.t = t_end if last else self.t + h
                self.accepted += 1
                if self.fixed:
                    continue
                fac = 0.9 * err ** -0.2 if err > 0 else 5.0
                fmax = 1.0 if self.rejected_last else 5.0
                self.h = min(max(h * min(fmax, max(0.2, fac)), self.h_min), self.h_max)
                self.rejected_last = False
            else:
                self.rejected += 1
                self.rejected_last = True
                if h <= self.h_min:
                    return "h_min"
                fac = 0.9 * err ** -0.2
                self.h = min(max(h * min(1.0, max(0.2, fac)), self.h_min), self.h_max)
        return "ok"


# Adams-Bashforth (order 4) predictor and Adams-Moulton (order 4) corrector weights, exact
# fractions: y_{n+1} = y_n + h sum_j b_j f_{n-j} (AB4) and y_n + h (m_p f(pred) + sum_j m_j
# f_{n-j}) (AM4), both from integrating the interpolating cubic of the right-hand side over the
# step.
AB4 = [F(55, 24), F(-59, 24), F(37, 24), F(-9, 24)]
AM4 = [F(9, 24), F(19, 24), F(-5, 24), F(1, 24)]  # f(t_{n+1}, predicted), f_n, f_{n-1}, f_{n-2}
RK4_C = [F(0), F(1, 2), F(1, 2), F(1)]
RK4_B = [F(1, 6), F(1, 3), F(1, 3), F(1, 6)]


class Abm4:
    """Fixed-step Adams-Bashforth-Moulton 4 in PECE mode (the multistep class of explicit
    steppers the paper names for vertex expansions, Sec. 5.2): predict with AB4, evaluate,
    correct with AM4, evaluate.  The first three steps are classical RK4 steps that build the
    history f_n, f_{n-1}, f_{n-2}, f_{n-3}.  A step that would pass t_end ends there: if that
    shortens it (by more than rounding, 1e-9 of h0) it is an RK4 step and the history restarts
    after it.  Steps of h0; no error control."""

    def __init__(self, f, y0, *, h0, max_steps, t0=0.0):
        self.f = f
        self.y = np.array(y0, dtype=np.float64)
        self.t = float(t0)
        self.h0 = h0
        self.max_steps = max_steps
        self.hist = []  # f_n, f_{n-1}, ... (newest first), all at step h0
        self.accepted = 0
        self.evals = 0

    def _f(self, t, y):
        self.evals += 1
        return np.asarray(self.f(t, y), dtype=np.float64)

    def _rk4(self, h):
        k1 = self.hist[0] if self.hist else self._f(self.t, self.y)
        ks = [k1]
        for s in range(1, 4):
            ks.append(self._f(self.t + float(RK4_C[s]) * h, self.y + float(RK4_C[s]) * h * ks[-1]))
        return self.y + h * sum(float(RK4_B[j]) * ks[j] for j in range(4))

    def advance(self, t_end):
        """Advance to t_end; returns "ok" or "max_steps"."""
        attempts = 0
        while self.t < t_end:
            if attempts >= self.max_steps:
                return "max_steps"
            attempts += 1
            h = self.h0
            last = self.t + h >= t_end * (1.0 - 1e-14) - 1e-300
            if last:
                h = t_end - self.t
            if last and h < self.h0 * (1.0 - 1e-9):
                # shortened final step: RK4, and the history (at step h0) is dropped
                self.y = self._rk4(h)
                self.t = t_end
                self.hist = [self._f(self.t, self.y)]
                self.accepted += 1
                continue
            if len(self.hist) < 4:
                if not self.hist:
                    self.hist = [self._f(self.t, self.y)]
                ynew = self._rk4(h)
            else:
                pred = self.y + h * sum(float(AB4[j]) * self.hist[j] for j in range(4))
                fp = self._f(self.t + h, pred)
                ynew = self.y + h * (float(AM4[0]) * fp +
                                     sum(float(AM4[j + 1]) * self.hist[j] for j in range(3)))
            self.t = t_end if last else self.t + h
            self.y = ynew
            self.hist = ([self._f(self.t, self.y)] + self.hist)[:4]
            self.accepted += 1
        return "ok"


# Fehlberg 7(8), exact fractions: nodes, stage coefficients (row i: a_i0 .. a_i,i-1), seventh-
# and eighth-order weights
C78 = [F(0), F(2, 27), F(1, 9), F(1, 6), F(5, 12), F(1, 2), F(5, 6), F(1, 6), F(2, 3), F(1, 3),
       F(1), F(0), F(1)]


def _row(i, entries):
    r = [F(0)] * i
    for j, v in entries.items():
        r[j] = v
    return r


A78 = [
    [],
    _row(1, {0: F(2, 27)}),
    _row(2, {0: F(1, 36), 1: F(1, 12)}),
    _row(3, {0: F(1, 24), 2: F(1, 8)}),
    _row(4, {0: F(5, 12), 2: F(-25, 16), 3: F(25, 16)}),
    _row(5, {0: F(1, 20), 3: F(1, 4), 4: F(1, 5)}),
    _row(6, {0: F(-25, 108), 3: F(125, 108), 4: F(-65, 27), 5: F(125, 54)}),
    _row(7, {0: F(31, 300), 4: F(61, 225), 5: F(-2, 9), 6: F(13, 900)}),
    _row(8, {0: F(2), 3: F(-53, 6), 4: F(704, 45), 5: F(-107, 9), 6: F(67, 90), 7: F(3)}),
    _row(9, {0: F(-91, 108), 3: F(23, 108), 4: F(-976, 135), 5: F(311, 54), 6: F(-19, 60),
             7: F(17, 6), 8: F(-1, 12)}),
    _row(10, {0: F(2383, 4100), 3: F(-341, 164), 4: F(4496, 1025), 5: F(-301, 82),
              6: F(2133, 4100), 7: F(45, 82), 8: F(45, 164), 9: F(18, 41)}),
    _row(11, {0: F(3, 205), 5: F(-6, 41), 6: F(-3, 205), 7: F(-3, 41), 8: F(3, 41),
              9: F(6, 41)}),
    _row(12, {0: F(-1777, 4100), 3: F(-341, 164), 4: F(4496, 1025), 5: F(-289, 82),
              6: F(2193, 4100), 7: F(51, 82), 8: F(33, 164), 9: F(12, 41), 11: F(1)}),
]
B7 = [F(41, 840), F(0), F(0), F(0), F(0), F(34, 105), F(9, 35), F(9, 35), F(9, 280), F(9, 280),
      F(41, 840), F(0), F(0)]
B8 = [F(0), F(0), F(0), F(0), F(0), F(34, 105), F(9, 35), F(9, 35), F(9, 280), F(9, 280), F(0),
      F(41, 840), F(41, 840)]


class Rkf78:
    """Adaptive Runge-Kutta-Fehlberg 7(8): the eighth-order solution with the difference of the
    two as its error estimate, the norm and step rule of Dopri5 with exponent -1/8.  Thirteen
    right-hand sides per attempted step (no stage is shared between steps; a rejected step
    keeps its first).  fixed_step: steps of exactly h0 without control."""

    def __init__(self, f, y0, *, rtol, atol, h0, h_min, h_max, max_steps, fixed_step=False,
                 t0=0.0):
        self.f = f
        self.y = np.array(y0, dtype=np.float64)
        self.t = float(t0)
        self.rtol, self.atol = rtol, atol
        self.h0, self.h_min, self.h_max = h0, h_min, h_max
        self.h = min(max(h0, h_min), h_max)
        self.max_steps = max_steps
        self.fixed = fixed_step
        self.k0 = None
        self.rejected_last = False
        self.accepted = 0
        self.rejected = 0
        self.evals = 0
        self.last_err = 0.0

    def _f(self, t, y):
        self.evals += 1
        return np.asarray(self.f(t, y), dtype=np.float64)

    def advance(self, t_end):
        """Advance to t_end; returns "ok", "max_steps" or "h_min"."""
        attempts = 0
        while self.t < t_end:
            if attempts >= self.max_steps:
                return "max_steps"
            attempts += 1
            h = self.h0 if self.fixed else self.h
            last = self.t + h >= t_end * (1.0 - 1e-14) - 1e-300
            if last:
                h = t_end - self.t
            if self.k0 is None:
                self.k0 = self._f(self.t, self.y)
            K = [self.k0]
            for s in range(1, 13):
                incr = sum(float(A78[s][j]) * K[j] for j in range(s))
                K.append(self._f(self.t + float(C78[s]) * h, self.y + h * incr))
            ynew = self.y + h * sum(float(B8[j]) * K[j] for j in range(13))
            if self.fixed:
                err = 0.0
            else:
                est = h * sum(float(B8[j] - B7[j]) * K[j] for j in range(13))
                sc = self.atol + self.rtol * np.maximum(np.abs(self.y), np.abs(ynew))
                err = math.sqrt(float(np.mean((est / sc) ** 2)))
            self.last_err = err
            if self.fixed or err <= 1.0:
                self.y = ynew
                self.k0 = None
                self.t = t_end if last else self.t + h
                self.accepted += 1
                if self.fixed:
                    continue
                fac = 0.9 * err ** -0.125 if err > 0 else 5.0
                fmax = 1.0 if self.rejected_last else 5.0
                self.h = min(max(h * min(fmax, max(0.2, fac)), self.h_min), self.h_max)
                self.rejected_last = False
            else:
                self.rejected += 1
                self.rejected_last = True
                if h <= self.h_min:
                    return "h_min"
                fac = 0.9 * err ** -0.125
                self.h = min(max(h * min(1.0, max(0.2, fac)), self.h_min), self.h_max)
        return "ok"


def respace(hist, ratio):
    """History f_n, f_{n-1}, f_{n-2}, f_{n-3} (spacing h) moved to spacing ratio * h: the cubic
    through the four points, p(s) at s = j ratio (s in units of h backwards from t_n), by
    Lagrange's formula."""
    out = [hist[0]]
    for j in range(1, 4):
        s = j * ratio
        acc = 0.0
        for i in range(4):
            w = 1.0
            for m in range(4):
                if m != i:
                    w *= (s - m) / (i - m)
            acc = acc + w * hist[i]
        out.append(acc)
    return out


class Abm4Var:
    """Adams-Bashforth-Moulton 4 PECE with a variable step.

    The first three steps are classical RK4 steps of h0 (no error estimate) that build the
    history.  Then each step predicts with AB4, evaluates, corrects with AM4 and estimates the
    corrector's local error by Milne's device, est = (19/270) (y_c - y_p); err is the RMS of
    est / (atol + rtol max(|y|, |y_c|)).  err <= 1 accepts (then the right-hand side at the new
    point joins the history), else the step is repeated smaller.  The next step is
    h min(fmax, max(0.2, 0.9 err^(-1/5))) clipped to [h_min, h_max], fmax = 1.5 (1 right after
    a rejection: growth moves the history by extrapolating its cubic, to at most 4.5 old steps
    back); a change of less than 10 % upwards is not taken.  A step that would pass t_end
    is shortened to end there.  Whenever the step changes, the history is moved onto the new
    spacing (respace)."""

    def __init__(self, f, y0, *, rtol, atol, h0, h_min, h_max, max_steps, t0=0.0):
        self.f = f
        self.y = np.array(y0, dtype=np.float64)
        self.t = float(t0)
        self.rtol, self.atol = rtol, atol
        self.h0, self.h_min, self.h_max = h0, h_min, h_max
        self.h = min(max(h0, h_min), h_max)  # the history's spacing once it is full
        self.max_steps = max_steps
        self.hist = []
        self.accepted = 0
        self.rejected = 0
        self.evals = 0
        self.last_err = 0.0
        self.rejected_last = False

    def _f(self, t, y):
        self.evals += 1
        return np.asarray(self.f(t, y), dtype=np.float64)

    def advance(self, t_end):
        """Advance to t_end; returns "ok", "max_steps" or "h_min"."""
        attempts = 0
        while self.t < t_end:
            if attempts >= self.max_steps:
                return "max_steps"
            attempts += 1
            if not self.hist:
                self.hist = [self._f(self.t, self.y)]
            h = self.h
            last = self.t + h >= t_end * (1.0 - 1e-14) - 1e-300
            if last:
                h = t_end - self.t
            if len(self.hist) < 4:
                # start: RK4 steps (the last one may be shortened; the history is then
                # restarted from the new point)
                k1 = self.hist[0]
                ks = [k1]
                for c in (0.5, 0.5, 1.0):
                    ks.append(self._f(self.t + c * h, self.y + c * h * ks[-1]))
                self.y = self.y + h * (ks[0] + 2 * ks[1] + 2 * ks[2] + ks[3]) / 6.0
                self.t = t_end if last else self.t + h
                fn = self._f(self.t, self.y)
                self.hist = [fn] if h != self.h else ([fn] + self.hist)[:4]
                self.accepted += 1
                continue
            if h != self.h:
                self.hist = respace(self.hist, h / self.h)
            pred = self.y + h * sum(float(AB4[j]) * self.hist[j] for j in range(4))
            fp = self._f(self.t + h, pred)
            corr = self.y + h * (float(AM4[0]) * fp +
                                 sum(float(AM4[j + 1]) * self.hist[j] for j in range(3)))
            est = (19.0 / 270.0) * (corr - pred)
            sc = self.atol + self.rtol * np.maximum(np.abs(self.y), np.abs(corr))
            err = math.sqrt(float(np.mean((est / sc) ** 2)))
            self.last_err = err
            if err <= 1.0:
                self.y = corr
                self.t = t_end if last else self.t + h
                self.hist = [self._f(self.t, self.y)] + self.hist[:3]
                self.accepted += 1
                fac = 0.9 * err ** -0.2 if err > 0 else 1.5
                fmax = 1.0 if self.rejected_last else 1.5
                fac = min(fmax, max(0.2, fac))
                if 1.0 <= fac < 1.1:
                    fac = 1.0
                hn = min(max(h * fac, self.h_min), self.h_max)
                self.h = h  # the history's spacing
                if hn != h:
                    self.hist = respace(self.hist, hn / h)
                self.h = hn
                self.rejected_last = False
            else:
                self.rejected += 1
                self.rejected_last = True
                if h <= self.h_min:
                    return "h_min"
                fac = min(1.0, max(0.2, 0.9 * err ** -0.2))
                hn = min(max(h * fac, self.h_min), self.h_max)
                self.hist = respace(self.hist, hn / h)
                self.h = hn
        return "ok"
