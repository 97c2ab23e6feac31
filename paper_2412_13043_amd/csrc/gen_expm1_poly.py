"""Coefficients of the float64 expm1 kernel polynomial used in frg_math.hpp.

expm1(r) = r + r^2 Q(r) on |r| <= ln2/2, with Q a degree-8 Chebyshev interpolant of
(expm1(r) - r)/r^2 (near-minimax; mpmath.chebyfit at 40 digits), printed highest degree first.
Run: python gen_expm1_poly.py
"""
import mpmath as mp

mp.mp.dps = 40
A = mp.log(2) / 2


def Q(r):
    if abs(r) < mp.mpf("1e-25"):
        return mp.mpf(1) / 2
    return (mp.expm1(r) - r) / (r * r)


if __name__ == "__main__":
    coeffs, err = mp.chebyfit(Q, [-A, A], 9, error=True)
    for k, c in enumerate(coeffs):
        print(f"    constexpr double Q{8 - k} = {float(c)!r};")
    worst = 0
    for i in range(4001):
        r = -A + 2 * A * i / 4000
        if r == 0:
            continue
        q = mp.mpf(0)
        for c in coeffs:
            q = q * r + mp.mpf(float(c))
        worst = max(worst, abs(r + r * r * q - mp.expm1(r)) / abs(mp.expm1(r)))
    print(f"// max relative error with double coefficients (exact arithmetic): {float(worst):.2e}")
