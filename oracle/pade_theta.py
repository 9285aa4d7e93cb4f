"""Largest 1-norm theta_m for which the [m/m] Pade approximant of exp reaches a
given unit roundoff u (Higham 2005, "The scaling and squaring method for the
matrix exponential revisited", Sec. 2).

TEST INFRASTRUCTURE (part of the oracle).  The backward error of r_m is
Delta A = h(A) with h(x) = log(e^{-x} r_m(x)) = sum_{k >= 2m+1} c_k x^k, and
||Delta A|| / ||A|| <= (sum_k |c_k| theta^k) / theta; theta_m solves
(sum_k |c_k| theta^k) / theta = u.  The series is formed in exact rational
arithmetic (power-series division, product with e^{-x}, then the logarithm by
the recurrence of L' = F'/F) and evaluated in 60-digit floating point.

    python oracle/pade_theta.py      prints theta_m for u = 2^-53 and 2^-24
"""
from __future__ import annotations

from fractions import Fraction
from math import factorial

import mpmath as mp


def pade_coefficients(m: int) -> list[Fraction]:
    """b_j = (2m - j)! m! / ((2m)! j! (m - j)!), so p(x) = sum b_j x^j, q(x) = p(-x)."""
    return [Fraction(factorial(2 * m - j) * factorial(m), factorial(2 * m) * factorial(j) * factorial(m - j))
            for j in range(m + 1)]


def backward_error_series(m: int, n: int) -> list[Fraction]:
    """Coefficients c_0..c_n of h(x) = log(e^{-x} p(x) / q(x))."""
    b = pade_coefficients(m)
    P = b + [Fraction(0)] * (n + 1 - len(b))
    Q = [c * (-1) ** j for j, c in enumerate(b)] + [Fraction(0)] * (n + 1 - len(b))
    R = [Fraction(0)] * (n + 1)
    for k in range(n + 1):                       # R = P / Q
        R[k] = (P[k] - sum(Q[i] * R[k - i] for i in range(1, k + 1))) / Q[0]
    E = [Fraction((-1) ** k, factorial(k)) for k in range(n + 1)]
    F = [sum(E[i] * R[k - i] for i in range(k + 1)) for k in range(n + 1)]   # F = e^{-x} R, F_0 = 1
    L = [Fraction(0)] * (n + 1)
    for k in range(1, n + 1):                    # log F: k L_k = k F_k - sum_{i<k} i L_i F_{k-i}
        L[k] = F[k] - sum(Fraction(i, k) * L[i] * F[k - i] for i in range(1, k))
    return L


def theta(m: int, u: float | mp.mpf, n: int = 150) -> float:
    mp.mp.dps = 60
    c = [mp.mpf(abs(x.numerator)) / x.denominator for x in backward_error_series(m, n)]
    u = mp.mpf(u)

    def g(x):
        return mp.fsum(ck * x ** k for k, ck in enumerate(c)) / x - u

    lo, hi = mp.mpf("1e-8"), mp.mpf("0.5")
    while g(hi) < 0:
        hi *= 1.5
    for _ in range(200):
        mid = (lo + hi) / 2
        if g(mid) < 0:
            lo = mid
        else:
            hi = mid
    return float(lo)


if __name__ == "__main__":
    for m in (3, 5, 7, 9, 13):
        print(m, repr(theta(m, mp.mpf(2) ** -53)), repr(theta(m, mp.mpf(2) ** -24)))
