"""Exact Clebsch-Gordan coefficients <j1 m1; j2 m2 | J M> with Condon-Shortley
phases, by Racah's closed formula evaluated in rational arithmetic.

All spins and projections are passed doubled (2j, 2m) so they are integers.
These coefficients define the SU(2)-coupled (multiplet) basis of the MPS
(Sec. "Conservation of the total spin in the DMRG-SCF procedure").
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache


def tri(a2, b2, c2):
    return abs(a2 - b2) <= c2 <= a2 + b2 and (a2 + b2 + c2) % 2 == 0


@lru_cache(maxsize=None)
def cg(j1, m1, j2, m2, J, M):
    """<j1 m1; j2 m2 | J M>, all arguments doubled."""
    if m1 + m2 != M or not tri(j1, j2, J):
        return 0.0
    if abs(m1) > j1 or abs(m2) > j2 or abs(M) > J:
        return 0.0
    if (j1 + m1) % 2 or (j2 + m2) % 2 or (J + M) % 2:
        return 0.0
    f = math.factorial
    a, b, c = (J + j1 - j2) // 2, (J - j1 + j2) // 2, (j1 + j2 - J) // 2
    pref = Fraction((J + 1) * f(a) * f(b) * f(c), f((j1 + j2 + J) // 2 + 1))
    pref *= (f((J + M) // 2) * f((J - M) // 2) * f((j1 - m1) // 2) * f((j1 + m1) // 2)
             * f((j2 - m2) // 2) * f((j2 + m2) // 2))
    s = Fraction(0)
    for k in range(c + 1):
        t = ((j1 - m1) // 2 - k, (j2 + m2) // 2 - k, (J - j2 + m1) // 2 + k, (J - j1 - m2) // 2 + k)
        if min(t) < 0:
            continue
        s += Fraction((-1) ** k, f(k) * f(c - k) * f(t[0]) * f(t[1]) * f(t[2]) * f(t[3]))
    if s == 0:
        return 0.0
    mag = math.sqrt(pref * s * s)
    return mag if s > 0 else -mag
