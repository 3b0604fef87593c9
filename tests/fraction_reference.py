"""A second, independent statement of the rounding rule and of the Taylor
step, in exact rationals (fractions.Fraction), used only to pin the oracle at
tiny sizes.

The rounding here never shifts integers: it locates the binade by comparing
the rational against powers of two, scales into [2**(p-1), 2**p), takes the
floor and compares the fractional part with 1/2.  Values stay Fractions
throughout, so this shares neither representation nor rounding code with the
oracle.
"""
from fractions import Fraction
import math


def binade(q: Fraction) -> int:
    """The integer e with 2**e <= |q| < 2**(e+1)."""
    q = abs(q)
    e = q.numerator.bit_length() - q.denominator.bit_length()
    two = Fraction(2)
    while two ** e > q:
        e -= 1
    while two ** (e + 1) <= q:
        e += 1
    return e


def rne(q: Fraction, p: int) -> Fraction:
    """Round-to-nearest, ties-to-even, to p significant bits."""
    if q == 0:
        return Fraction(0)
    sign = 1 if q > 0 else -1
    a = abs(q)
    ulp = Fraction(2) ** (binade(a) - p + 1)
    t = a / ulp
    fl = math.floor(t)
    rest = t - fl
    if rest > Fraction(1, 2) or (rest == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return sign * fl * ulp


def step_coefficients(x, y, z, N, p, sigma=10, R=28, b=None):
    """Equation (3) with the project's rounding points, in Fractions."""
    if b is None:
        b = rne(Fraction(8, 3), p)
    A, B, G = [x], [y], [z]
    for i in range(N):
        s1 = rne(sum(A[i - k] * G[k] for k in range(i + 1)), p)
        s2 = rne(sum(A[i - k] * B[k] for k in range(i + 1)), p)
        A.append(rne((sigma * B[i] - sigma * A[i]) / (i + 1), p))
        B.append(rne((R * A[i] - B[i] - s1) / (i + 1), p))
        G.append(rne((s2 - b * G[i]) / (i + 1), p))
    return A, B, G


def horner(c, tau, p):
    h = c[-1]
    for i in range(len(c) - 2, -1, -1):
        h = rne(h * tau + c[i], p)
    return h


def step(state, N, p, tau=None, **kw):
    if tau is None:
        tau = rne(Fraction(1, 100), p)
    A, B, G = step_coefficients(*state, N, p, **kw)
    return (horner(A, tau, p), horner(B, tau, p), horner(G, tau, p))


def exact_coefficients(x, y, z, N, sigma=10, R=28, b=Fraction(8, 3)):
    """Equation (3) with no rounding at all."""
    A, B, G = [x], [y], [z]
    for i in range(N):
        s1 = sum(A[i - k] * G[k] for k in range(i + 1))
        s2 = sum(A[i - k] * B[k] for k in range(i + 1))
        A.append((sigma * B[i] - sigma * A[i]) / (i + 1))
        B.append((R * A[i] - B[i] - s1) / (i + 1))
        G.append((s2 - b * G[i]) / (i + 1))
    return A, B, G
