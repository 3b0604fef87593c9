"""Binary multiple-precision floating point in plain Python integers.

A value is BF(s, m, e) meaning s * m * 2**e with s in {-1, 0, +1}.  A rounded
(normalised) value with precision p has 2**(p-1) <= m < 2**p; zero is
BF(0, 0, 0).  This mirrors the role of the GMP numbers the paper uses
(Section 4) with a binary exponent and one explicit rounding rule:
round-to-nearest, ties-to-even.

Exact intermediate values are pairs (X, e) meaning the integer X times 2**e;
they are never rounded until `round_exact` / `round_ratio` is called.

Every function here is written from the definition of the operation; there
is no blocking or reordering.
"""
from fractions import Fraction
from typing import Iterable, NamedTuple, Tuple


class BF(NamedTuple):
    s: int  # sign: -1, 0 or +1
    m: int  # mantissa magnitude, >= 0
    e: int  # exponent of the mantissa's least significant bit

    def frac(self) -> Fraction:
        """Exact rational value."""
        if self.s == 0:
            return Fraction(0)
        v = Fraction(self.s * self.m)
        return v * (Fraction(2) ** self.e)


ZERO = BF(0, 0, 0)


def digits_to_limbs(K: int) -> int:
    """Number of 32-bit limbs for K decimal digits.

    The paper states the precision in decimal digits K (Section 1, Section 5:
    K=800) or in bits (Section 5: 8000 bits).  Reading used here: the
    smallest whole number of 64-bit words whose bit count reaches K*log2(10),
    counted in 32-bit limbs, L = 2*ceil(ceil(K*log2 10)/64).
    ceil(K*log2 10) is the bit length of 10**K (10**K is never a power of 2).
    """
    if K < 1:
        raise ValueError("K must be >= 1")
    bits = (10 ** K).bit_length()
    return 2 * ((bits + 63) // 64)


def round_ratio(num: int, den: int, exp: int, p: int) -> BF:
    """Round (num/den) * 2**exp to p bits, round-to-nearest ties-to-even.

    num is any integer, den a positive integer.  Found by choosing the shift
    k for which q = floor(|num| * 2**k / den) has exactly p bits and then
    deciding the rounding from the remainder.
    """
    if den <= 0:
        raise ValueError("den must be positive")
    if p < 2:
        raise ValueError("p must be >= 2")
    if num == 0:
        return ZERO
    s = 1 if num > 0 else -1
    n = -num if num < 0 else num
    k = p - (n.bit_length() - den.bit_length())
    while True:
        if k >= 0:
            q, r = divmod(n << k, den)
            d = den
        else:
            d = den << (-k)
            q, r = divmod(n, d)
        if q >= (1 << p):
            k -= 1
        elif q < (1 << (p - 1)):
            k += 1
        else:
            break
    # value = (q + r/d) * 2**(exp-k), with 0 <= r < d
    if 2 * r > d or (2 * r == d and (q & 1)):
        q += 1
        if q == (1 << p):
            q >>= 1
            k -= 1
    return BF(s, q, exp - k)


def round_exact(x: Tuple[int, int], p: int) -> BF:
    """Round the exact value X * 2**e to p bits (RNE)."""
    X, e = x
    return round_ratio(X, 1, e, p)


def exact(v: BF) -> Tuple[int, int]:
    """The exact value of a BF as (signed integer, exponent)."""
    return (v.s * v.m, v.e)


def exact_mul(u: BF, v: BF) -> Tuple[int, int]:
    """Exact product of two BF values."""
    return (u.s * u.m * v.s * v.m, u.e + v.e)


def exact_sum(terms: Iterable[Tuple[int, int]]) -> Tuple[int, int]:
    """Exact sum of (X, e) terms: shift every term to the smallest exponent
    among the nonzero terms and add the integers.  The empty sum is (0, 0)."""
    terms = [t for t in terms if t[0] != 0]
    if not terms:
        return (0, 0)
    emin = min(e for _, e in terms)
    return (sum(X << (e - emin) for X, e in terms), emin)


def round_sum(terms: Iterable[Tuple[int, int]], p: int) -> BF:
    """One rounding of an exact sum."""
    return round_exact(exact_sum(terms), p)


def div_round(x: Tuple[int, int], d: int, p: int) -> BF:
    """Round (X * 2**e) / d to p bits for a positive integer d."""
    X, e = x
    return round_ratio(X, d, e, p)


def from_fraction(q: Fraction, p: int) -> BF:
    """Round an exact rational to p bits."""
    return round_ratio(q.numerator, q.denominator, 0, p)


def parse(text: str, p: int) -> BF:
    """Parse an exact decimal ("-15.8", "1e-2") or rational ("8/3") string
    and round it once to p bits."""
    return from_fraction(Fraction(text.strip()), p)


def from_double(v: float, p: int) -> BF:
    """A float64 value as a BF (exact whenever p >= 53)."""
    return from_fraction(Fraction(v), p)


def to_double(v: BF) -> float:
    """Nearest float64 (RNE).  CPython's int/int true division is correctly
    rounded, which makes this the round-to-nearest of the exact value."""
    if v.s == 0:
        return 0.0
    q = v.frac()
    return q.numerator / q.denominator


def neg(v: BF) -> BF:
    return BF(-v.s, v.m, v.e)


def is_normalized(v: BF, p: int) -> bool:
    if v.s == 0:
        return v.m == 0
    return (1 << (p - 1)) <= v.m < (1 << p)
