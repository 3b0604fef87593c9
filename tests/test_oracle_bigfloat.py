"""Pins of the oracle's number type and rounding (CPU only).

Each check compares against something other than the oracle itself:
brute-force enumeration of representable values, the Fraction-based rounder
of fraction_reference, mpmath's correctly rounded fdot/fdiv at precision p,
and CPython's correctly rounded int/int division.
"""
import random
from fractions import Fraction

import mpmath
import pytest

from oracle.bigfloat import (BF, ZERO, digits_to_limbs, div_round, exact_mul,
                             from_double, parse, round_ratio, round_sum,
                             to_double, is_normalized)
import fraction_reference as fr


def brute_rne(q: Fraction, p: int) -> Fraction:
    """Nearest p-bit value by enumerating every candidate mantissa of the
    two binades around q; ties go to the even mantissa."""
    if q == 0:
        return Fraction(0)
    sign = 1 if q > 0 else -1
    a = abs(q)
    cands = []
    for e in range(-20, 20):
        scale = Fraction(2) ** e
        for m in range(1 << (p - 1), 1 << p):
            v = m * scale
            if abs(v - a) <= a:       # prune far away values
                cands.append((abs(v - a), m & 1, v))
    cands.sort(key=lambda t: (t[0], t[1]))
    return sign * cands[0][2]


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6])
def test_rne_matches_brute_force_small_p(p):
    qs = set()
    for num in range(-70, 71):
        for den in range(1, 13):
            qs.add(Fraction(num, den))
    for q in sorted(qs):
        got = round_ratio(q.numerator, q.denominator, 0, p)
        assert got.frac() == brute_rne(q, p), (q, p)
        assert is_normalized(got, p)


def test_explicit_ties_to_even():
    p = 4
    # 8..15 are 4-bit mantissas; halfway cases go to the even neighbour.
    assert round_ratio(17, 2, 0, p).frac() == 8      # 8.5 -> 8
    assert round_ratio(19, 2, 0, p).frac() == 10     # 9.5 -> 10
    assert round_ratio(-19, 2, 0, p).frac() == -10
    assert round_ratio(31, 2, 0, p).frac() == 16     # 15.5 -> 16 (carry into next binade)
    assert round_ratio(33, 1, 0, p).frac() == 32     # 33 -> 32 (tie, 16 is even)
    assert round_ratio(35, 1, 0, p).frac() == 36     # 35 -> 36 (tie, 18 is even)
    r = round_ratio(31, 2, 0, p)
    assert r.m == 8 and r.e == 1 and is_normalized(r, p)


@pytest.mark.parametrize("p", [64, 384, 1024])
def test_rne_matches_fraction_reference(p):
    rnd = random.Random(p)
    for _ in range(300):
        num = rnd.randrange(-(1 << (p + 40)), 1 << (p + 40))
        den = rnd.randrange(1, 1 << rnd.randrange(1, 80))
        e = rnd.randrange(-200, 200)
        q = Fraction(num, den) * Fraction(2) ** e
        assert round_ratio(num, den, e, p).frac() == fr.rne(q, p)


def _mp(v: BF):
    return mpmath.mpf((0 if v.s >= 0 else 1, v.m, v.e, v.m.bit_length())) if v.s else mpmath.mpf(0)


def _bf_from_mp(x) -> Fraction:
    s, man, e, _ = x._mpf_
    return Fraction(0) if man == 0 else (-1 if s else 1) * Fraction(man) * Fraction(2) ** e


@pytest.mark.parametrize("L", [2, 12, 22])
def test_cauchy_round_matches_mpmath_fdot(L):
    """exact-sum-then-round of a product sum equals mpmath.fdot at prec p
    (mpmath sums exactly and rounds once, round-nearest-even)."""
    p = 32 * L
    rnd = random.Random(L)
    mpmath.mp.prec = p
    for trial in range(150):
        n = rnd.randrange(1, 12)
        us = [BF(rnd.choice([-1, 1]), rnd.randrange(1 << (p - 1), 1 << p), rnd.randrange(-40, 40) - p) for _ in range(n)]
        vs = [BF(rnd.choice([-1, 1]), rnd.randrange(1 << (p - 1), 1 << p), rnd.randrange(-40, 40) - p) for _ in range(n)]
        if trial % 3 == 0 and n >= 2:
            # forced cancellation: the last product nearly cancels the first
            us[-1] = BF(-us[0].s, us[0].m, us[0].e)
            vs[-1] = BF(vs[0].s, vs[0].m + rnd.randrange(0, 3) if vs[0].m + 3 < (1 << p) else vs[0].m, vs[0].e)
        ours = round_sum([exact_mul(u, v) for u, v in zip(us, vs)], p)
        ref = mpmath.fdot([_mp(u) for u in us], [_mp(v) for v in vs])
        assert ours.frac() == _bf_from_mp(ref)
        # the order of the terms does not change the result
        perm = list(range(n))
        rnd.shuffle(perm)
        again = round_sum([exact_mul(us[j], vs[j]) for j in perm], p)
        assert again == ours
    mpmath.mp.prec = 53


@pytest.mark.parametrize("p", [384, 6656])
def test_div_round_matches_mpmath(p):
    rnd = random.Random(p)
    mpmath.mp.prec = p
    for _ in range(100):
        X = rnd.randrange(-(1 << (2 * p)), 1 << (2 * p))
        e = rnd.randrange(-3 * p, p)
        d = rnd.randrange(1, 4000)
        ours = div_round((X, e), d, p)
        mpmath.mp.prec = 4 * p + 64           # the numerator is built exactly
        num = mpmath.mpf((0 if X >= 0 else 1, abs(X), e, abs(X).bit_length())) if X else mpmath.mpf(0)
        mpmath.mp.prec = p
        assert ours.frac() == fr.rne(Fraction(X) * Fraction(2) ** e / d, p)
        ref = mpmath.fdiv(num, d)
        assert ours.frac() == _bf_from_mp(ref)
    mpmath.mp.prec = 53


def test_near_tie_divisions_against_fraction_reference():
    """Numerators built to sit next to a rounding tie after division."""
    p = 64
    for d in range(1, 200):
        for off in (-1, 0, 1):
            # q*d + off over d, with q an odd 65-bit integer: (q + off/d) near a tie at p bits
            q = (1 << 64) + 2 * d + 1
            X = q * d + off
            ours = div_round((X, 0), d, p)
            assert ours.frac() == fr.rne(Fraction(X, d), p)


def test_digits_to_limbs_reading():
    assert [digits_to_limbs(K) for K in (100, 200, 300, 400, 800, 1600, 2000, 4000)] == \
        [12, 22, 32, 42, 84, 168, 208, 416]
    for K in range(1, 300):
        L = digits_to_limbs(K)
        assert 2 ** (32 * L) >= 10 ** K          # p bits hold K digits
        assert L % 2 == 0 and 2 ** (32 * (L - 2)) < 10 ** K   # and no whole word less would


def test_parse_and_double_export():
    p = 384
    mpmath.mp.prec = p
    for s in ("-15.8", "-17.48", "35.64", "8/3", "1/100", "1e-2", "0"):
        v = parse(s, p)
        if s == "0":
            assert v == ZERO
            continue
        ref = mpmath.mpf(s) if "/" not in s else mpmath.mpf(s.split("/")[0]) / int(s.split("/")[1])
        assert v.frac() == _bf_from_mp(ref)
    mpmath.mp.prec = 53
    v = parse("-15.8", p)
    assert to_double(v) == -15.8
    assert to_double(parse("1/3", p)) == 1 / 3
    x = 0.1234567891234
    assert from_double(x, 64).frac() == Fraction(x)
    assert to_double(from_double(x, 64)) == x
