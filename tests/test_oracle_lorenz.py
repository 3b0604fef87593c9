"""Pins of the oracle's Taylor step for the Lorenz system (CPU only).

What fixes the result independently of the oracle:
  * the Fraction-based statement of the same rounding points
    (fraction_reference) at tiny N;
  * the paper's separate first-coefficient formulas (Section 2);
  * the exact, unrounded recursion (rounding error stays within a few ulps);
  * closed forms: the z-axis solution z0*exp(-b t) and the sigma=0 affine
    system solved by a matrix exponential (mpmath.expm);
  * an independent integrator (mpmath.odefun);
  * N=1 reducing to explicit Euler;
  * the paper's own verification procedure (Section 1): a rerun at larger K
    and N agrees over the whole interval to the expected number of digits.
"""
from fractions import Fraction
import math

import mpmath
import pytest

from oracle import lorenz as lz
from oracle.bigfloat import BF, ZERO, parse, to_double, exact_mul, round_exact
import fraction_reference as fr
from workloads import BENCH_X0


def frac_state(s):
    return tuple(v.frac() for v in s)


def ulp(v: BF) -> Fraction:
    return Fraction(2) ** v.e


@pytest.mark.parametrize("L,N,nsteps", [(2, 1, 3), (2, 3, 3), (2, 4, 2), (3, 6, 2)])
def test_step_matches_fraction_reference(L, N, nsteps):
    ctx = lz.make_context(L=L, N=N)
    s = lz.state_from_strings(ctx, BENCH_X0)
    q = frac_state(s)
    for _ in range(nsteps):
        s = lz.step(ctx, s)
        q = fr.step(q, N, ctx.p)
        assert frac_state(s) == q


def test_coefficients_match_fraction_reference():
    ctx = lz.make_context(L=4, N=8)
    s = lz.state_from_strings(ctx, BENCH_X0)
    a, b, g, _, _ = lz.coefficients(ctx, s)
    A, B, G = fr.step_coefficients(*frac_state(s), 8, ctx.p)
    assert [v.frac() for v in a] == A
    assert [v.frac() for v in b] == B
    assert [v.frac() for v in g] == G


def test_first_coefficients_closed_form():
    """alpha1 = -sigma a0 + sigma b0, beta1 = R a0 - b0 - a0 g0,
    gamma1 = a0 b0 - b g0 (the paper's formulas before equation (3)), with the
    product a0*g0 and a0*b0 rounded once as a one-term Cauchy sum."""
    ctx = lz.make_context(K_digits=100, N=3)
    p = ctx.p
    x, y, z = lz.state_from_strings(ctx, BENCH_X0)
    a, b, g, _, _ = lz.coefficients(ctx, (x, y, z))
    X, Y, Z = x.frac(), y.frac(), z.frac()
    xz = fr.rne(X * Z, p)
    xy = fr.rne(X * Y, p)
    assert a[1].frac() == fr.rne(-10 * X + 10 * Y, p)
    assert b[1].frac() == fr.rne(28 * X - Y - xz, p)
    assert g[1].frac() == fr.rne(xy - ctx.b.frac() * Z, p)


def test_rounded_recursion_close_to_exact_recursion():
    ctx = lz.make_context(K_digits=100, N=30)
    s = lz.state_from_strings(ctx, BENCH_X0)
    a, b, g, _, _ = lz.coefficients(ctx, s)
    A, B, G = fr.exact_coefficients(*frac_state(s), 30, b=ctx.b.frac())
    for got, ref in ((a, A), (b, B), (g, G)):
        for i, (v, q) in enumerate(zip(got, ref)):
            if q == 0:
                assert v == ZERO
                continue
            rel = abs(v.frac() - q) / abs(q)
            assert rel < Fraction(40 * (i + 1) ** 2, 2 ** (ctx.p - 1)), i


def test_z_axis_invariant_and_closed_form():
    """x0 = y0 = 0: x and y stay exactly 0, all Cauchy sums vanish, and
    z_n = z0 * exp(-b n tau) up to rounding and truncation."""
    ctx = lz.make_context(K_digits=100, N=40)
    p = ctx.p
    s = (ZERO, ZERO, parse("35.64", p))
    nsteps = 60
    a, b, g, s1, s2 = lz.coefficients(ctx, s)
    assert all(v == ZERO for v in a + b + s1 + s2)
    z = s
    for _ in range(nsteps):
        z = lz.step(ctx, z)
    assert z[0] == ZERO and z[1] == ZERO
    # exact rational truncated series, one factor per step
    bt = -ctx.b.frac() * ctx.tau.frac()
    fac = sum(bt ** i / math.factorial(i) for i in range(ctx.N + 1))
    ref = parse("35.64", p).frac() * fac ** nsteps
    rel = abs(z[2].frac() - ref) / ref
    assert rel < Fraction(nsteps * ctx.N * 4, 2 ** (p - 1))
    mpmath.mp.prec = p + 64
    t = mpmath.mpf(ctx.tau.frac().numerator) / ctx.tau.frac().denominator * nsteps
    bm = mpmath.mpf(ctx.b.frac().numerator) / ctx.b.frac().denominator
    z0 = parse("35.64", p).frac()
    closed = mpmath.mpf(z0.numerator) / z0.denominator
    closed = closed * mpmath.exp(-bm * t)
    got = mpmath.mpf(z[2].frac().numerator) / z[2].frac().denominator
    digits = -mpmath.log10(abs(got - closed) / closed)
    mpmath.mp.prec = 53
    assert digits > 100 - 6


def test_sigma_zero_affine_closed_form():
    """sigma = 0: x stays x0 exactly and (y, z) solves the affine system
    y' = R x0 - y - x0 z, z' = x0 y - b z, whose solution is a matrix
    exponential."""
    ctx = lz.make_context(K_digits=100, N=40, sigma="0")
    p = ctx.p
    s0 = lz.state_from_strings(ctx, ("0.75", "-1.5", "2.25"))
    nsteps = 50
    s = s0
    for _ in range(nsteps):
        s = lz.step(ctx, s)
    assert s[0] == s0[0]
    mpmath.mp.prec = p + 64
    f = lambda q: mpmath.mpf(q.numerator) / q.denominator
    x0, y0, z0 = (f(v.frac()) for v in s0)
    bm = f(ctx.b.frac())
    t = f(ctx.tau.frac()) * nsteps
    M = mpmath.matrix([[-1, -x0], [x0, -bm]])
    c = mpmath.matrix([28 * x0, 0])
    Minv_c = mpmath.lu_solve(M, c)
    v0 = mpmath.matrix([y0, z0])
    v = mpmath.expm(M * t) * (v0 + Minv_c) - Minv_c
    for got, ref in ((s[1], v[0]), (s[2], v[1])):
        err = abs(f(got.frac()) - ref) / abs(ref)
        assert -mpmath.log10(err) > 100 - 6
    mpmath.mp.prec = 53


def test_against_independent_integrator_mpmath_odefun():
    ctx = lz.make_context(K_digits=100, N=40)
    s = lz.state_from_strings(ctx, BENCH_X0)
    nsteps = 30
    for _ in range(nsteps):
        s = lz.step(ctx, s)
    mpmath.mp.dps = 45
    b = mpmath.mpf(8) / 3
    sol = mpmath.odefun(lambda t, v: [10 * (v[1] - v[0]), 28 * v[0] - v[1] - v[0] * v[2],
                                      v[0] * v[1] - b * v[2]],
                        0, [mpmath.mpf("-15.8"), mpmath.mpf("-17.48"), mpmath.mpf("35.64")])
    ref = sol(mpmath.mpf(nsteps) / 100)
    for got, r in zip(s, ref):
        q = got.frac()
        err = abs(mpmath.mpf(q.numerator) / q.denominator - r) / abs(r)
        assert err < mpmath.mpf(10) ** -35
    mpmath.mp.dps = 15


def test_order_one_is_explicit_euler():
    """N = 1: x_{n+1} = x_n + tau f(x_n); with the rounding points this is
    within a few ulps of the exact Euler step."""
    ctx = lz.make_context(L=4, N=1)
    p = ctx.p
    s = lz.state_from_strings(ctx, BENCH_X0)
    for _ in range(3):
        X, Y, Z = frac_state(s)
        tau = ctx.tau.frac()
        bb = ctx.b.frac()
        ref = (X + tau * 10 * (Y - X), Y + tau * (28 * X - Y - X * Z), Z + tau * (X * Y - bb * Z))
        s = lz.step(ctx, s)
        for v, q in zip(s, ref):
            assert abs(v.frac() - q) <= 4 * ulp(v)


def test_paper_verification_rerun_agreement():
    """Section 1: the solution is reliable if a rerun at larger K and N
    coincides with it over the whole interval.  Reading of the expected
    agreement: at least min(0.98K, 1.1N) - 0.40 t - 3 digits at time t
    (truncation error of order N, precision K, Lyapunov loss ~0.39 digits
    per time unit)."""
    c1 = lz.make_context(K_digits=100, N=40)
    c2 = lz.make_context(K_digits=125, N=50)
    s1 = lz.state_from_strings(c1, BENCH_X0)
    s2 = lz.state_from_strings(c2, BENCH_X0)
    worst = None
    for n in range(1, 801):
        s1 = lz.step(c1, s1)
        s2 = lz.step(c2, s2)
        if n % 100 == 0:
            t = n / 100
            for u, v in zip(s1, s2):
                d = abs(u.frac() - v.frac())
                if d == 0:
                    continue
                dig = -math.log10(float(d / abs(v.frac())))
                bound = min(0.98 * 100, 1.1 * 40) - 0.40 * t - 3
                assert dig >= bound, (n, dig, bound)
                worst = dig if worst is None else min(worst, dig)
    assert worst is not None and worst > 20


def test_parallel_oracle_matches_single_process():
    """The Cauchy sums split over worker processes into exact partials (the
    paper's per-thread containers, Section 4), added and rounded once by the
    master, give the single-process oracle's coefficients bit for bit, for
    several worker counts (including more workers than terms)."""
    from oracle.parallel import ParallelOracle
    ctx = lz.make_context(K_digits=60, N=30)
    x0 = lz.state_from_strings(ctx, ("-15.8", "-17.48", "35.64"))
    a, b, g, _, _ = lz.coefficients(ctx, x0)
    for workers in (1, 3, 5):
        with ParallelOracle(ctx, workers) as po:
            pa, pb, pg = po.coefficients(x0)
        assert (pa, pb, pg) == (a, b, g), workers
