"""Pins of the polynomial-system oracle (oracle/poly.py) to things other than
itself: the separately pinned Lorenz oracle, closed-form solutions, and the
defining property that the Taylor polynomial solves the system up to its
order, within a rigorous rounding bound."""
from decimal import Decimal, getcontext
from fractions import Fraction

import pytest

from oracle import lorenz as lz
from oracle import poly
from oracle.bigfloat import from_fraction
from workloads import BENCH_X0, POLY_SYSTEMS, POLY_X0


def system(name, L, N, tau="1/100"):
    nvar, terms = POLY_SYSTEMS[name]
    return poly.make_context(nvar, [poly.Term(*t) for t in terms], L=L, N=N, tau=tau)


def state(ctx, texts):
    from oracle.bigfloat import parse
    return tuple(parse(t, ctx.p) for t in texts)


@pytest.mark.parametrize("L,N", [(1, 6), (4, 20), (12, 40)])
def test_lorenz_terms_reproduce_the_lorenz_oracle(L, N):
    """The Lorenz terms give the Lorenz recursion bit for bit: coefficients
    of one step and three whole steps."""
    pc = system("lorenz", L, N)
    lc = lz.make_context(L=L, N=N)
    x0 = lz.state_from_strings(lc, BENCH_X0)
    xs, _ = poly.coefficients(pc, x0)
    a, b, g, _, _ = lz.coefficients(lc, x0)
    assert xs == [a, b, g]
    assert poly.integrate(pc, x0, 3) == lz.integrate(lc, x0, 3)


def test_square_has_the_geometric_series():
    """x' = x^2 from x0 = 1/8: x(t) = x0 / (1 - x0 t), whose Taylor
    coefficients are x0^(i+1), exact in binary; every Cauchy sum is
    (i+1) x0^(i+2), so every rounding is exact."""
    ctx = system("square", 4, 30)
    x0 = state(ctx, POLY_X0["square"])
    xs, _ = poly.coefficients(ctx, x0)
    for i, c in enumerate(xs[0]):
        assert c == from_fraction(Fraction(1, 8) ** (i + 1), ctx.p), i


def test_decay_follows_the_exponential():
    """x' = -x from 1: after n steps of size tau_p the value is exp(-n tau_p)
    up to the series remainder (about tau^(N+1) / (N+1)!, far below the
    precision) and one rounding error per coefficient and Horner step."""
    L, N, n = 8, 40, 20
    ctx = system("decay", L, N)
    x = poly.integrate(ctx, state(ctx, POLY_X0["decay"]), n)
    getcontext().prec = 150
    t = ctx.tau.frac() * n
    ref = (-(Decimal(t.numerator) / Decimal(t.denominator))).exp()
    got = Decimal(x[0].frac().numerator) / Decimal(x[0].frac().denominator)
    bound = Decimal(n * (2 * N + 4)) * (Decimal(2) ** (-ctx.p))
    assert abs(got - ref) <= bound


def test_oscillator_keeps_its_radius():
    """x' = -y, y' = x: x^2 + y^2 stays 1 up to the rounding errors."""
    L, N, n = 8, 40, 30
    ctx = system("oscillator", L, N)
    x, y = poly.integrate(ctx, state(ctx, POLY_X0["oscillator"]), n)
    r2 = x.frac() ** 2 + y.frac() ** 2
    assert abs(r2 - 1) <= Fraction(n * (4 * N + 8), 2 ** ctx.p)
    assert abs(x.frac() - 1) > Fraction(1, 100)  # the state did move (t = 0.3)


def residual_within_bound(terms, nvar, ctx, xs):
    """The Taylor polynomial P_v(t) = sum_i x_{v,i} t^i satisfies
    P_v' = f_v(P) up to degree N-1: the residual's coefficient of t^i is at
    most 2^(1-p) ((i+1) |x_{v,i+1}| + sum of |coef| sum_k |x_{u,i-k} x_{w,k}|
    over the product terms) (the roundings of the new coefficient and of the
    Cauchy sums), with a factor 2 of margin.  Computed with exact rationals
    from the polynomial definition, not from the recursion."""
    X = [[c.frac() for c in row] for row in xs]
    N = ctx.N
    unit = Fraction(2, 2 ** ctx.p)

    def mul(a, b):  # polynomial product truncated to degree N - 1
        out = [Fraction(0)] * N
        for i in range(N):
            for k in range(i + 1):
                out[i] += a[i - k] * b[k]
        return out

    for v in range(nvar):
        deriv = [(i + 1) * X[v][i + 1] for i in range(N)]
        rhs = [Fraction(0)] * N
        slack = [(i + 1) * abs(X[v][i + 1]) for i in range(N)]
        for (eq, coef, u, w) in terms:
            if eq != v:
                continue
            c = Fraction(coef)
            if u < 0:
                rhs[0] += c
            elif w < 0:
                for i in range(N):
                    rhs[i] += c * X[u][i]
            else:
                prod = mul(X[u], X[w])
                absprod = mul([abs(t) for t in X[u]], [abs(t) for t in X[w]])
                for i in range(N):
                    rhs[i] += c * prod[i]
                    slack[i] += abs(c) * absprod[i]
        for i in range(N):
            if abs(deriv[i] - rhs[i]) > unit * slack[i] * 2 + unit:
                return False
    return True


@pytest.mark.parametrize("name", ["rossler", "chen", "rossler4", "lorenz"])
def test_series_solves_the_system(name):
    nvar, terms = POLY_SYSTEMS[name]
    ctx = system(name, 3, 14)
    xs, _ = poly.coefficients(ctx, state(ctx, POLY_X0[name]))
    assert residual_within_bound(terms, nvar, ctx, xs)


@pytest.mark.parametrize("drop", range(7))
def test_dropped_term_is_caught(drop):
    """The residual check fails when any one term is dropped from the
    oracle's copy of the system (a planted mistake, on the CPU)."""
    nvar, terms = POLY_SYSTEMS["rossler"]
    bad = poly.make_context(nvar, [poly.Term(*t) for j, t in enumerate(terms) if j != drop],
                            L=3, N=10)
    xs, _ = poly.coefficients(bad, state(bad, POLY_X0["rossler"]))
    assert not residual_within_bound(terms, nvar, bad, xs)


def test_swapped_cauchy_index_is_caught():
    """A Cauchy sum read with both indices running the same way
    (sum_k x_{u,k} x_{w,k}) breaks the residual check."""
    nvar, terms = POLY_SYSTEMS["chen"]
    ctx = system("chen", 3, 10)
    orig = poly.cauchy_sum
    try:
        from oracle.bigfloat import exact_mul, round_sum
        poly.cauchy_sum = lambda c, xs, u, w, i: round_sum(
            [exact_mul(xs[u][k], xs[w][k]) for k in range(i + 1)], c.p)
        xs, _ = poly.coefficients(ctx, state(ctx, POLY_X0["chen"]))
    finally:
        poly.cauchy_sum = orig
    assert not residual_within_bound(terms, nvar, ctx, xs)
