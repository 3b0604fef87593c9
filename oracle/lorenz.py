"""Taylor series method for the Lorenz system, exactly as the paper states it.

  * Lorenz system (equation (1)): x' = -sigma x + sigma y, y' = R x - y - x z,
    z' = x y - b z, with sigma = 10, R = 28, b = 8/3 (Section 2).
  * N-th order Taylor step (equation (2)): x_{n+1} = x_n + sum_{i=1}^N
    alpha_i tau^i (likewise y with beta, z with gamma), evaluated by Horner's
    rule (Section 2, the paragraph after equation (3)).
  * Taylor coefficients (normalised derivatives) from the Leibniz recursion
    (equation (3)), for i = 0..N-1:
        alpha_{i+1} = (-sigma alpha_i + sigma beta_i) / (i+1)
        beta_{i+1}  = (R alpha_i - beta_i - s1_i) / (i+1)
        gamma_{i+1} = (s2_i - b gamma_i) / (i+1)
    with the two Cauchy-product sums s1_i = sum_{k=0}^i alpha_{i-k} gamma_k,
    s2_i = sum_{k=0}^i alpha_{i-k} beta_k (the sums the paper parallelises,
    Section 2 and Section 4).  alpha_0, beta_0, gamma_0 are the current state
    (x_n, y_n, z_n).

Rounding points (one RNE rounding to p bits each):
  s1_i, s2_i (exact sum of exact products); each new coefficient (exact
  numerator / (i+1)); each Horner step h <- h*tau + c_i.  The parameters
  sigma, R, b and the step tau are p-bit numbers (10 and 28 exactly, 8/3 and
  1/100 rounded once); every numerator is exact.
"""
from dataclasses import dataclass
from fractions import Fraction
from typing import List, Sequence, Tuple

from .bigfloat import (BF, ZERO, digits_to_limbs, div_round, exact, exact_mul,
                       exact_sum, parse, round_sum, from_fraction)


def neg(x: Tuple[int, int]) -> Tuple[int, int]:
    """Negation of an exact (X, e) value."""
    return (-x[0], x[1])


@dataclass
class Context:
    """Problem definition: the Lorenz parameters, precision and order."""
    L: int                      # 32-bit limbs; p = 32*L bits
    N: int                      # Taylor order
    sigma_text: str = "10"
    R_text: str = "28"
    b_text: str = "8/3"
    tau_text: str = "1/100"
    sigma: BF = None            # p-bit roundings of the parameters and the
    R: BF = None                # step (10 and 28 are exact; 8/3 and 1/100
    b: BF = None                # are rounded once)
    tau: BF = None

    @property
    def p(self) -> int:
        return 32 * self.L

    def __post_init__(self):
        if self.L < 1 or self.N < 1:
            raise ValueError("L and N must be >= 1")
        if self.sigma is None:
            self.sigma = parse(self.sigma_text, self.p)
        if self.R is None:
            self.R = parse(self.R_text, self.p)
        if self.b is None:
            self.b = parse(self.b_text, self.p)
        if self.tau is None:
            self.tau = parse(self.tau_text, self.p)


def make_context(K_digits: int = None, N: int = 40, L: int = None,
                 b: str = "8/3", tau: str = "1/100",
                 sigma: str = "10", R: str = "28") -> Context:
    if L is None:
        L = digits_to_limbs(K_digits)
    return Context(L=L, N=N, sigma_text=str(sigma), R_text=str(R),
                   b_text=str(b), tau_text=str(tau))


def state_from_strings(ctx: Context, xs: Sequence[str]) -> Tuple[BF, BF, BF]:
    """Initial state from exact decimal or rational strings, each rounded once."""
    return tuple(parse(s, ctx.p) for s in xs)


def state_from_fractions(ctx: Context, xs: Sequence[Fraction]) -> Tuple[BF, BF, BF]:
    return tuple(from_fraction(Fraction(q), ctx.p) for q in xs)


def cauchy_terms(u: Sequence[BF], v: Sequence[BF], i: int):
    """Exact products u_{i-k} v_k for k = 0..i (one Cauchy-product sum)."""
    return [exact_mul(u[i - k], v[k]) for k in range(i + 1)]


def next_coefficients(ctx: Context, a: Sequence[BF], b: Sequence[BF],
                      g: Sequence[BF], i: int):
    """One index transition of the recursion (equation (3)): from the
    coefficients alpha_0..alpha_i, beta_0..beta_i, gamma_0..gamma_i (the
    lists may be longer; only indices 0..i are read) to alpha_{i+1},
    beta_{i+1}, gamma_{i+1}.  Returns (alpha_{i+1}, beta_{i+1}, gamma_{i+1},
    s1_i, s2_i) with the two rounded Cauchy-product sums."""
    p = ctx.p
    s1 = round_sum(cauchy_terms(a, g, i), p)
    s2 = round_sum(cauchy_terms(a, b, i), p)
    return tails(ctx, a, b, g, i, s1, s2) + (s1, s2)


def tails(ctx: Context, a: Sequence[BF], b: Sequence[BF], g: Sequence[BF], i: int,
          s1: BF, s2: BF):
    """alpha_{i+1}, beta_{i+1}, gamma_{i+1} of equation (3) from the
    coefficients of index i and the rounded Cauchy sums s1_i, s2_i: each
    numerator exact, divided by i+1 with one rounding."""
    p = ctx.p
    d = i + 1
    num_a = exact_sum([neg(exact_mul(ctx.sigma, a[i])), exact_mul(ctx.sigma, b[i])])
    num_b = exact_sum([exact_mul(ctx.R, a[i]), neg(exact(b[i])), neg(exact(s1))])
    num_g = exact_sum([exact(s2), neg(exact_mul(ctx.b, g[i]))])
    return (div_round(num_a, d, p), div_round(num_b, d, p), div_round(num_g, d, p))


def coefficients(ctx: Context, state: Tuple[BF, BF, BF]):
    """Taylor coefficients alpha, beta, gamma (lists of N+1 BF) and the
    rounded Cauchy sums s1, s2 (lists of N) for one step from `state`
    (equation (3); the i=0 case gives the first-coefficient formulas)."""
    a: List[BF] = [state[0]]
    b: List[BF] = [state[1]]
    g: List[BF] = [state[2]]
    s1s: List[BF] = []
    s2s: List[BF] = []
    for i in range(ctx.N):
        an, bn, gn, s1, s2 = next_coefficients(ctx, a, b, g, i)
        s1s.append(s1)
        s2s.append(s2)
        a.append(an)
        b.append(bn)
        g.append(gn)
    return a, b, g, s1s, s2s


def horner(ctx: Context, c: Sequence[BF]) -> BF:
    """h = c_N; for i = N-1..0: h = round(h*tau + c_i).  This is the series
    of equation (2) (c_0 = x_n) evaluated by Horner's rule."""
    p = ctx.p
    h = c[ctx.N]
    for i in range(ctx.N - 1, -1, -1):
        h = round_sum([exact_mul(h, ctx.tau), exact(c[i])], p)
    return h


def step(ctx: Context, state: Tuple[BF, BF, BF]) -> Tuple[BF, BF, BF]:
    """One Taylor step (equation (2)) from `state`."""
    a, b, g, _, _ = coefficients(ctx, state)
    return (horner(ctx, a), horner(ctx, b), horner(ctx, g))


def integrate(ctx: Context, state: Tuple[BF, BF, BF], nsteps: int,
              keep_states: bool = False):
    """`nsteps` Taylor steps.  Returns the final state, and with
    keep_states=True also the list of all states s_0..s_nsteps."""
    states = [state] if keep_states else None
    s = state
    for _ in range(nsteps):
        s = step(ctx, s)
        if keep_states:
            states.append(s)
    return (s, states) if keep_states else s
