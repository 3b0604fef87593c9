"""Taylor series method for polynomial vector fields of degree at most two.

Test infrastructure: a slow, exact reference for the parity tests of the GPU
path, never called by it.

The paper derives its recursion for the Lorenz system and notes (Section 2,
the paragraph on automatic differentiation; Section 6) that any right-hand
side built from sums and products gives sums of the same kind as
equation (3): the Taylor coefficients of a product of two series are its
Cauchy-product sums.  This module applies that to systems

    dx_v/dt = c_v + sum_u A_vu x_u + sum_{u <= w} B_vuw x_u x_w,  v = 0..V-1

given as a list of terms (equation v, coefficient, and zero, one or two
variables).  With x_{v,0} the current state, for i = 0..N-1:

    S^{uw}_i  = sum_{k=0}^{i} x_{u,i-k} x_{w,k}          (each distinct pair u <= w)
    x_{v,i+1} = ([i = 0] c_v + sum_u A_vu x_{u,i} + sum B_vuw S^{uw}_i) / (i+1)

and the step is equation (2), evaluated by Horner's rule.

Rounding points (one RNE rounding to p bits each), as for the Lorenz
system: each Cauchy sum S^{uw}_i (exact sum of exact products); each new
coefficient (exact numerator, divided by i+1); each Horner step
h <- h*tau + c_i.  The coefficients and the step are p-bit numbers (each
rounded once from its exact decimal or rational text).  With the Lorenz
terms this is exactly the recursion of the Lorenz module: sigma (y - x)
splits into sigma y and -sigma x (exact products, the same exact sum),
-x z and x y are the sums s1 and s2 with coefficients -1 and 1.
"""
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

from .bigfloat import BF, div_round, exact, exact_mul, exact_sum, parse, round_sum


@dataclass(frozen=True)
class Term:
    """coef * x_u * x_w in equation eq (u, w = -1: absent)."""
    eq: int
    coef: str
    u: int = -1
    w: int = -1


@dataclass
class Context:
    """A system of nvar equations, precision L limbs (p = 32 L) and order N."""
    nvar: int
    terms: Tuple[Term, ...]
    L: int
    N: int
    tau_text: str = "1/100"
    coefs: List[BF] = field(default=None)
    tau: BF = None
    pairs: List[Tuple[int, int]] = field(default=None)

    @property
    def p(self) -> int:
        return 32 * self.L

    def __post_init__(self):
        if self.L < 1 or self.N < 1 or self.nvar < 1:
            raise ValueError("L, N and nvar must be >= 1")
        for t in self.terms:
            if not 0 <= t.eq < self.nvar or not -1 <= t.u < self.nvar or not -1 <= t.w < self.nvar:
                raise ValueError(f"bad term {t}")
            if t.u < 0 and t.w >= 0:
                raise ValueError(f"bad term {t}")
        self.terms = tuple(self.terms)
        self.coefs = [parse(t.coef, self.p) for t in self.terms]
        self.tau = parse(self.tau_text, self.p)
        pairs = []
        for t in self.terms:
            if t.w >= 0:
                q = (min(t.u, t.w), max(t.u, t.w))
                if q not in pairs:
                    pairs.append(q)
        self.pairs = pairs


def make_context(nvar: int, terms: Sequence[Term], L: int, N: int, tau: str = "1/100") -> Context:
    return Context(nvar=nvar, terms=tuple(terms), L=L, N=N, tau_text=str(tau))


def cauchy_sum(ctx: Context, xs: Sequence[Sequence[BF]], u: int, w: int, i: int) -> BF:
    """S^{uw}_i = sum_{k=0}^i x_{u,i-k} x_{w,k}, rounded once."""
    return round_sum([exact_mul(xs[u][i - k], xs[w][k]) for k in range(i + 1)], ctx.p)


def next_coefficients(ctx: Context, xs: Sequence[Sequence[BF]], i: int):
    """From the coefficients of indices 0..i of every variable to those of
    index i+1 (returned as a list over the variables), with the rounded
    Cauchy sums of index i (a dict keyed by pair)."""
    sums = {q: cauchy_sum(ctx, xs, q[0], q[1], i) for q in ctx.pairs}
    out = []
    for v in range(ctx.nvar):
        num = []
        for t, c in zip(ctx.terms, ctx.coefs):
            if t.eq != v:
                continue
            if t.u < 0:
                if i == 0:
                    num.append(exact(c))          # the constant term: only in x_{v,1}
            elif t.w < 0:
                num.append(exact_mul(c, xs[t.u][i]))
            else:
                num.append(exact_mul(c, sums[(min(t.u, t.w), max(t.u, t.w))]))
        out.append(div_round(exact_sum(num), i + 1, ctx.p))
    return out, sums


def coefficients(ctx: Context, state: Sequence[BF]):
    """Taylor coefficients (nvar lists of N+1) and the rounded Cauchy sums
    (a list of N dicts) for one step from `state`."""
    xs: List[List[BF]] = [[s] for s in state]
    sums = []
    for i in range(ctx.N):
        new, s = next_coefficients(ctx, xs, i)
        sums.append(s)
        for v in range(ctx.nvar):
            xs[v].append(new[v])
    return xs, sums


def horner(ctx: Context, c: Sequence[BF]) -> BF:
    """h = c_N; for i = N-1..0: h = round(h*tau + c_i) (equation (2))."""
    h = c[ctx.N]
    for i in range(ctx.N - 1, -1, -1):
        h = round_sum([exact_mul(h, ctx.tau), exact(c[i])], ctx.p)
    return h


def step(ctx: Context, state: Sequence[BF]) -> Tuple[BF, ...]:
    xs, _ = coefficients(ctx, state)
    return tuple(horner(ctx, xs[v]) for v in range(ctx.nvar))


def integrate(ctx: Context, state: Sequence[BF], nsteps: int) -> Tuple[BF, ...]:
    s = tuple(state)
    for _ in range(nsteps):
        s = step(ctx, s)
    return s
