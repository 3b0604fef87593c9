"""Pins of the oracle's reverse-mode derivative (CPU only).

  * exact forward-mode tangents (dual numbers in Fractions) of one
    unrounded step give the Jacobian the reverse sweep must reproduce;
  * central differences of whole runs of the oracle's forward map agree with
    the run gradient to relative 10^-(K/2-10).
"""
from fractions import Fraction

import pytest

from oracle import lorenz as lz
from oracle.adjoint import grad_sqnorm, reverse_step
from oracle.bigfloat import BF, ZERO, parse, exact
from workloads import BENCH_X0, box_state, double_strings


class Dual:
    """value + sum_j d[j] eps_j, exact rationals, 6 tangent directions."""
    __slots__ = ("v", "d")

    def __init__(self, v, d=None):
        self.v = Fraction(v)
        self.d = list(d) if d is not None else [Fraction(0)] * 6

    def __add__(self, o):
        o = o if isinstance(o, Dual) else Dual(o)
        return Dual(self.v + o.v, [a + b for a, b in zip(self.d, o.d)])

    __radd__ = __add__

    def __neg__(self):
        return Dual(-self.v, [-a for a in self.d])

    def __sub__(self, o):
        return self + (-(o if isinstance(o, Dual) else Dual(o)))

    def __rsub__(self, o):
        return Dual(o) - self

    def __mul__(self, o):
        o = o if isinstance(o, Dual) else Dual(o)
        return Dual(self.v * o.v, [self.v * b + o.v * a for a, b in zip(self.d, o.d)])

    __rmul__ = __mul__

    def __truediv__(self, k):
        return Dual(self.v / k, [a / k for a in self.d])


def seed(v, j):
    d = [Fraction(0)] * 6
    d[j] = Fraction(1)
    return Dual(v, d)


def exact_step_tangent(x, y, z, sigma, R, b, tau, N):
    """One unrounded step (equations (2)-(3)) in dual numbers."""
    A, B, G = [x], [y], [z]
    for i in range(N):
        s1 = sum((A[i - k] * G[k] for k in range(i + 1)), Dual(0))
        s2 = sum((A[i - k] * B[k] for k in range(i + 1)), Dual(0))
        A.append((sigma * B[i] - sigma * A[i]) / (i + 1))
        B.append((R * A[i] - B[i] - s1) / (i + 1))
        G.append((s2 - b * G[i]) / (i + 1))
    out = []
    for c in (A, B, G):
        h = c[N]
        for i in range(N - 1, -1, -1):
            h = h * tau + c[i]
        out.append(h)
    return out


@pytest.mark.parametrize("N", [1, 2, 4])
def test_reverse_step_matches_exact_forward_tangents(N):
    ctx = lz.make_context(L=6, N=N)
    p = ctx.p
    st = lz.state_from_strings(ctx, BENCH_X0)
    x, y, z = (seed(v.frac(), j) for j, v in enumerate(st))
    sig, R, b = seed(ctx.sigma.frac(), 3), seed(ctx.R.frac(), 4), seed(ctx.b.frac(), 5)
    out = exact_step_tangent(x, y, z, sig, R, b, ctx.tau.frac(), N)
    for row in range(3):
        bar = [ZERO, ZERO, ZERO]
        bar[row] = parse("1", p)
        (gx, gy, gz), (ds, dR, db) = reverse_step(ctx, st, tuple(bar))
        got = [gx.frac(), gy.frac(), gz.frac()] + \
              [Fraction(X) * Fraction(2) ** e for X, e in (ds, dR, db)]
        ref = out[row].d
        scale = max(abs(r) for r in ref)
        for g_, r_ in zip(got, ref):
            assert abs(g_ - r_) <= scale * Fraction(1, 2 ** (p - 20)), (row, N)


def _loss(ctx, x0):
    s = lz.integrate(ctx, x0, _loss.nsteps)
    return sum(v.frac() ** 2 for v in s)


@pytest.mark.parametrize("K,N,nsteps", [(100, 10, 12)])
def test_run_gradient_matches_central_differences(K, N, nsteps):
    ctx = lz.make_context(K_digits=K, N=N)
    p = ctx.p
    x0 = lz.state_from_strings(ctx, double_strings(box_state(400)))
    _, grads = grad_sqnorm(ctx, x0, nsteps)
    _loss.nsteps = nsteps
    h = Fraction(1, 2 ** (p // 3))
    tol = Fraction(1, 10 ** (K // 2 - 10))
    # initial state
    for j in range(3):
        xp = list(x0)
        xm = list(x0)
        xp[j] = lz.state_from_fractions(ctx, [x0[j].frac() + h] * 3)[0]
        xm[j] = lz.state_from_fractions(ctx, [x0[j].frac() - h] * 3)[0]
        fd = (_loss(ctx, tuple(xp)) - _loss(ctx, tuple(xm))) / (2 * h)
        assert abs(grads[j].frac() - fd) <= tol * abs(fd), j
    # parameters sigma, R, b (the b derivative is taken at the rounded b)
    for j, name in ((3, "sigma"), (4, "R"), (5, "b")):
        base = getattr(ctx, name).frac()
        kw = dict(L=ctx.L, N=N, sigma=str(ctx.sigma.frac()), R=str(ctx.R.frac()), b=str(ctx.b.frac()))
        kw[name] = str(base + h)
        cp = lz.make_context(**kw)
        kw[name] = str(base - h)
        cm = lz.make_context(**kw)
        assert getattr(cp, name).frac() == base + h
        fd = (_loss(cp, x0) - _loss(cm, x0)) / (2 * h)
        assert abs(grads[j].frac() - fd) <= tol * abs(fd), name
