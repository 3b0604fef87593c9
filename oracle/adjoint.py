"""Reverse-mode derivative of the Taylor step (not part of the paper's method;
it differentiates the recursion of equation (3) and the series of equation (2)
as stated in Section 2).

For one step with coefficients a, b, g (alpha, beta, gamma) and incoming
adjoints X, Y, Z of the new state, the derivation treats every rounding as
the identity (the derivative of the exact map) and evaluates it in p-bit
arithmetic with one RNE rounding per quantity:

  Horner (equation (2)):  d x_{n+1} / d a_i = tau^i, so
      qx_0 = X,  qx_i = round(qx_{i-1} * tau),  i = 1..N     (same for y, z)
  Recursion (equation (3)), for m = N..0, with u_m, v_m, w_m the adjoints of
  the numerators of a_{m+1}, b_{m+1}, g_{m+1}:
      u_m = round(abar_{m+1} / (m+1)),  v_m = round(bbar_{m+1}/(m+1)),
      w_m = round(gbar_{m+1}/(m+1))                             (m <= N-1)
      abar_m = round( qx_m + [m<N](-sigma u_m + R v_m)
                      + sum_{j=m}^{N-1} (-v_j g_{j-m} + w_j b_{j-m}) )
      bbar_m = round( qy_m + [m<N]( sigma u_m - v_m)
                      + sum_{j=m}^{N-1} w_j a_{j-m} )
      gbar_m = round( qz_m + [m<N](-bpar w_m)
                      + sum_{j=m}^{N-1} (-v_j) a_{j-m} )
  (a_m enters s1_j and s2_j for j >= m with partners g_{j-m}, b_{j-m}; b_m
  and g_m enter s2_j and s1_j with partner a_{j-m}.)
  The new incoming adjoints are abar_0, bbar_0, gbar_0.
  Parameter derivatives of this step (exact sums):
      dsigma = sum_{i<N} u_i (b_i - a_i),  dR = sum_{i<N} v_i a_i,
      dbpar  = -sum_{i<N} w_i g_i
  and each running parameter adjoint is updated with one rounding per step:
      sigmabar <- round(sigmabar + dsigma)   (same for R, bpar).
"""
from fractions import Fraction
from typing import List, Tuple

from .bigfloat import (BF, ZERO, div_round, exact, exact_mul, exact_sum,
                       round_exact, round_sum, to_double)
from .lorenz import Context, coefficients, integrate, neg


def tau_powers(ctx: Context, seed: BF) -> List[BF]:
    """q_0 = seed, q_i = round(q_{i-1} * tau), i = 1..N."""
    q = [seed]
    for _ in range(ctx.N):
        q.append(round_exact(exact_mul(q[-1], ctx.tau), ctx.p))
    return q


def reverse_step(ctx: Context, state, bar):
    """Adjoint of one step.  `state` is the step's starting state, `bar` the
    adjoints (X, Y, Z) of its end state.  Returns the adjoints of the
    starting state and the exact parameter derivatives (X, e) pairs."""
    p, N = ctx.p, ctx.N
    a, b, g, _, _ = coefficients(ctx, state)
    qx = tau_powers(ctx, bar[0])
    qy = tau_powers(ctx, bar[1])
    qz = tau_powers(ctx, bar[2])
    abar: List[BF] = [ZERO] * (N + 1)
    bbar: List[BF] = [ZERO] * (N + 1)
    gbar: List[BF] = [ZERO] * (N + 1)
    u: List[BF] = [ZERO] * N
    v: List[BF] = [ZERO] * N
    w: List[BF] = [ZERO] * N
    for m in range(N, -1, -1):
        ta = [exact(qx[m])]
        tb = [exact(qy[m])]
        tg = [exact(qz[m])]
        if m < N:
            u[m] = div_round(exact(abar[m + 1]), m + 1, p)
            v[m] = div_round(exact(bbar[m + 1]), m + 1, p)
            w[m] = div_round(exact(gbar[m + 1]), m + 1, p)
            ta += [neg(exact_mul(ctx.sigma, u[m])), exact_mul(ctx.R, v[m])]
            tb += [exact_mul(ctx.sigma, u[m]), neg(exact(v[m]))]
            tg += [neg(exact_mul(ctx.b, w[m]))]
        for j in range(m, N):
            ta.append(neg(exact_mul(v[j], g[j - m])))
            ta.append(exact_mul(w[j], b[j - m]))
            tb.append(exact_mul(w[j], a[j - m]))
            tg.append(neg(exact_mul(v[j], a[j - m])))
        abar[m] = round_sum(ta, p)
        bbar[m] = round_sum(tb, p)
        gbar[m] = round_sum(tg, p)
    dsig = exact_sum([exact_mul(u[i], b[i]) for i in range(N)]
                     + [neg(exact_mul(u[i], a[i])) for i in range(N)])
    dR = exact_sum([exact_mul(v[i], a[i]) for i in range(N)])
    dbp = exact_sum([neg(exact_mul(w[i], g[i])) for i in range(N)])
    return (abar[0], bbar[0], gbar[0]), (dsig, dR, dbp)


# Losses of the final state x(T) = (x, y, z) whose gradient the reverse sweep
# computes, and the seed (the adjoint of x(T)) each one starts from:
#   "sqnorm": x^2 + y^2 + z^2, seed 2 x(T) (exact: an exponent increment);
#   "x", "y", "z": one component of x(T), seed the unit vector (exact).
LOSSES = ("sqnorm", "x", "y", "z")

ONE_BF = BF(1, 1, 0)


def loss_seed(loss: str, xT):
    """The exact adjoint of x(T) for `loss` (three BF values)."""
    if loss == "sqnorm":
        return tuple(BF(v.s, v.m, v.e + 1) if v.s else ZERO for v in xT)
    if loss in ("x", "y", "z"):
        j = "xyz".index(loss)
        return tuple(ONE_BF if c == j else ZERO for c in range(3))
    raise ValueError(f"unknown loss {loss!r}")


def loss_value(loss: str, xT) -> float:
    """The loss of x(T) computed exactly and rounded once to float64."""
    if loss == "sqnorm":
        tot = sum((v.frac() ** 2 for v in xT), Fraction(0))
        return tot.numerator / tot.denominator
    if loss in ("x", "y", "z"):
        return to_double(xT["xyz".index(loss)])
    raise ValueError(f"unknown loss {loss!r}")


def grad(ctx: Context, x0, nsteps: int, loss: str = "sqnorm", states=None):
    """Gradient of a loss of x(T), T = nsteps*tau, with respect to
    (x0, y0, z0, sigma, R, b), by a forward run with per-step checkpoints
    and a reverse sweep from the loss's exact seed.  Returns (final_state,
    grads) where grads is a list of 6 BF values."""
    p = ctx.p
    if states is None:
        _, states = integrate(ctx, x0, nsteps, keep_states=True)
    xT = states[nsteps]
    bar = loss_seed(loss, xT)
    psig, pR, pb = ZERO, ZERO, ZERO
    for n in range(nsteps - 1, -1, -1):
        bar, (dsig, dR, dbp) = reverse_step(ctx, states[n], bar)
        psig = round_sum([exact(psig), dsig], p)
        pR = round_sum([exact(pR), dR], p)
        pb = round_sum([exact(pb), dbp], p)
    return xT, [bar[0], bar[1], bar[2], psig, pR, pb]


def grad_sqnorm(ctx: Context, x0, nsteps: int, states=None):
    """Gradient of ||x(T)||^2 (the seed is the exact 2*x(T))."""
    return grad(ctx, x0, nsteps, "sqnorm", states)


def grad_sqnorm_fp64(ctx: Context, x0, nsteps: int):
    xT, g = grad_sqnorm(ctx, x0, nsteps)
    return xT, [to_double(v) for v in g]
