"""Parity at the full sizes of the K=2000/N=600 and K=4000/N=3500
trajectories, where the oracle cannot redo whole steps in seconds: the
oracle recomputes sampled transitions from the GPU's own outputs.

 * coefficient i+1 of equation (3) from the GPU's coefficients 0..i
   (sampled i, including the first and the last);
 * the Horner sum of equation (2) of the GPU's coefficients, against the
   GPU's state after one step.
Because every GPU quantity is a deterministic function of the previous ones,
agreement of every sampled transition with the oracle on the same inputs is
the bit-exact parity of those transitions (GPU)."""
import sys

import pytest

from oracle import lorenz as lz
from oracle.bigfloat import BF, div_round, exact, exact_mul, exact_sum, round_sum
from workloads import BENCH_X0, box_state, double_strings

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def neg(x):
    return (-x[0], x[1])


def oracle_next(ctx, a, b, g, i):
    """(a_{i+1}, b_{i+1}, g_{i+1}) from coefficients 0..i (equation (3))."""
    p = ctx.p
    s1 = round_sum(lz.cauchy_terms(a, g, i), p)
    s2 = round_sum(lz.cauchy_terms(a, b, i), p)
    na = exact_sum([neg(exact_mul(ctx.sigma, a[i])), exact_mul(ctx.sigma, b[i])])
    nb = exact_sum([exact_mul(ctx.R, a[i]), neg(exact(b[i])), neg(exact(s1))])
    ng = exact_sum([exact(s2), neg(exact_mul(ctx.b, g[i]))])
    d = i + 1
    return div_round(na, d, p), div_round(nb, d, p), div_round(ng, d, p)


def check_size(gpu_lib, K, N, xs, samples):
    ctx = lz.make_context(K_digits=K, N=N)
    x0 = lz.state_from_strings(ctx, xs)
    p = gpu_lib.Lorenz(K=K, N=N)
    say("coefficients", K, N)
    ga, gb, gg = p.coefficients([tuple(v) for v in x0])
    assert (ga[0], gb[0], gg[0]) == tuple(tuple(v) for v in x0)
    a = [BF(*v) for v in ga]
    b = [BF(*v) for v in gb]
    g = [BF(*v) for v in gg]
    for i in samples:
        say("transition", i)
        ref = oracle_next(ctx, a, b, g, i)
        assert (tuple(ref[0]), tuple(ref[1]), tuple(ref[2])) == (ga[i + 1], gb[i + 1], gg[i + 1]), i
    say("horner")
    step = p.integrate([tuple(v) for v in x0], 1)
    assert step == [tuple(lz.horner(ctx, c)) for c in (a, b, g)]


def test_k2000_n600_sampled_transitions(gpu_lib):
    check_size(gpu_lib, 2000, 600, double_strings(box_state(2)), [0, 1, 2, 17, 299, 598, 599])


def test_k4000_n3500_sampled_transitions(gpu_lib):
    check_size(gpu_lib, 4000, 3500, BENCH_X0, [0, 1, 5, 1000, 3498, 3499])
