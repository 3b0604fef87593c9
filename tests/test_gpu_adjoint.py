"""The hand-written adjoint (reverse sweep over checkpoints) against the
oracle's adjoint, bit for bit, and against central differences of GPU
forward runs (GPU)."""
import sys
from fractions import Fraction

import pytest

from oracle import lorenz as lz
from oracle import adjoint as oad
from oracle.adjoint import grad_sqnorm
from oracle.bigfloat import to_double
from workloads import BENCH_X0, box_state, double_strings

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("L,N,nsteps,wgs", [(4, 6, 3, 0), (4, 6, 3, 1), (12, 40, 5, 0),
                                            (12, 40, 5, 7), (32, 90, 4, 0), (2, 1, 4, 0)])
def test_gradient_matches_oracle_adjoint(gpu_lib, L, N, nsteps, wgs):
    say("adjoint", L, N, nsteps, wgs)
    ctx = lz.make_context(L=L, N=N)
    x0 = lz.state_from_strings(ctx, double_strings(box_state(400)) if L == 32 else BENCH_X0)
    xT, ref = grad_sqnorm(ctx, x0, nsteps)
    p = gpu_lib.Lorenz(L=L, N=N)
    p.set_schedule(wgs)
    g64, gbf, fin, lv = p.grad([tuple(v) for v in x0], nsteps)
    assert fin == [tuple(v) for v in xT]
    assert gbf == [tuple(v) for v in ref]
    assert g64 == [to_double(v) for v in ref]
    assert lv == oad.loss_value("sqnorm", xT)


def test_gradient_matches_central_differences_of_gpu_runs(gpu_lib):
    """d||x(T)||^2 / d x0_j from GPU forward runs at x0 +- h, h = 2^-(p/3),
    to relative 10^-(K/2-10) at K = 100."""
    K, N, nsteps = 100, 20, 10
    p = gpu_lib.Lorenz(K=K, N=N)
    ctx = lz.make_context(K_digits=K, N=N)
    x0 = lz.state_from_strings(ctx, BENCH_X0)
    g64, gbf, _, _ = p.grad([tuple(v) for v in x0], nsteps)
    h = Fraction(1, 2 ** (ctx.p // 3))
    tol = Fraction(1, 10 ** (K // 2 - 10))

    def loss(state):
        fin = p.integrate([tuple(v) for v in state], nsteps)
        return sum((Fraction(s * m) * Fraction(2) ** e) ** 2 for (s, m, e) in fin)

    for j in range(3):
        xp, xm = list(x0), list(x0)
        xp[j] = lz.state_from_fractions(ctx, [x0[j].frac() + h] * 3)[0]
        xm[j] = lz.state_from_fractions(ctx, [x0[j].frac() - h] * 3)[0]
        fd = (loss(xp) - loss(xm)) / (2 * h)
        s, m, e = gbf[j]
        g = Fraction(s * m) * Fraction(2) ** e
        assert abs(g - fd) <= tol * abs(fd), j


def test_autograd_function_matches_grad(gpu_lib):
    import torch
    p = gpu_lib.Lorenz(K=100, N=20)
    x0 = torch.tensor([-15.8, -17.48, 35.64], dtype=torch.float64, requires_grad=True)
    params = torch.tensor([10.0, 28.0, p.to_double(p.param(2))], dtype=torch.float64,
                          requires_grad=True)
    fn = gpu_lib.LorenzSqNorm()
    loss = fn.apply(x0, params, p, 6)
    (3.0 * loss).backward()
    g64, _, fin, lv = p.grad([p.from_double(v) for v in (-15.8, -17.48, 35.64)], 6)
    assert loss.item() == lv
    assert x0.grad.tolist() == [3.0 * v for v in g64[:3]]
    assert params.grad.tolist() == [3.0 * v for v in g64[3:]]


@pytest.mark.parametrize("loss", ["x", "y", "z"])
def test_component_loss_matches_oracle_adjoint(gpu_lib, loss):
    """Gradient of one component of x(T) (a Jacobian row): seed the unit
    vector; bit-exact against the oracle's adjoint with the same seed."""
    L, N, nsteps = 12, 40, 4
    say("component loss", loss)
    ctx = lz.make_context(L=L, N=N)
    x0 = lz.state_from_strings(ctx, BENCH_X0)
    xT, ref = oad.grad(ctx, x0, nsteps, loss)
    p = gpu_lib.Lorenz(L=L, N=N)
    g64, gbf, fin, lv = p.grad([tuple(v) for v in x0], nsteps, loss)
    assert fin == [tuple(v) for v in xT]
    assert gbf == [tuple(v) for v in ref]
    assert lv == oad.loss_value(loss, xT)


def test_grad_batch_matches_oracle_and_single_calls(gpu_lib):
    """Uneven (K, N) trajectories in one forward and one reverse launch:
    each gradient and loss equals the oracle's and the single call's."""
    shapes = [(4, 6, 3), (12, 40, 5), (32, 90, 2), (12, 40, 1), (2, 1, 4)]
    probs, x0s, refs = [], [], []
    for t, (L, N, n) in enumerate(shapes):
        ctx = lz.make_context(L=L, N=N)
        x0 = lz.state_from_strings(ctx, double_strings(box_state(400 + t)))
        probs.append(gpu_lib.Lorenz(L=L, N=N))
        x0s.append([tuple(v) for v in x0])
        refs.append(oad.grad(ctx, x0, n, "sqnorm"))
    say("grad batch", len(shapes))
    g, lv, fin = gpu_lib.grad_batch(probs, x0s, [s[2] for s in shapes])
    for t in range(len(shapes)):
        xT, ref = refs[t]
        assert fin[t] == [tuple(v) for v in xT], t
        assert g[t] == [to_double(v) for v in ref], t
        assert lv[t] == oad.loss_value("sqnorm", xT), t
        g1, _, _, l1 = probs[t].grad(x0s[t], shapes[t][2])
        assert (g1, l1) == (g[t], lv[t]), t
