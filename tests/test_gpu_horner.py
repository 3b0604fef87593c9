"""The Horner sum of equation (2) for step sizes n/d with small n and d,
where each step round(tau h + c) is computed as the exact numerator
n h + r 2^E h + d c divided by d (d tau_p = n + r 2^E exactly), against the
oracle and against the full p x p-bit product (MPTS_TAU=product), bit for
bit (GPU)."""
import os
import sys

import pytest

from oracle import lorenz as lz
from oracle.adjoint import grad_sqnorm
from workloads import BENCH_X0, box_state, double_strings

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make(gpu_lib, path, **kw):
    """A context whose Horner steps use the short division ("rational") or
    the full product ("product")."""
    old = os.environ.get("MPTS_TAU")
    try:
        if path == "product":
            os.environ["MPTS_TAU"] = "product"
        else:
            os.environ.pop("MPTS_TAU", None)
        return gpu_lib.Lorenz(**kw)
    finally:
        if old is None:
            os.environ.pop("MPTS_TAU", None)
        else:
            os.environ["MPTS_TAU"] = old


# step sizes: the paper's 1/100, negative, other periodic binary expansions
# (rounded up and down), an exact power of two (r = 0), a reducible decimal
# (5/1000), a numerator above 1, and one beyond the short-division limits
# (full product)
TAUS = ["1/100", "-1/100", "1/300", "1/120", "3/1000", "1/128", "5e-3", "7/4096",
        "-0.0123456789012345678901"]


@pytest.mark.parametrize("tau", TAUS)
@pytest.mark.parametrize("L,N,wgs", [(4, 20, 1), (13, 30, 5)])
def test_horner_matches_oracle(gpu_lib, tau, L, N, wgs):
    say("horner", tau, L, N, wgs)
    ctx = lz.make_context(L=L, N=N, tau=tau)
    x0 = lz.state_from_strings(ctx, BENCH_X0)
    ref = lz.integrate(ctx, x0, 3)
    p = make(gpu_lib, "rational", L=L, N=N, tau=tau)
    p.set_schedule(wgs)
    assert p.integrate([tuple(v) for v in x0], 3) == [tuple(v) for v in ref]


def test_horner_zero_rows_match_oracle(gpu_lib):
    """A zero accumulator and zero addends (x = y = 0 stays on the z axis)."""
    ctx = lz.make_context(L=6, N=12)
    x0 = lz.state_from_strings(ctx, ("0", "0", "3.5"))
    ref = lz.integrate(ctx, x0, 4)
    for wgs in (1, 4):
        p = make(gpu_lib, "rational", L=6, N=12)
        p.set_schedule(wgs)
        assert p.integrate([tuple(v) for v in x0], 4) == [tuple(v) for v in ref], wgs


@pytest.mark.parametrize("L,N,wgs,steps", [(84, 120, 16, 3), (208, 300, 256, 2), (416, 200, 256, 2)])
def test_horner_division_and_product_give_the_same_bits(gpu_lib, L, N, wgs, steps):
    say("horner rational vs product", L, N, wgs, steps)
    out = []
    for path in ("rational", "product"):
        p = make(gpu_lib, path, L=L, N=N)
        p.set_schedule(wgs)
        out.append(p.integrate([p.from_str(v) for v in BENCH_X0], steps))
    assert out[0] == out[1]


@pytest.mark.parametrize("tau", ["1/100", "-1/300"])
def test_adjoint_powers_of_tau_match_oracle(gpu_lib, tau):
    """The adjoint's powers tau^i (the same short division, no addend)."""
    say("adjoint tau powers", tau)
    ctx = lz.make_context(L=8, N=16, tau=tau)
    x0 = lz.state_from_strings(ctx, double_strings(box_state(7)))
    xT, ref = grad_sqnorm(ctx, x0, 3)
    p = make(gpu_lib, "rational", L=8, N=16, tau=tau)
    p.set_schedule(4)
    _, gbf, fin, _ = p.grad([tuple(v) for v in x0], 3)
    assert fin == [tuple(v) for v in xT]
    assert gbf == [tuple(v) for v in ref]
