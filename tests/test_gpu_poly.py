"""Polynomial vector fields of degree two on the GPU (k_poly, one workgroup
per trajectory) against the oracle (oracle/poly.py), bit for bit: the Taylor
coefficients of a step, whole steps of batches, the short-division and the
full-product Horner paths, and the Lorenz terms against the Lorenz kernel."""
import os
import sys

import pytest

from oracle import poly
from oracle.bigfloat import parse
from workloads import POLY_ENSEMBLE, POLY_SYSTEMS, POLY_X0, poly_states

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_ctx(name, L, N, tau="1/100"):
    nvar, terms = POLY_SYSTEMS[name]
    return poly.make_context(nvar, [poly.Term(*t) for t in terms], L=L, N=N, tau=tau)


def gpu_system(gpu_lib, name, L, N, tau="1/100", product=False):
    nvar, terms = POLY_SYSTEMS[name]
    old = os.environ.get("MPTS_TAU")
    try:
        if product:
            os.environ["MPTS_TAU"] = "product"
        else:
            os.environ.pop("MPTS_TAU", None)
        return gpu_lib.Poly(nvar, terms, L=L, N=N, tau=tau)
    finally:
        if old is None:
            os.environ.pop("MPTS_TAU", None)
        else:
            os.environ["MPTS_TAU"] = old


def state(ctx, texts):
    return tuple(parse(t, ctx.p) for t in texts)


@pytest.mark.parametrize("name", sorted(POLY_SYSTEMS))
@pytest.mark.parametrize("L,N", [(2, 12), (9, 30)])
def test_coefficients_match_oracle(gpu_lib, name, L, N):
    say("poly coefficients", name, L, N)
    ctx = oracle_ctx(name, L, N)
    x0 = state(ctx, POLY_X0[name])
    ref, _ = poly.coefficients(ctx, x0)
    got = gpu_system(gpu_lib, name, L, N).coefficients([tuple(v) for v in x0])
    for v in range(ctx.nvar):
        for i in range(N + 1):
            assert got[v][i] == tuple(ref[v][i]), (name, v, i)


@pytest.mark.parametrize("name", ["rossler", "chen", "rossler4", "oscillator"])
@pytest.mark.parametrize("product", [False, True])
def test_batch_steps_match_oracle(gpu_lib, name, product):
    """Five trajectories, four steps, in one launch; both Horner paths."""
    L, N, steps = 4, 16, 4
    say("poly batch", name, product)
    ctx = oracle_ctx(name, L, N)
    x0s = [state(ctx, x) for x in poly_states(11, 5, name)]
    p = gpu_system(gpu_lib, name, L, N, product=product)
    got = p.integrate([[tuple(v) for v in x] for x in x0s], steps)
    for t, x in enumerate(x0s):
        assert got[t] == tuple(tuple(v) for v in poly.integrate(ctx, x, steps)), t


@pytest.mark.parametrize("tau", ["1/100", "-1/300", "1/128", "-0.0123456789012345678901"])
def test_step_sizes_match_oracle(gpu_lib, tau):
    """Rational step sizes (short division, with and without the r term)
    and one beyond its limits (full product)."""
    L, N = 5, 20
    say("poly tau", tau)
    ctx = oracle_ctx("chen", L, N, tau)
    x0 = state(ctx, POLY_X0["chen"])
    got = gpu_system(gpu_lib, "chen", L, N, tau).integrate([[tuple(v) for v in x0]], 3)
    assert got[0] == tuple(tuple(v) for v in poly.integrate(ctx, x0, 3))


def test_lorenz_terms_match_the_lorenz_kernel(gpu_lib):
    """The Lorenz system given as terms runs the same bits as the Lorenz
    kernel (k_run), at K=300 digits, N=90."""
    nvar, terms = POLY_SYSTEMS["lorenz"]
    lor = gpu_lib.Lorenz(L=32, N=90)
    x0 = [lor.from_str(v) for v in POLY_X0["lorenz"]]
    ref = lor.integrate(x0, 3)
    got = gpu_lib.Poly(nvar, terms, L=32, N=90).integrate([x0], 3)
    assert got[0] == tuple(ref)


def test_order_one_and_zero_state(gpu_lib):
    """N = 1 (explicit Euler) and a state with zero components (the z axis
    of the Lorenz terms stays on the axis)."""
    for name, x0t, N in (("rossler", POLY_X0["rossler"], 1), ("lorenz", ("0", "0", "7/2"), 12)):
        ctx = oracle_ctx(name, 3, N)
        x0 = state(ctx, x0t)
        got = gpu_system(gpu_lib, name, 3, N).integrate([[tuple(v) for v in x0]], 3)
        assert got[0] == tuple(tuple(v) for v in poly.integrate(ctx, x0, 3)), name


def test_ensemble_samples_match_oracle(gpu_lib):
    """The Roessler ensemble workload (K=300, N=90) in one launch; three of
    its trajectories checked against the oracle after two steps."""
    E = POLY_ENSEMBLE
    p = gpu_lib.Poly(*POLY_SYSTEMS[E["system"]], K=E["K"], N=E["N"])
    ctx = oracle_ctx(E["system"], p.L, E["N"])
    x0s = [state(ctx, x) for x in poly_states(E["seed"], E["count"], E["system"])]
    say("poly ensemble", p.L, E["N"], len(x0s))
    got = p.integrate([[tuple(v) for v in x] for x in x0s], 2)
    for t in (0, 31, E["count"] - 1):
        assert got[t] == tuple(tuple(v) for v in poly.integrate(ctx, x0s[t], 2)), t
