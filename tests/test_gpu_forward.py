"""Parity of the HIP forward path with the oracle, bit for bit (GPU).

Every comparison is on raw (sign, mantissa, exponent) triples: the device
computes each Cauchy sum exactly and rounds once, so the result cannot depend
on how the kernel splits or orders the reduction, and any difference is a
defect.
"""
import sys

import pytest

from oracle import lorenz as lz
from oracle.bigfloat import BF, ZERO
from workloads import BENCH_X0, box_state, double_strings

pytestmark = pytest.mark.gpu


def T(v):
    return tuple(v)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("L,N,ic", [(2, 6, "bench"), (12, 40, "bench"), (5, 17, 11), (12, 40, 12),
                                    (22, 60, 13), (1, 9, 14)])
def test_coefficients_match_oracle(gpu_lib, L, N, ic):
    say("coefficients", L, N, ic)
    ctx = lz.make_context(L=L, N=N)
    xs = BENCH_X0 if ic == "bench" else double_strings(box_state(ic))
    x0 = lz.state_from_strings(ctx, xs)
    a, b, g, _, _ = lz.coefficients(ctx, x0)
    p = gpu_lib.Lorenz(L=L, N=N)
    ga, gb, gg = p.coefficients([T(v) for v in x0])
    for name, ref, got in (("alpha", a, ga), ("beta", b, gb), ("gamma", g, gg)):
        for i, (r, q) in enumerate(zip(ref, got)):
            assert T(r) == q, (name, i)


@pytest.mark.parametrize("wgs", [0, 1, 7, 256])
def test_z_axis_zero_terms(gpu_lib, wgs):
    """x0 = y0 = 0: every coefficient of x and y is an exact zero (zero rows
    in the Cauchy sums and in the single products), on one workgroup and on
    groups that split the products."""
    say("z axis", wgs)
    ctx = lz.make_context(L=12, N=40)
    x0 = (ZERO, ZERO, lz.state_from_strings(ctx, ("0", "0", "35.64"))[2])
    ref = lz.integrate(ctx, x0, 20)
    p = gpu_lib.Lorenz(L=12, N=40)
    p.set_schedule(wgs)
    got = p.integrate([T(v) for v in x0], 20)
    assert [T(v) for v in ref] == got
    assert got[0] == (0, 0, 0) and got[1] == (0, 0, 0)


@pytest.mark.parametrize("wgs", [1, 2, 3, 7, 16, 24, 256, 0])
def test_schedule_does_not_change_bits(gpu_lib, wgs):
    """Any number of workgroups per trajectory gives the same bits: one
    workgroup (every frame in LDS), a leader with one follower, Horner
    chains on three workgroups, odd counts, the split into eight term
    groups at its smallest (16, 24) and with every CU (256), and the
    automatic choice (0)."""
    say("schedule", wgs)
    ctx = lz.make_context(L=12, N=40)
    x0 = lz.state_from_strings(ctx, BENCH_X0)
    ref = lz.integrate(ctx, x0, 25)
    p = gpu_lib.Lorenz(L=12, N=40)
    p.set_schedule(wgs)
    assert p.integrate([T(v) for v in x0], 25) == [T(v) for v in ref]


def test_k100_n40_full_run_with_checkpoints(gpu_lib):
    """K=100 digits, N=40, tau=0.01, 1000 steps from (-15.8, -17.48, 35.64):
    the whole trajectory is bit-identical to the oracle."""
    say("k100 n40 1000 steps")
    ctx = lz.make_context(K_digits=100, N=40)
    x0 = lz.state_from_strings(ctx, BENCH_X0)
    ref_final, ref_states = lz.integrate(ctx, x0, 1000, keep_states=True)
    p = gpu_lib.Lorenz(K=100, N=40)
    final, states = p.integrate([T(v) for v in x0], 1000, checkpoints=True)
    assert final == [T(v) for v in ref_final]
    for n in range(0, 1001, 50):
        assert states[n] == [T(v) for v in ref_states[n]], n


def test_k100_n40_matches_stored_states(gpu_lib):
    """The K=100, N=40 trajectory against the stored oracle states of
    tests/golden (steps 0, 1, 2, 10, 50, 100), bit for bit."""
    from test_golden import load_states
    say("k100 n40 stored states")
    stored = load_states()
    ctx = lz.make_context(K_digits=100, N=40)
    x0 = lz.state_from_strings(ctx, BENCH_X0)
    last = max(n for n, _ in stored)
    p = gpu_lib.Lorenz(K=100, N=40)
    _, states = p.integrate([T(v) for v in x0], last, checkpoints=True)
    for (n, c), v in stored.items():
        assert tuple(states[n]["xyz".index(c)]) == v, (n, c)


def test_k2000_n600_transition(gpu_lib):
    """One step at K=2000 digits (208 limbs), N=600 from the seeded initial
    state, against the oracle."""
    say("k2000 n600 one step")
    ctx = lz.make_context(K_digits=2000, N=600)
    x0 = lz.state_from_strings(ctx, double_strings(box_state(2)))
    ref = lz.step(ctx, x0)
    p = gpu_lib.Lorenz(K=2000, N=600)
    assert p.integrate([T(v) for v in x0], 1) == [T(v) for v in ref]


@pytest.mark.parametrize("wgs", [0, 1, 7, 256])
def test_spread_beyond_window_is_reported(gpu_lib, wgs):
    """A sum whose terms differ by far more than the device window: the call
    fails with MPTS_ERANGE instead of returning an inexact value, on every
    schedule."""
    say("spread", wgs)
    p = gpu_lib.Lorenz(L=4, N=4)
    p.set_schedule(wgs)
    ctx = lz.make_context(L=4, N=4)
    x0 = lz.state_from_strings(ctx, ("1e-300", "1", "1"))
    with pytest.raises(gpu_lib.MptsError) as ei:
        p.integrate([T(v) for v in x0], 1)
    assert ei.value.code == gpu_lib.MPTS_ERANGE
