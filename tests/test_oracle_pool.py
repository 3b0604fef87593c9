"""The fan-out of oracle checks used by the whole-run GPU parity tests
(CPU): it must accept the oracle's own trajectory and catch a one-bit change
in a checkpoint, a coefficient and a final state."""
import os

import pytest

import oracle_pool as op
from oracle import lorenz as lz
from workloads import BENCH_X0


@pytest.fixture(scope="module")
def pool():
    p = op.make_pool(4)
    yield p
    p.shutdown()


def flip(v):
    s, m, e = v
    return (s, m ^ 1, e)


def test_step_checks_find_a_flipped_bit(pool):
    ctx = lz.make_context(K_digits=100, N=20)
    x0 = lz.state_from_strings(ctx, BENCH_X0)
    _, st = lz.integrate(ctx, x0, 12, keep_states=True)
    st = [[tuple(v) for v in s] for s in st]
    assert [f.result() for f in [pool.submit(op.step_task, ctx.L, 20, n, st[n], st[n + 1])
                                 for n in range(12)]] == [None] * 12
    st[6][2] = flip(st[6][2])
    bad = [f.result() for f in [pool.submit(op.step_task, ctx.L, 20, n, st[n], st[n + 1])
                                for n in range(12)]]
    assert [n for n in bad if n is not None] == [5, 6]


def test_transition_and_horner_checks_find_a_flipped_bit(pool):
    ctx = lz.make_context(K_digits=60, N=25)
    x0 = lz.state_from_strings(ctx, BENCH_X0)
    a, b, g, _, _ = lz.coefficients(ctx, x0)
    nxt = lz.step(ctx, x0)
    coefs = [[tuple(v) for v in c] for c in (a, b, g)]
    path = op.store_coefficients(coefs)
    try:
        assert pool.submit(op.transitions_task, ctx.L, 25, path, list(range(25))).result() == []
        assert all(pool.submit(op.horner_task, ctx.L, 25, path, c, tuple(nxt[c])).result()
                   for c in range(3))
    finally:
        os.unlink(path)
    coefs[1][13] = flip(coefs[1][13])
    path = op.store_coefficients(coefs)
    try:
        bad = pool.submit(op.transitions_task, ctx.L, 25, path, list(range(25))).result()
        assert 12 in bad and 13 in bad
    finally:
        os.unlink(path)
    # the Horner sum only sees bits of the coefficients that survive the
    # powers of tau: change a high bit of beta_1
    coefs[1][13] = flip(coefs[1][13])
    s, m, e = coefs[1][1]
    coefs[1][1] = (s, m ^ (1 << (ctx.p - 30)), e)
    path = op.store_coefficients(coefs)
    try:
        assert not pool.submit(op.horner_task, ctx.L, 25, path, 1, tuple(nxt[1])).result()
        assert pool.submit(op.horner_task, ctx.L, 25, path, 0, tuple(nxt[0])).result()
    finally:
        os.unlink(path)
