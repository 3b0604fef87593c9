"""The early Cauchy products on the int8 matrix cores (7-bit pieces, Toeplitz
blocks, i32 accumulators flushed into 64-bit columns) against the oracle and
against the VALU tile path, bit for bit (GPU).

MPTS_EARLY=valu or =mfma, read when a context is created, selects the
path; by default a context whose rows have at least 140 digits and fit the
matrix-core accumulators (at most 487 digits, L <= 425 limbs) uses the
matrix cores whenever its trajectory runs on two or more workgroups."""
import os
import sys

import pytest

from oracle import lorenz as lz
from workloads import BENCH_X0, box_state, double_strings

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make(gpu_lib, path, **kw):
    """A context on the given path: "early" (matrix cores for the early
    products) or "valu"."""
    keys = ("MPTS_EARLY",)
    old = {k: os.environ.get(k) for k in keys}
    try:
        for k in keys:
            os.environ.pop(k, None)
        os.environ["MPTS_EARLY"] = "valu" if path == "valu" else "mfma"
        return gpu_lib.Lorenz(**kw)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


# (L, N, workgroups): one output tile (L <= 84), two, three and four tiles
# (L = 208, 416, 425: the largest size the accumulators hold), one follower
# doing every term (G = 2: several accumulator flushes per index at L = 416),
# odd and XCD-sized groups
CASES = [(1, 9, 3), (4, 30, 7), (12, 40, 24), (22, 60, 16), (42, 70, 5), (84, 60, 33),
         (168, 50, 64), (208, 40, 256), (416, 30, 256), (425, 20, 100), (416, 150, 2)]


@pytest.mark.parametrize("L,N,wgs", CASES)
def test_mfma_coefficients_match_oracle(gpu_lib, L, N, wgs):
    say("mfma coefficients", L, N, wgs)
    ctx = lz.make_context(L=L, N=N)
    x0 = lz.state_from_strings(ctx, double_strings(box_state(20 + L)))
    a, b, g, _, _ = lz.coefficients(ctx, x0)
    p = make(gpu_lib, "early", L=L, N=N)
    p.set_schedule(wgs)
    ga, gb, gg = p.coefficients([tuple(v) for v in x0])
    for name, ref, got in (("alpha", a, ga), ("beta", b, gb), ("gamma", g, gg)):
        for i, (r, q) in enumerate(zip(ref, got)):
            assert tuple(r) == q, (name, i)


@pytest.mark.parametrize("L,N,wgs", [(416, 400, 256), (425, 300, 64)])
def test_mfma_and_valu_coefficients_agree(gpu_lib, L, N, wgs):
    say("mfma vs valu coefficients", L, N, wgs)
    out = []
    for path in ("early", "valu"):
        p = make(gpu_lib, path, L=L, N=N)
        p.set_schedule(wgs)
        out.append(p.coefficients([p.from_str(v) for v in BENCH_X0]))
    for c in range(3):
        for i, (a, b) in enumerate(zip(out[0][c], out[1][c])):
            assert a == b, (c, i)


@pytest.mark.parametrize("L,N,wgs,steps", [(12, 40, 7, 30), (84, 120, 64, 4), (208, 600, 256, 3),
                                           (416, 400, 256, 2)])
@pytest.mark.parametrize("path", ["early"])
def test_mfma_and_valu_paths_give_the_same_bits(gpu_lib, L, N, wgs, steps, path):
    say("mfma vs valu", path, L, N, wgs, steps)
    x0 = None
    out = []
    for path in (path, "valu"):
        p = make(gpu_lib, path, L=L, N=N)
        p.set_schedule(wgs)
        if x0 is None:
            x0 = [p.from_str(v) for v in BENCH_X0]
        out.append(p.integrate(x0, steps))
    assert out[0] == out[1]


def test_mfma_z_axis_and_spread_error(gpu_lib):
    """Zero rows (x = y = 0) on the matrix-core path, and a spread beyond the
    device window still reported as MPTS_ERANGE."""
    from oracle.bigfloat import ZERO
    ctx = lz.make_context(L=12, N=40)
    x0 = (ZERO, ZERO, lz.state_from_strings(ctx, ("0", "0", "35.64"))[2])
    ref = lz.integrate(ctx, x0, 5)
    p = make(gpu_lib, "early", L=12, N=40)
    p.set_schedule(16)
    assert p.integrate([tuple(v) for v in x0], 5) == [tuple(v) for v in ref]
    q = make(gpu_lib, "early", L=4, N=4)
    q.set_schedule(9)
    bad = lz.state_from_strings(lz.make_context(L=4, N=4), ("1e-300", "1", "1"))
    with pytest.raises(gpu_lib.MptsError) as ei:
        q.integrate([tuple(v) for v in bad], 1)
    assert ei.value.code == gpu_lib.MPTS_ERANGE
