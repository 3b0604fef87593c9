"""The allocation-free entry point (mpts_integrate_dev_noalloc: workspace in
the library's own device array) against mpts_integrate_dev on a caller
workspace, bit for bit, on two calls in a row with the second smaller; and
the rejection of a size beyond the array (GPU)."""
import sys

import pytest

from oracle import lorenz as lz
from workloads import BENCH_X0, box_state, double_strings

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_both(gpu_lib, K, N, xs, nsteps, wgs=0):
    import torch
    p = gpu_lib.Lorenz(K=K, N=N)
    p.set_schedule(wgs)
    x0 = [p.from_str(v) for v in xs]
    x0_dev = p.pack_state(x0).cuda()
    # reference: caller workspace
    out_ref = torch.empty_like(x0_dev)
    ws = p.workspace(nsteps)
    p.integrate_dev(x0_dev, nsteps, out_ref, ws=ws)
    p.check(ws)
    # the library's scratch array, with checkpoints
    out = torch.full_like(x0_dev, -7)
    ck = torch.zeros((nsteps + 1) * x0_dev.numel(), dtype=torch.int32, device="cuda")
    p.integrate_dev_noalloc(x0_dev, nsteps, out, ck)
    p.check(None)
    torch.cuda.synchronize()
    return p, x0, out_ref.cpu(), out.cpu(), ck.cpu().view(nsteps + 1, -1)


def test_noalloc_matches_workspace_call_twice_second_smaller(gpu_lib):
    say("noalloc: K=2000 N=600 4 steps, then K=100 N=40 30 steps")
    p, x0, ref, got, ck = run_both(gpu_lib, 2000, 600, double_strings(box_state(2)), 4)
    assert got.tolist() == ref.tolist()
    assert ck[4].tolist() == ref.tolist()
    p2, x02, ref2, got2, ck2 = run_both(gpu_lib, 100, 40, BENCH_X0, 30, wgs=7)
    assert got2.tolist() == ref2.tolist()
    ctx = lz.make_context(K_digits=100, N=40)
    oracle = lz.integrate(ctx, lz.state_from_strings(ctx, BENCH_X0), 30)
    assert p2.unpack_state(got2) == [tuple(v) for v in oracle]
    assert p2.unpack_state(ck2[0]) == [tuple(v) for v in x02]


def test_noalloc_rejects_sizes_beyond_the_array(gpu_lib):
    import torch
    p = gpu_lib.Lorenz(L=512, N=8000)
    x0 = p.pack_state([p.from_str(v) for v in BENCH_X0]).cuda()
    out = torch.empty_like(x0)
    with pytest.raises(gpu_lib.MptsError) as ei:
        p.integrate_dev_noalloc(x0, 1, out)
    assert ei.value.code == gpu_lib.MPTS_ENOSPC
    assert "scratch array" in str(ei.value)
