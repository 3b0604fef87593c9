"""Resumable long runs (GPU): a run stopped after a segment and resumed from
its state file is bit-identical to an uninterrupted run and to the oracle;
the lockstep verification rerun records the agreement per segment."""
import json
import os
import sys

import pytest

from oracle import lorenz as lz
from workloads import BENCH_X0

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_stop_and_resume_is_bit_exact(gpu_lib, tmp_path):
    from paper_1908_09301_amd.longrun import LongRun
    say("longrun resume K=100 N=40")
    a = LongRun(str(tmp_path / "a.json"), N=40, K=100)
    assert a.advance(60, 20) == 60
    b = LongRun(str(tmp_path / "b.json"), N=40, K=100)
    assert b.advance(30, 10) == 30
    del b
    # a new process would construct it the same way: from the file alone
    b2 = LongRun(str(tmp_path / "b.json"), N=0)
    assert b2.step == 30
    assert b2.advance(60, 15) == 60
    assert b2.state() == a.state()
    ctx = lz.make_context(K_digits=100, N=40)
    ref = lz.integrate(ctx, lz.state_from_strings(ctx, BENCH_X0), 60)
    assert a.state() == [tuple(v) for v in ref]
    meta = json.load(open(tmp_path / "b.json"))
    assert [s["to_step"] for s in meta["segments"]] == [10, 20, 30, 45, 60]


def test_verification_rerun_in_lockstep(gpu_lib, tmp_path):
    from paper_1908_09301_amd.longrun import LongRun
    say("longrun verify K=100 N=40 vs 125/50")
    r = LongRun(str(tmp_path / "v.json"), N=40, K=100, verify=(125, 50))
    assert r.advance(200, 50) == 200
    segs = r.meta["segments"]
    assert len(segs) == 4
    # rerun criterion: at least min(0.98 K, 1.1 N) - 0.40 t - 3 digits
    for s in segs:
        t = s["to_step"] * 0.01
        assert s["agreement_digits"] >= min(98.0, 44.0) - 0.40 * t - 3, s
    assert os.path.exists(tmp_path / "v.json")
