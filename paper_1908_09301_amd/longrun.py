"""Resumable long runs on the library (paper, Section 5: the interval
[0, 5000] at N = 2000 and 8000 bits, about 9 days 14 hours on 28 cores).

A long run is a sequence of segments of the device-resident integration
(mpts_integrate_dev); after every segment the exact p-bit state and the step
count go to a JSON state file (written to a temporary name and renamed, so a
run killed at any moment leaves the last complete segment), and a later call
resumes from it.  Because a Taylor step is a pure function of the p-bit
state, a resumed run is bit-identical to an uninterrupted one.  With a
verification precision the rerun of the paper's procedure (larger K and N)
advances in lockstep in the same batched launch, and the agreement of the
two runs is recorded per segment.

    python -m paper_1908_09301_amd.longrun --bits 8000 --N 2000 --T 5000 \\
        --segment 200 --state run.json --budget-s 600
"""
import argparse
import json
import math
import os
import sys
import time
from typing import List, Optional, Sequence

from . import cns, mpts


def _enc(v):
    s, m, e = v
    return [s, format(m, "x"), e]


def _dec(v):
    s, mh, e = v
    return (int(s), int(mh, 16), int(e))


class LongRun:
    """One trajectory (and optionally its verification rerun) advanced in
    segments with its state persisted after each."""

    def __init__(self, path: str, N: int, K: Optional[int] = None, L: Optional[int] = None,
                 x0: Sequence[str] = ("-15.8", "-17.48", "35.64"), tau: str = "1/100",
                 verify: Optional[Sequence[int]] = None):
        self.path = path
        if os.path.exists(path):
            with open(path) as f:
                self.meta = json.load(f)
        else:
            self.meta = {"N": N, "K": K, "L": L, "tau": tau, "x0": list(x0), "step": 0,
                         "verify": list(verify) if verify else None, "segments": []}
        m = self.meta
        self.prob = mpts.Lorenz(K=m["K"], N=m["N"], L=m["L"], tau=m["tau"])
        self.ref = None
        if m["verify"]:
            K2, N2 = m["verify"]
            self.ref = mpts.Lorenz(K=K2, N=N2, tau=m["tau"])
        if "state" not in m:
            m["state"] = [_enc(self.prob.from_str(s)) for s in m["x0"]]
            if self.ref is not None:
                m["ref_state"] = [_enc(self.ref.from_str(s)) for s in m["x0"]]

    @property
    def step(self) -> int:
        return self.meta["step"]

    def state(self):
        return [_dec(v) for v in self.meta["state"]]

    def _save(self):
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.meta, f)
        os.replace(tmp, self.path)

    def advance(self, to_step: int, segment: int, budget_s: float = float("inf")) -> int:
        """Run segments until step `to_step` or until the wall-clock budget
        is spent (after a whole segment); returns the step reached."""
        import torch
        m = self.meta
        t_start = time.perf_counter()
        ws = self.prob.workspace(segment)
        while m["step"] < to_step and time.perf_counter() - t_start < budget_s:
            n = min(segment, to_step - m["step"])
            t0 = time.perf_counter()
            if self.ref is None:
                x = self.prob.pack_state(self.state()).cuda()
                out = torch.empty_like(x)
                self.prob.integrate_dev(x, n, out, ws=ws)
                self.prob.check(ws)
                new = self.prob.unpack_state(out)
                rec = {"steps": n}
            else:
                cur = [self.state(), [_dec(v) for v in m["ref_state"]]]
                new, ref_new = mpts.integrate_batch([self.prob, self.ref], cur, [n, n],
                                                    flags=mpts.MPTS_GRAPH)
                m["ref_state"] = [_enc(v) for v in ref_new]
                rec = {"steps": n,
                       "agreement_digits": round(cns.agreement_digits(
                           new, ref_new, cns.digits_of(self.ref)), 3)}
            dt = time.perf_counter() - t0
            m["state"] = [_enc(v) for v in new]
            m["step"] += n
            rec.update({"to_step": m["step"], "seconds": round(dt, 4), "steps_per_s": n / dt})
            m["segments"].append(rec)
            self._save()
        return m["step"]


def main(argv: Optional[List[str]] = None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--state", required=True, help="JSON state file (created or resumed)")
    ap.add_argument("--N", type=int, required=True)
    ap.add_argument("--K", type=int, default=None, help="decimal digits")
    ap.add_argument("--bits", type=int, default=None, help="precision in bits (multiple of 32)")
    ap.add_argument("--T", type=float, required=True, help="end of the interval [0, T]")
    ap.add_argument("--tau", default="1/100")
    ap.add_argument("--segment", type=int, default=100)
    ap.add_argument("--budget-s", type=float, default=float("inf"))
    ap.add_argument("--verify", type=str, default=None, help="rerun precision K,N")
    ap.add_argument("--x0", type=str, default="-15.8,-17.48,35.64")
    a = ap.parse_args(argv)
    L = None if a.bits is None else math.ceil(a.bits / 32)
    verify = [int(t) for t in a.verify.split(",")] if a.verify else None
    run = LongRun(a.state, a.N, K=a.K, L=L, x0=a.x0.split(","), tau=a.tau, verify=verify)
    from fractions import Fraction
    steps = int(Fraction(str(a.T)) / Fraction(a.tau))
    reached = run.advance(steps, a.segment, a.budget_s)
    segs = run.meta["segments"]
    rate = segs[-1]["steps_per_s"] if segs else None
    print(json.dumps({"state": a.state, "step": reached, "of": steps, "last_steps_per_s": rate,
                      "remaining_s_at_last_rate": (steps - reached) / rate if rate else None}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
