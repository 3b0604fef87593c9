"""Clean numerical simulation on top of the library: verification by rerun
and critical-predictable-time sweeps (paper, Section 1).

The paper's procedure: a run with K decimal digits and Taylor order N is
trusted over an interval when a second run with larger K and N coincides
with it there; the critical predictable time T_c(K, N) is how long a run
stays reliable, and T_c-K / T_c-N diagrams choose K and N for a target
interval.  Here every run is the library's (mpts_integrate_batch: all the
(K, N) variants of a sweep and the reference share one persistent launch per
segment of steps), and the comparison is exact: the agreement of two p-bit
states is -log10 of the largest relative difference of their components,
computed on the exact values.

Definitions used here (the paper gives the procedure, not formulas):
  agreement(t)  = min over x, y, z of -log10(|u - v| / |v|) (v the reference
                  component; identical values agree to the reference's full
                  precision);
  T_c(K, N)     = the first checkpoint time at which agreement with the
                  reference falls below `digits` decimal digits (default 2,
                  a 1 % deviation), or None if it never does in the interval;
  rerun check   = agreement(t) >= min(0.98 K, 1.1 N) - 0.40 t - 3 at every
                  checkpoint, for the rerun at (ceil(1.25 K), ceil(1.25 N)):
                  the truncation of an order-N step leaves about 1.1 N
                  correct digits, K digits bound the rounding, and the
                  Lorenz flow loses about 0.40 digits per time unit.
"""
import argparse
import json
import math
import sys
from fractions import Fraction
from typing import Dict, List, Optional, Sequence, Tuple

from . import mpts

Value = Tuple[int, int, int]  # (sign, mantissa, exponent): sign * m * 2^e


def exact(v: Value) -> Fraction:
    s, m, e = v
    return Fraction(s * m) * (Fraction(2) ** e) if s else Fraction(0)


def agreement_digits(u: Sequence[Value], v: Sequence[Value], full: float) -> float:
    """Decimal digits to which state u agrees with the reference state v:
    min over components of -log10(|u_c - v_c| / |v_c|), capped at `full`
    (the reference's precision in digits; equal components agree fully)."""
    worst = full
    for a, b in zip(u, v):
        fa, fb = exact(a), exact(b)
        if fa == fb:
            continue
        if fb == 0:
            return 0.0 if fa != 0 else worst
        rel = abs(fa - fb) / abs(fb)
        # -log10 of an exact rational, from its numerator and denominator
        d = -(_log10_int(rel.numerator) - _log10_int(rel.denominator))
        worst = min(worst, d)
    return max(worst, 0.0)


def _log10_int(n: int) -> float:
    if n <= 0:
        raise ValueError("positive integer expected")
    b = n.bit_length()
    if b <= 1000:
        return math.log10(n)
    # scale into double range: log10(n) = log10(n >> s) + s log10(2)
    s = b - 1000
    return math.log10(n >> s) + s * math.log10(2.0)


def run_segments(problems: Sequence["mpts.Lorenz"], x0s, total_steps: int, every: int,
                 flags: int = mpts.MPTS_GRAPH | mpts.MPTS_AUTOTUNE):
    """All trajectories together in one batched launch per segment of `every`
    steps (the library's ensemble path), each segment starting from the exact
    final states of the last.  Returns the states at steps 0, every, 2 every,
    ... (a list per checkpoint, one state per trajectory)."""
    states = [list(x0s)]
    cur = list(x0s)
    done = 0
    while done < total_steps:
        n = min(every, total_steps - done)
        cur = mpts.integrate_batch(problems, cur, [n] * len(problems), flags=flags)
        done += n
        states.append(cur)
    return states


def digits_of(problem: "mpts.Lorenz") -> float:
    return problem.p * math.log10(2.0)


def tc_sweep(variants: Sequence[Tuple[int, int]], reference: Tuple[int, int], x0: Sequence[str],
             T: float, tau: float = 0.01, every: int = 10, digits: float = 2.0):
    """T_c of every (K, N) variant against the reference run, all in one
    batched launch per segment.  x0: exact decimal or rational strings, each
    rounded once at every run's own precision.  Returns a dict with the
    agreement curves and T_c per variant."""
    nsteps = int(round(T / tau))
    keys = list(variants) + [reference]
    probs = [mpts.Lorenz(K=K, N=N) for (K, N) in keys]
    x0s = [[p.from_str(s) for s in x0] for p in probs]
    states = run_segments(probs, x0s, nsteps, every)
    ref = len(keys) - 1
    out = {"reference": {"K": reference[0], "N": reference[1]}, "steps": nsteps, "tau": tau,
           "every": every, "threshold_digits": digits, "variants": []}
    times = [k * every * tau for k in range(len(states))]
    for v, (K, N) in enumerate(variants):
        curve = [agreement_digits(st[v], st[ref], digits_of(probs[ref])) for st in states]
        tc = next((t for t, a in zip(times, curve) if a < digits), None)
        out["variants"].append({"K": K, "N": N, "Tc": tc,
                                "agreement": [(round(t, 6), round(a, 3)) for t, a in zip(times, curve)]})
    return out


def verify_rerun(K: int, N: int, x0: Sequence[str], T: float, tau: float = 0.01,
                 every: int = 10, factor: float = 1.25):
    """The paper's verification: the run at (K, N) against a rerun at
    (ceil(factor K), ceil(factor N)) over [0, T].  Returns the agreement
    curve, the expected-digits bound at each checkpoint and whether the run
    meets it everywhere."""
    K2, N2 = math.ceil(factor * K), math.ceil(factor * N)
    res = tc_sweep([(K, N)], (K2, N2), x0, T, tau=tau, every=every, digits=0.0)
    curve = res["variants"][0]["agreement"]
    bound = [(t, min(0.98 * K, 1.1 * N) - 0.40 * t - 3) for t, _ in curve]
    ok = all(a >= b for (_, a), (_, b) in zip(curve, bound))
    return {"K": K, "N": N, "rerun": {"K": K2, "N": N2}, "T": T, "agreement": curve,
            "expected": [(t, round(b, 3)) for t, b in bound], "verified": ok}


def main(argv: Optional[List[str]] = None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    v = sub.add_parser("verify", help="run (K, N) and the rerun at 1.25 (K, N); compare")
    v.add_argument("--K", type=int, required=True)
    v.add_argument("--N", type=int, required=True)
    v.add_argument("--T", type=float, required=True)
    v.add_argument("--every", type=int, default=10)
    s = sub.add_parser("sweep", help="T_c of (K, N) variants against a reference run")
    s.add_argument("--Ks", type=str, required=True, help="comma-separated K values")
    s.add_argument("--Ns", type=str, required=True, help="comma-separated N values (one, or one per K)")
    s.add_argument("--ref", type=str, required=True, help="reference K,N")
    s.add_argument("--T", type=float, required=True)
    s.add_argument("--every", type=int, default=10)
    s.add_argument("--digits", type=float, default=2.0)
    for p in (v, s):
        p.add_argument("--x0", type=str, default="-15.8,-17.48,35.64")
    a = ap.parse_args(argv)
    x0 = a.x0.split(",")
    if a.cmd == "verify":
        print(json.dumps(verify_rerun(a.K, a.N, x0, a.T, every=a.every)))
        return 0
    Ks = [int(t) for t in a.Ks.split(",")]
    Ns = [int(t) for t in a.Ns.split(",")]
    if len(Ns) == 1:
        Ns = Ns * len(Ks)
    if len(Ks) == 1:
        Ks = Ks * len(Ns)
    ref = tuple(int(t) for t in a.ref.split(","))
    print(json.dumps(tc_sweep(list(zip(Ks, Ns)), ref, x0, a.T, every=a.every, digits=a.digits)))
    return 0


if __name__ == "__main__":
    sys.exit(main())
