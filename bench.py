#!/usr/bin/env python3
"""Benchmark: Taylor steps per second of the multiple-precision Taylor series
method for the Lorenz system on one MI355X.

Workload lorenz_k2000_n600: sigma=10, R=28, b=8/3 (rounded to p bits),
K=2000 decimal digits (L=208 32-bit limbs, p=6656 bits), Taylor order N=600,
tau=1/100, one trajectory from the seeded initial state (seed 2, uniform in
[-20,20]x[-25,25]x[5,45]).  A "step" is one whole Taylor step: the N
coefficients of the Leibniz recursion (equation (3)) with their Cauchy sums,
and the Horner evaluation of the series (equation (2)).

The timed region is one device-resident persistent launch of `--steps`
steps (inputs already in HBM), bracketed by synchronisations and timed with
events on the launch stream.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "lorenz_k2000_n600"
K_DIGITS, N_ORDER = 2000, 600
INT_VALU_PEAK = 256 * 4 * 16 * 2.4e9  # 32x32-bit multiply-adds per second (full issue rate)


def limb_macs_per_step(N: int, L: int) -> float:
    """Algorithmic 32-bit limb multiply-accumulates of one Taylor step,
    N(N+5) L^2: N(N+1) Cauchy products, N products b*g_i and 3N Horner
    products of L x L limbs (the scalings by the integers sigma and R are not
    counted)."""
    return float(N * (N + 5)) * L * L


def oracle_baseline(seconds_budget: float = 20.0):
    """The oracle, as it stands, on this host: steps of the same workload
    until the budget is used (at least one)."""
    from oracle import lorenz as lz
    from workloads import box_state, double_strings
    ctx = lz.make_context(K_digits=K_DIGITS, N=N_ORDER)
    s = lz.state_from_strings(ctx, double_strings(box_state(2)))
    n = 0
    t0 = time.perf_counter()
    while True:
        s = lz.step(ctx, s)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= seconds_budget or n >= 3:
            break
    return {"value": n / dt, "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} step(s) of {WORKLOAD} from the seeded state, single-threaded CPython"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--wgs", type=int, default=0, help="workgroups per trajectory (0: all CUs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the trajectory's "
              "coefficient recursion is sequential and this build does not shard it", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1908_09301_amd import mpts
    from workloads import box_state

    torch.cuda.set_device(0)
    prob = mpts.Lorenz(K=K_DIGITS, N=N_ORDER)
    if args.wgs:
        prob.set_schedule(args.wgs)
    x0 = [prob.from_double(v) for v in box_state(2)]
    x0_dev = prob.pack_state(x0).cuda()
    xout = torch.empty_like(x0_dev)
    ws = prob.workspace(max(args.steps, args.warmup))

    if args.warmup > 0:
        prob.integrate_dev(x0_dev, args.warmup, xout, ws=ws)
        prob.check(ws)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    prob.integrate_dev(x0_dev, args.steps, xout, ws=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prob.check(ws)
    ms = e0.elapsed_time(e1)
    ms_per_step = ms / args.steps
    value = args.steps / (ms * 1e-3)
    macs = limb_macs_per_step(N_ORDER, prob.L) * args.steps
    achieved = macs / (ms * 1e-3)

    line = {
        "metric": "Taylor steps/s at (K,N)",
        "value": value,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "K_digits": K_DIGITS, "N": N_ORDER, "limbs": prob.L,
                   "p_bits": prob.p, "tau": "1/100", "x0": "seed 2, uniform box",
                   "workgroups": args.wgs or "all CUs"},
        "limb_mac_per_s": achieved,
        "wall_s": wall,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": INT_VALU_PEAK / 1e12,
                     "unit": "T limb-MAC/s", "frac": achieved / INT_VALU_PEAK, "traffic": None},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = oracle_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
