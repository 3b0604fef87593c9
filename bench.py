#!/usr/bin/env python3
"""Benchmark: Taylor steps per second of the multiple-precision Taylor series
method for the Lorenz system on one MI355X.

Default workload lorenz_k4000_n3500: sigma=10, R=28, b=8/3 (rounded to p
bits), K=4000 decimal digits (L=416 32-bit limbs, p=13312 bits), Taylor
order N=3500, tau=1/100, one trajectory from (-15.8, -17.48, 35.64) (the
paper's benchmark initial state, Section 5).  A "step" is one whole Taylor
step: the N coefficients of the Leibniz recursion (equation (3)) with their
Cauchy sums, and the Horner evaluation of the series (equation (2)).

The timed region is one device-resident persistent launch of `--steps`
steps (inputs already in HBM), bracketed by synchronisations and timed with
events on the launch stream.  Prints one JSON line.

Other modes (reported separately, not the headline line):
  --workload lorenz_k2000_n600 | lorenz_k100_n40   other single trajectories
  --mode adjoint     forward vs reverse-sweep time (K=300, N=90 x16; K=4000, N=100)
  --mode batch       256-trajectory ensemble in one launch vs one launch each
  --mode peak        measured issue rates of v_mad_i64_i32 and the int8 MFMA
  --copy-calibration one device copy of 1 GiB (for counter calibration)
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# 32x32-bit multiply-adds per second at the full VALU issue rate:
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
INT_VALU_PEAK = 256 * 4 * 16 * 2.4e9
# dense int8 matrix-core multiply-adds per second (5.0 POPS / 2)
MFMA_I8_PEAK = 2.5e15

SINGLE = {
    "lorenz_k2000_n600": dict(K=2000, N=600, x0="seed2"),
    "lorenz_k100_n40": dict(K=100, N=40, x0="bench"),
    "lorenz_k4000_n3500": dict(K=4000, N=3500, x0="bench"),
}


def limb_macs_per_step(N: int, L: int) -> float:
    """Algorithmic 32-bit limb multiply-accumulates of one Taylor step,
    N(N+5) L^2: N(N+1) Cauchy products, N products b*g_i and 3N Horner
    products of L x L limbs (the scalings by the integers sigma and R are not
    counted)."""
    return float(N * (N + 5)) * L * L


def initial_state(kind):
    from workloads import BENCH_X0, box_state
    if kind == "seed2":
        return ("double", box_state(2))
    return ("str", BENCH_X0)


def cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_baseline(workload: str, seconds_budget: float = 15.0):
    """The oracle on this host's cores: the coefficient recursion of step 0
    with each Cauchy sum split over worker processes into exact partials,
    added and rounded once by the master (the paper's reduction, Section 4;
    same bits as the single-process oracle).  Indices 0, 1, 2, ... are run
    until the budget is spent; the rate in limb products per second, divided
    by the N(N+5) products of a whole step, gives steps per second."""
    from oracle import lorenz as lz
    from oracle.parallel import ParallelOracle
    from workloads import double_strings
    w = SINGLE[workload]
    ctx = lz.make_context(K_digits=w["K"], N=w["N"])
    kind, v = initial_state(w["x0"])
    s = lz.state_from_strings(ctx, double_strings(v) if kind == "double" else v)
    workers = max(1, min(os.cpu_count() or 1, 64))
    with ParallelOracle(ctx, workers) as po:
        # the recursion in chunks of indices, each chunk restarted from
        # index 0 with a larger prefix, until the budget is spent
        M = 8
        while True:
            t0 = time.perf_counter()
            po.coefficients(s, upto=min(M, ctx.N))
            dt = time.perf_counter() - t0
            if dt >= seconds_budget or M >= ctx.N:
                break
            M = min(ctx.N, int(M * max(1.2, min(4.0, (seconds_budget / max(dt, 1e-3)) ** 0.5))))
    M = min(M, ctx.N)
    done = M * (M + 1) + M  # Cauchy products and b*g_i of indices 0..M-1
    per_step = float(ctx.N * (ctx.N + 5))
    return {"value": done / dt / per_step, "unit": "steps/s", "cores": workers, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"coefficient indices 0..{M - 1} of step 0 of {workload} ({dt:.1f} s), "
                      f"Cauchy sums split over {workers} worker processes (exact partials, one "
                      f"rounding); rate of limb products scaled to the N(N+5) products of a step"}


def run_single(args):
    import torch
    from paper_1908_09301_amd import mpts
    w = SINGLE[args.workload]
    prob = mpts.Lorenz(K=w["K"], N=w["N"])
    if args.wgs:
        prob.set_schedule(args.wgs)
    kind, v = initial_state(w["x0"])
    x0 = [prob.from_double(t) for t in v] if kind == "double" else [prob.from_str(t) for t in v]
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
    macs = limb_macs_per_step(w["N"], prob.L) * args.steps
    achieved = macs / (ms * 1e-3)
    nd = (32 * prob.L + 27 + 27) // 28
    pieces = 4 * nd
    # algorithmic int8 products of the Cauchy sums' pieces (the part the
    # matrix cores take when the path uses them)
    i8 = float(w["N"] * (w["N"] + 1)) * pieces * pieces * args.steps
    line = {
        "metric": "Taylor steps/s at (K,N)",
        "value": args.steps / (ms * 1e-3),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "none (one GPU)",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": args.workload, "K_digits": w["K"], "N": w["N"], "limbs": prob.L,
                   "p_bits": prob.p, "tau": "1/100",
                   "x0": "seed 2, uniform box" if w["x0"] == "seed2" else "(-15.8,-17.48,35.64)",
                   "workgroups": args.wgs or "all CUs",
                   "early_products": "valu" if os.environ.get("MPTS_EARLY") == "valu" else "mfma"},
        "limb_mac_per_s": achieved,
        "wall_s": wall,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": INT_VALU_PEAK / 1e12,
                     "unit": "T limb-MAC/s", "frac": achieved / INT_VALU_PEAK,
                     "traffic": traffic_from_profiles(args.workload, args.steps)},
        "mfma": {"achieved": i8 / (ms * 1e-3) / 1e12, "peak": MFMA_I8_PEAK / 1e12,
                 "unit": "T int8-MAC/s (Cauchy-sum pieces)", "frac": i8 / (ms * 1e-3) / MFMA_I8_PEAK},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = oracle_baseline(args.workload)
    print(json.dumps(line), flush=True)


def traffic_from_profiles(workload: str, steps: int):
    """HBM bytes of one launch of `steps` steps of the forward kernel, from the
    committed counter summary (measured on a launch of its own step count and
    scaled by steps), when it was taken on the current kernel source (else
    null)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_run_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    for ln in open(path):
        if "=" in ln and not ln.startswith("#"):
            k, v = ln.split("=", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1908_09301_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, fn), "rb").read())
    if fields.get("source_sha256") != h.hexdigest():
        return None
    try:
        return float(fields["hbm_bytes_per_launch"]) * steps / int(fields["steps"])
    except (KeyError, ValueError, ZeroDivisionError):
        return None


def run_adjoint(args):
    """Reverse-sweep cost against the forward run (t(reverse: recompute +
    adjoint) / t(forward), same steps): the 16-seed K=300, N=90 batch (one
    forward launch with checkpoints and one reverse launch, mpts_grad_batch,
    against the forward-only batch), and one trajectory on the widest rows
    (K=4000) at N=100.  The K=4000/N=3500 adjoint reports MPTS_ERANGE (its
    gather sums span far more than the exact-sum window)."""
    import torch
    from paper_1908_09301_amd import mpts
    from workloads import BENCH_X0, box_state
    out = {"metric": "adjoint/forward ratio"}
    n = args.steps
    probs = [mpts.Lorenz(K=300, N=90) for _ in range(16)]
    x0s = [[p.from_double(v) for v in box_state(400 + t)] for t, p in enumerate(probs)]
    mpts.grad_batch(probs, x0s, [2] * 16)  # warm up
    mpts.integrate_batch(probs, x0s, [2] * 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mpts.integrate_batch(probs, x0s, [n] * 16)
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    mpts.grad_batch(probs, x0s, [n] * 16)
    t_grad = time.perf_counter() - t0
    out["adjoint_k300_n90_x16"] = {"steps": n, "forward_s": t_fwd, "forward_plus_reverse_s": t_grad,
                                   "reverse_over_forward": (t_grad - t_fwd) / t_fwd,
                                   "total_over_forward": t_grad / t_fwd}
    m = max(1, min(args.steps, 20))
    p = mpts.Lorenz(K=4000, N=100)
    x0 = [p.from_str(v) for v in BENCH_X0]
    p.grad(x0, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.integrate(x0, m)
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    p.grad(x0, m)
    t_grad = time.perf_counter() - t0
    out["k4000_n100"] = {"steps": m, "forward_s": t_fwd, "forward_plus_reverse_s": t_grad,
                         "reverse_over_forward": (t_grad - t_fwd) / t_fwd,
                         "total_over_forward": t_grad / t_fwd}
    p5 = mpts.Lorenz(K=4000, N=3500)
    try:
        p5.grad([p5.from_str(v) for v in BENCH_X0], 1)
        out["lorenz_k4000_n3500"] = "ran"
    except mpts.MptsError as e:
        out["lorenz_k4000_n3500"] = f"MptsError {e.code}: gather sums beyond the exact-sum window"
    print(json.dumps(out), flush=True)


def run_batch(args):
    """The 256-trajectory ensemble (uneven K, N) in one graph launch vs the
    same trajectories launched one at a time."""
    import torch
    from paper_1908_09301_amd import mpts
    from workloads import ensemble, perturbed_strings
    ens = ensemble(seed=3, count=256)
    by = {}
    probs, x0s = [], []
    for e in ens:
        key = (e["K"], e["N"])
        if key not in by:
            by[key] = mpts.Lorenz(K=e["K"], N=e["N"])
        p = by[key]
        probs.append(p)
        x0s.append([p.from_str(v) for v in perturbed_strings(e["delta"])])
    n = args.steps
    flags = mpts.MPTS_GRAPH | mpts.MPTS_AUTOTUNE
    mpts.integrate_batch(probs, x0s, [n] * 256, flags=flags)  # tune, capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mpts.integrate_batch(probs, x0s, [n] * 256, flags=flags)
    t_batch = time.perf_counter() - t0
    t_single = 0.0
    per_class = {}
    for key, p in by.items():
        t = [i for i in range(256) if (ens[i]["K"], ens[i]["N"]) == key][0]
        p.integrate(x0s[t], 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p.integrate(x0s[t], n)
        per_class[key] = time.perf_counter() - t0
    for e in ens:
        t_single += per_class[(e["K"], e["N"])]
    print(json.dumps({"metric": "batch ratio", "workload": "ensemble256_mixed", "steps": n,
                      "batch_s": t_batch, "one_launch_each_s": t_single,
                      "ratio": t_single / t_batch,
                      "per_class_single_s": {f"{k[0]}/{k[1]}": v for k, v in per_class.items()}}),
          flush=True)


def run_poly(args):
    """Polynomial vector fields (k_poly, one workgroup per trajectory): the
    Roessler ensemble (64 trajectories, K=300, N=90) in one launch, and the
    Lorenz system given as terms against the Lorenz batch path on 16 of the
    same-size trajectories."""
    import torch
    from paper_1908_09301_amd import mpts
    from workloads import POLY_ENSEMBLE, POLY_SYSTEMS, poly_states
    E = POLY_ENSEMBLE
    nvar, terms = POLY_SYSTEMS[E["system"]]
    p = mpts.Poly(nvar, terms, K=E["K"], N=E["N"])
    x0s = [[p.from_str(v) for v in x] for x in poly_states(E["seed"], E["count"], E["system"])]
    n = args.steps
    p.integrate(x0s, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.integrate(x0s, n)
    t = time.perf_counter() - t0
    # limb MACs of one trajectory step (schoolbook count): the Cauchy sums of
    # the product pairs, the products of non-unit coefficients, the Horner steps
    N, L = E["N"], p.L
    pairs = {(min(u, w), max(u, w)) for (_, _, u, w) in terms if w >= 0}
    nprod = sum(1 for (_, c, u, _) in terms if u >= 0 and c not in ("1", "-1"))
    macs = (len(pairs) * N * (N + 1) // 2 + nprod * N + nvar * N) * L * L
    out = {"metric": "polynomial-system ensemble", "workload": f"{E['system']}_k{E['K']}_n{N}_x{E['count']}",
           "steps": n, "s": t, "trajectory_steps_per_s": E["count"] * n / t,
           "ms_per_step": t / n * 1e3, "limb_mac_per_s": E["count"] * n * macs / t,
           "frac_of_alu_peak": E["count"] * n * macs / t / INT_VALU_PEAK}
    # the Lorenz terms on k_poly vs the Lorenz batch path, 16 trajectories
    ln, lt = POLY_SYSTEMS["lorenz"]
    q = mpts.Poly(ln, lt, K=E["K"], N=E["N"])
    lor = mpts.Lorenz(K=E["K"], N=E["N"])
    xs = [[lor.from_str(v) for v in x] for x in poly_states(7, 16, "lorenz")]
    q.integrate(xs, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    q.integrate(xs, n)
    tq = time.perf_counter() - t0
    mpts.integrate_batch([lor] * 16, xs, [n] * 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mpts.integrate_batch([lor] * 16, xs, [n] * 16)
    tl = time.perf_counter() - t0
    out["lorenz_terms_x16"] = {"poly_s": tq, "lorenz_batch_s": tl, "poly_over_lorenz": tq / tl}
    print(json.dumps(out), flush=True)


def run_peak():
    """Measured issue rates of the two arithmetic units (registers only)."""
    from paper_1908_09301_amd import mpts
    mad = mpts.probe_rate(mpts.MPTS_PROBE_VALU_MAD)
    i8 = mpts.probe_rate(mpts.MPTS_PROBE_MFMA_I8)
    print(json.dumps({"metric": "measured peak", "v_mad_i64_i32_per_s": mad,
                      "v_mad_frac_of_stated": mad / INT_VALU_PEAK,
                      "mfma_i8_mac_per_s": i8, "mfma_frac_of_stated": i8 / MFMA_I8_PEAK,
                      "stated_valu_peak": INT_VALU_PEAK, "stated_mfma_i8_peak": MFMA_I8_PEAK}),
          flush=True)


def copy_calibration():
    import torch
    a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": 1 << 30}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--wgs", type=int, default=0, help="workgroups per trajectory (0: all CUs)")
    ap.add_argument("--workload", default="lorenz_k4000_n3500", choices=sorted(SINGLE))
    ap.add_argument("--mode", default="single", choices=["single", "adjoint", "batch", "peak", "poly"])
    ap.add_argument("--copy-calibration", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); this build measures the "
              "single-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
    elif args.mode == "adjoint":
        run_adjoint(args)
    elif args.mode == "batch":
        run_batch(args)
    elif args.mode == "poly":
        run_poly(args)
    elif args.mode == "peak":
        run_peak()
    else:
        run_single(args)


if __name__ == "__main__":
    main()
