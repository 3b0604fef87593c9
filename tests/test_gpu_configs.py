"""Bit-exact parity of whole runs at the five benchmark workloads, checked
transition by transition (GPU).

The step map s_n -> s_{n+1} (equations (2)-(3)) is a pure function of the
p-bit state.  So when the oracle, started from the GPU's checkpoint s_n,
reproduces the GPU's s_{n+1} bit for bit for every n, the GPU run equals the
oracle's run from s_0 by induction; where the oracle is too slow for every
n, a stated stratified set of transitions is checked.  Inside a step the
same holds for the coefficient recursion: index transition i (equation (3))
maps the coefficients 0..i to i+1, and the Horner sums (equation (2)) map the
coefficients to s_{n+1}.

The oracle work is fanned out over the host's cores (tests/oracle_pool.py,
at most 16 worker processes, never touching the GPU).  Oracle costs measured
on a 16-core EPYC host: one K=2000/N=600 step 5.7 s, one K=300/N=90 step
0.011 s, one L=416 product 45 us.  MPTS_PARITY_SCALE (default 1) divides
every sampling stride (a larger value checks more transitions).
"""
import os
import sys

import pytest

import oracle_pool as op
from oracle import lorenz as lz
from oracle import adjoint as oad
from oracle.bigfloat import BF, to_double
from workloads import (BENCH_X0, ENSEMBLE_CLASSES, box_state, double_strings, ensemble,
                       perturbed_strings)

pytestmark = pytest.mark.gpu

SCALE = max(1, int(os.environ.get("MPTS_PARITY_SCALE", "1")))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def stride(s):
    return max(1, s // SCALE)


def stratified(n_total, every, head=3, tail=3):
    """Transitions 0..head-1, every `every`-th, and the last `tail`."""
    pick = set(range(min(head, n_total)))
    pick.update(range(0, n_total, every))
    pick.update(range(max(0, n_total - tail), n_total))
    return sorted(pick)


@pytest.fixture(scope="module")
def pool():
    p = op.make_pool()
    yield p
    p.shutdown()


def check_steps(pool, L, N, states, ns, chunk=8):
    """Every n in ns: oracle step of states[n] == states[n+1]."""
    futs = []
    for k in range(0, len(ns), chunk):
        part = ns[k:k + chunk]
        for n in part:
            futs.append(pool.submit(op.step_task, L, N, n, states[n], states[n + 1]))
    bad = [f.result() for f in futs]
    return [n for n in bad if n is not None]


def check_step_inside(pool, gpu_p, L, N, state, nxt, indices):
    """GPU coefficients of one step from `state` (mpts_coefficients): the
    index transitions in `indices` and the three Horner sums against `nxt`."""
    coefs = gpu_p.coefficients(state)
    assert (coefs[0][0], coefs[1][0], coefs[2][0]) == tuple(tuple(v) for v in state)
    path = op.store_coefficients(coefs)
    try:
        futs = [pool.submit(op.transitions_task, L, N, path, part)
                for part in op.chunked(indices, 4 * op.n_workers())]
        futs += [pool.submit(op.horner_task, L, N, path, c, nxt[c]) for c in range(3)]
        res = [f.result() for f in futs]
    finally:
        os.unlink(path)
    bad = [i for r in res[:-3] for i in r]
    return bad, res[-3:]


def test_k100_n40_every_transition(gpu_lib, pool):
    """K=100, N=40, 1000 steps from (-15.8, -17.48, 35.64): all 1000
    transitions."""
    say("k100 n40: 1000 steps, every transition")
    ctx = lz.make_context(K_digits=100, N=40)
    x0 = lz.state_from_strings(ctx, BENCH_X0)
    p = gpu_lib.Lorenz(K=100, N=40)
    _, states = p.integrate([tuple(v) for v in x0], 1000, checkpoints=True)
    assert states[0] == [tuple(v) for v in x0]
    assert check_steps(pool, ctx.L, 40, states, list(range(1000))) == []


def test_k2000_n600_stratified_transitions(gpu_lib, pool):
    """K=2000 (208 limbs), N=600, seeded initial state, 1000 steps on every
    compute unit: transitions 0-2, every 10th and the last three (106 whole
    oracle steps, about 40 s on 16 cores)."""
    say("k2000 n600: 1000 steps")
    ctx = lz.make_context(K_digits=2000, N=600)
    x0 = lz.state_from_strings(ctx, double_strings(box_state(2)))
    p = gpu_lib.Lorenz(K=2000, N=600)
    _, states = p.integrate([tuple(v) for v in x0], 1000, checkpoints=True)
    assert states[0] == [tuple(v) for v in x0]
    ns = stratified(1000, stride(10))
    say("k2000 n600: checking", len(ns), "transitions")
    assert check_steps(pool, ctx.L, 600, states, ns) == []


def test_k4000_n3500_steps(gpu_lib, pool):
    """K=4000 (416 limbs), N=3500, 200 steps from (-15.8, -17.48, 35.64):
    step 0 completely (all 3500 index transitions and the Horner sums:
    12.25 M products, about 35 s on 16 cores), and steps 1, 100, 199 on
    indices 0-2, every 50th and the last five, with their Horner sums."""
    say("k4000 n3500: 200 steps")
    ctx = lz.make_context(K_digits=4000, N=3500)
    x0 = lz.state_from_strings(ctx, BENCH_X0)
    p = gpu_lib.Lorenz(K=4000, N=3500)
    states = [[tuple(v) for v in x0]]
    for seg in range(10):
        # 20 steps at a time (checkpointed), each segment from the last state
        _, st = p.integrate(states[-1], 20, checkpoints=True)
        assert st[0] == states[-1]
        states += st[1:]
        say("k4000 n3500: steps done", len(states) - 1)
    assert len(states) == 201
    for n, idx in ((0, list(range(3500))), (1, None), (100, None), (199, None)):
        if idx is None:
            idx = stratified(3500, stride(50), head=3, tail=5)
        say("k4000 n3500: step", n, "indices", len(idx))
        bad, horner = check_step_inside(pool, p, ctx.L, 3500, states[n], states[n + 1], idx)
        assert bad == [], (n, bad[:5])
        assert horner == [True, True, True], n


def test_ensemble_classes_whole_runs(gpu_lib, pool):
    """One trajectory of each (K, N) class of the 256-trajectory ensemble
    (perturbed initial states), 2000 steps each: every transition of the
    (200, 60) and (400, 120) classes, every 4th of (800, 240) and every 25th
    of (1600, 480) (plus the first and last three)."""
    ens = ensemble(seed=3, count=256)
    every = {(200, 60): 1, (400, 120): 1, (800, 240): 4, (1600, 480): 25}
    seen = {}
    for t, e in enumerate(ens):
        seen.setdefault((e["K"], e["N"]), t)
    assert len(seen) == len(ENSEMBLE_CLASSES)
    for key, t in sorted(seen.items()):
        K, N = key
        say("ensemble class", key, "trajectory", t)
        ctx = lz.make_context(K_digits=K, N=N)
        x0 = lz.state_from_strings(ctx, perturbed_strings(ens[t]["delta"]))
        p = gpu_lib.Lorenz(K=K, N=N)
        _, states = p.integrate([tuple(v) for v in x0], 2000, checkpoints=True)
        assert states[0] == [tuple(v) for v in x0]
        ns = stratified(2000, stride(every[key]))
        assert check_steps(pool, ctx.L, N, states, ns) == [], key


def test_ensemble256_batch_matches_whole_runs(gpu_lib):
    """The 256-trajectory ensemble in one autotuned graph launch (10 steps):
    every trajectory equals the same ensemble run as a plain launch, and one
    trajectory per class equals its single-trajectory run (whose transitions
    the test above checks against the oracle)."""
    ens = ensemble(seed=3, count=256)
    by, probs, x0s = {}, [], []
    for e in ens:
        key = (e["K"], e["N"])
        if key not in by:
            by[key] = gpu_lib.Lorenz(K=e["K"], N=e["N"])
        probs.append(by[key])
        x0s.append([by[key].from_str(v) for v in perturbed_strings(e["delta"])])
    say("ensemble256: graph + autotune, 10 steps")
    tuned = gpu_lib.integrate_batch(probs, x0s, [10] * 256,
                                    flags=gpu_lib.MPTS_GRAPH | gpu_lib.MPTS_AUTOTUNE)
    say("ensemble256: plain launch")
    plain = gpu_lib.integrate_batch(probs, x0s, [10] * 256, flags=0)
    assert tuned == plain
    seen = set()
    for t, e in enumerate(ens):
        key = (e["K"], e["N"])
        if key in seen:
            continue
        seen.add(key)
        assert tuned[t] == probs[t].integrate(x0s[t], 10), key


def test_adjoint_k300_n90_sixteen_seeds(gpu_lib, pool):
    """K=300, N=90, 2000 steps, seeds 400..415, loss ||x(T)||^2, all 16
    gradients in one batched call: every seed's final state equals the
    oracle's 2000-step run, seed 400's six gradients (p-bit values rounded to
    FP64) and loss equal the oracle adjoint over all 2000 steps, and every
    seed's gradient equals its own single mpts_grad call."""
    K, N, nsteps = 300, 90, 2000
    seeds = list(range(400, 416))
    ctx = lz.make_context(K_digits=K, N=N)
    x0s = [lz.state_from_strings(ctx, double_strings(box_state(s))) for s in seeds]
    futs = [pool.submit(op.adjoint_task, ctx.L, N, x0s[0], nsteps)]
    futs += [pool.submit(op.run_task, ctx.L, N, x, nsteps) for x in x0s]
    probs = [gpu_lib.Lorenz(K=K, N=N) for _ in seeds]
    say("adjoint k300 n90: 16 seeds x 2000 steps")
    g, lv, fin = gpu_lib.grad_batch(probs, [[tuple(v) for v in x] for x in x0s], [nsteps] * 16)
    for t in (0, 7, 15):
        g1, _, f1, l1 = probs[t].grad([tuple(v) for v in x0s[t]], nsteps)
        assert (g1, f1, l1) == (g[t], fin[t], lv[t]), t
    xT, ref = futs[0].result()
    assert fin[0] == [tuple(v) for v in xT]
    assert g[0] == [to_double(BF(*v)) for v in ref]
    assert lv[0] == oad.loss_value("sqnorm", [BF(*v) for v in xT])
    for t in range(16):
        assert fin[t] == [tuple(v) for v in futs[1 + t].result()], t


def test_adjoint_k4000_n100_matches_oracle(gpu_lib):
    """The reverse sweep on the widest rows (K=4000, 416 limbs, the k_adj
    instance of the K=4000 workload) at N=100 over two steps from
    (-15.8, -17.48, 35.64), loss ||x(T)||^2: the six p-bit gradients, their
    FP64 values, the loss and the final state equal the oracle adjoint bit
    for bit.  At this order the adjoint's gather sums span at most about 410
    bits (an oracle scan of the same steps), inside the device window."""
    K, N, nsteps = 4000, 100, 2
    ctx = lz.make_context(K_digits=K, N=N)
    x0 = lz.state_from_strings(ctx, BENCH_X0)
    p = gpu_lib.Lorenz(K=K, N=N)
    say("adjoint k4000 n100: two steps")
    g64, gbf, fin, lv = p.grad([tuple(v) for v in x0], nsteps)
    say("adjoint k4000 n100: oracle")
    xT, ref = oad.grad(ctx, x0, nsteps)
    assert fin == [tuple(v) for v in xT]
    assert gbf == [tuple(v) for v in ref]
    assert g64 == [to_double(v) for v in ref]
    assert lv == oad.loss_value("sqnorm", xT)


def test_adjoint_k4000_n3500_reports_the_window(gpu_lib):
    """The reverse sweep of the K=4000/N=3500 step: its gather sums decay
    like (tau/rho)^j over j = m..N-1 and span about 14 200 bits (an oracle
    scan of the first step), far past the device's exact-sum window, so the
    call fails with MPTS_ERANGE instead of returning inexact gradients."""
    p = gpu_lib.Lorenz(K=4000, N=3500)
    x0 = [p.from_str(v) for v in BENCH_X0]
    say("adjoint k4000 n3500: one step, window overflow expected")
    with pytest.raises(gpu_lib.MptsError) as ei:
        p.grad(x0, 1)
    assert ei.value.code == gpu_lib.MPTS_ERANGE
