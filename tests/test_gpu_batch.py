"""Batched ensembles (one persistent launch, trajectories of uneven K and N,
optional hipGraph capture and autotuned workgroups per trajectory) against
the oracle, bit for bit (GPU)."""
import sys

import pytest

from oracle import lorenz as lz
from workloads import ENSEMBLE_CLASSES, ensemble, perturbed_strings

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_batch():
    """Nine trajectories of three small (L, N) classes and uneven lengths."""
    specs = []
    for t in range(9):
        L, N = [(2, 6), (5, 17), (12, 40)][t % 3]
        d = (1e-3 * (t + 1), -2e-3 * t, 3e-3)
        specs.append((L, N, 3 + t, perturbed_strings(d)))
    return specs


def run_batch(gpu_lib, specs, flags):
    probs = [gpu_lib.Lorenz(L=L, N=N) for (L, N, _, _) in specs]
    x0s = [[p.from_str(v) for v in xs] for p, (_, _, _, xs) in zip(probs, specs)]
    return gpu_lib.integrate_batch(probs, x0s, [n for (_, _, n, _) in specs], flags=flags), probs


def oracle_runs(specs):
    out = []
    for (L, N, n, xs) in specs:
        ctx = lz.make_context(L=L, N=N)
        out.append([tuple(v) for v in lz.integrate(ctx, lz.state_from_strings(ctx, xs), n)])
    return out


@pytest.mark.parametrize("flags", ["plain", "graph", "autotune+graph"])
def test_small_mixed_batch_matches_oracle(gpu_lib, flags):
    say("batch", flags)
    f = {"plain": 0, "graph": gpu_lib.MPTS_GRAPH,
         "autotune+graph": gpu_lib.MPTS_GRAPH | gpu_lib.MPTS_AUTOTUNE}[flags]
    specs = small_batch()
    ref = oracle_runs(specs)
    got, _ = run_batch(gpu_lib, specs, f)
    assert got == ref


def test_graph_replays_match_eager(gpu_lib):
    """The captured graph is replayed several times, with eager work and
    synchronisations between the replays; every replay equals the eager run."""
    import torch
    specs = small_batch()
    eager, _ = run_batch(gpu_lib, specs, 0)
    probs = [gpu_lib.Lorenz(L=L, N=N) for (L, N, _, _) in specs]
    x0s = [[p.from_str(v) for v in xs] for p, (_, _, _, xs) in zip(probs, specs)]
    ns = [n for (_, _, n, _) in specs]
    for rep in range(4):
        got = gpu_lib.integrate_batch(probs, x0s, ns, flags=gpu_lib.MPTS_GRAPH)
        assert got == eager, rep
        # eager work in between: a single-trajectory run and a device sync
        probs[0].integrate(x0s[0], 2)
        torch.cuda.synchronize()


def test_ensemble256_one_step_sampled(gpu_lib):
    """The 256-trajectory ensemble with uneven (K, N) from four classes and
    perturbed initial states, one step, in one autotuned graph launch: one
    trajectory of each class checked against the oracle, and every
    trajectory equal to its own single-trajectory run."""
    say("ensemble256 one step")
    ens = ensemble(seed=3, count=256)
    probs_by_class = {}
    probs, x0s = [], []
    for e in ens:
        key = (e["K"], e["N"])
        if key not in probs_by_class:
            probs_by_class[key] = gpu_lib.Lorenz(K=e["K"], N=e["N"])
        p = probs_by_class[key]
        probs.append(p)
        x0s.append([p.from_str(v) for v in perturbed_strings(e["delta"])])
    got = gpu_lib.integrate_batch(probs, x0s, [1] * 256,
                                  flags=gpu_lib.MPTS_GRAPH | gpu_lib.MPTS_AUTOTUNE)
    seen = set()
    for t, e in enumerate(ens):
        key = (e["K"], e["N"])
        if key in seen:
            continue
        seen.add(key)
        ctx = lz.make_context(K_digits=e["K"], N=e["N"])
        ref = lz.step(ctx, lz.state_from_strings(ctx, perturbed_strings(e["delta"])))
        assert got[t] == [tuple(v) for v in ref], (t, key)
    assert len(seen) == len(ENSEMBLE_CLASSES)
    for t in range(0, 256, 37):
        single = probs[t].integrate(x0s[t], 1)
        assert got[t] == single, t
