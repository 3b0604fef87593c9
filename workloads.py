"""Seeded synthetic inputs for the Lorenz Taylor-series workloads.

Holds no arithmetic of the method: it only draws and names inputs (initial
states as exact decimal strings or float64 values, seeds, (K, N) classes), so
that the oracle-side tests and the HIP-side tests and benchmark are fed the
same data.  RNG: numpy.random.default_rng(seed) (PCG64).

Workloads (the Lorenz parameters are always sigma=10, R=28, b=8/3, step
tau=1/100; the benchmark initial state (-15.8, -17.48, 35.64) is the one the
paper takes for its performance runs, Section 5):
  lorenz_k100_n40      K=100 digits, N=40, 1000 steps, fixed initial state
  lorenz_k2000_n600    K=2000, N=600, 1000 steps, seeded initial state
  ensemble256_mixed    256 trajectories, (K, N) drawn from 4 classes,
                       perturbed fixed initial state, 2000 steps
  adjoint_k300_n90     K=300, N=90, 2000 steps, 16 seeded initial states
  lorenz_k4000_n3500   K=4000, N=3500, 200 steps, fixed initial state
"""
from typing import List, Tuple

import numpy as np

BENCH_X0 = ("-15.8", "-17.48", "35.64")
PARAMS = {"sigma": "10", "R": "28", "b": "8/3", "tau": "1/100"}

BOX_LO = (-20.0, -25.0, 5.0)
BOX_HI = (20.0, 25.0, 45.0)

ENSEMBLE_CLASSES = ((200, 60), (400, 120), (800, 240), (1600, 480))

WORKLOADS = {
    "lorenz_k100_n40": dict(K=100, N=40, nsteps=1000),
    "lorenz_k2000_n600": dict(K=2000, N=600, nsteps=1000, seed=2),
    "ensemble256_mixed": dict(count=256, nsteps=2000, seed=3),
    "adjoint_k300_n90": dict(K=300, N=90, nsteps=2000, seeds=tuple(range(400, 416))),
    "lorenz_k4000_n3500": dict(K=4000, N=3500, nsteps=200),
}


def box_state(seed: int) -> Tuple[float, float, float]:
    """One initial state uniform in [-20,20]x[-25,25]x[5,45] (float64, so it
    is exact at every precision used here)."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(BOX_LO, BOX_HI)
    return tuple(float(t) for t in v)


def box_states(seeds) -> List[Tuple[float, float, float]]:
    return [box_state(s) for s in seeds]


def ensemble(seed: int = 3, count: int = 256):
    """Per-trajectory (K, N) class and float64 perturbation of the benchmark
    initial state.  Returns a list of dicts with K, N and the three
    perturbations (each uniform in [-1e-30, 1e-30])."""
    rng = np.random.default_rng(seed)
    cls = rng.integers(0, len(ENSEMBLE_CLASSES), count)
    delta = rng.uniform(-1e-30, 1e-30, (count, 3))
    out = []
    for t in range(count):
        K, N = ENSEMBLE_CLASSES[int(cls[t])]
        out.append(dict(K=K, N=N, delta=tuple(float(d) for d in delta[t])))
    return out


def perturbed_strings(delta) -> Tuple[str, str, str]:
    """The benchmark initial state plus exact float64 perturbations, as exact
    rational strings "num/den" (the perturbation's binary value is exact)."""
    from fractions import Fraction
    out = []
    for base, d in zip(BENCH_X0, delta):
        q = Fraction(base) + Fraction(d)
        out.append(f"{q.numerator}/{q.denominator}")
    return tuple(out)


def double_strings(v) -> Tuple[str, ...]:
    """Exact decimal-free rational strings of float64 values."""
    from fractions import Fraction
    out = []
    for t in v:
        q = Fraction(t)
        out.append(f"{q.numerator}/{q.denominator}")
    return tuple(out)


def random_limb_values(seed: int, count: int, L: int, spread_bits: int = 24):
    """Random signed (sign, mantissa, exponent) triples with normalised
    32*L-bit mantissas and exponents spread over `spread_bits`; for unit
    parity tests of the accumulate-and-round primitives."""
    rng = np.random.default_rng(seed)
    p = 32 * L
    out = []
    for _ in range(count):
        limbs = rng.integers(0, 1 << 32, L, dtype=np.uint64)
        m = 0
        for j in range(L):
            m |= int(limbs[j]) << (32 * j)
        m |= 1 << (p - 1)
        s = int(rng.choice([-1, 1]))
        e = int(rng.integers(-spread_bits, spread_bits + 1)) - p
        out.append((s, m, e))
    return out


# ---------------------------------------------------------------------------
# Polynomial vector fields of degree <= 2 (inputs only): each system is a
# number of variables and a tuple of terms (equation, coefficient text,
# u, w) meaning coef * x_u * x_w in dx_eq/dt (u, w = -1: absent).

POLY_SYSTEMS = {
    # the Lorenz system in this form (sigma (y - x), R x - y - x z, x y - b z)
    "lorenz": (3, ((0, "-10", 0, -1), (0, "10", 1, -1), (1, "28", 0, -1), (1, "-1", 1, -1),
                   (1, "-1", 0, 2), (2, "1", 0, 1), (2, "-8/3", 2, -1))),
    # Roessler: x' = -y - z, y' = x + a y, z' = b + z x - c z (a = b = 0.2, c = 5.7)
    "rossler": (3, ((0, "-1", 1, -1), (0, "-1", 2, -1), (1, "1", 0, -1), (1, "0.2", 1, -1),
                    (2, "0.2", -1, -1), (2, "1", 2, 0), (2, "-5.7", 2, -1))),
    # Chen: x' = a (y - x), y' = (c - a) x - x z + c y, z' = x y - b z (a = 35, b = 3, c = 28)
    "chen": (3, ((0, "35", 1, -1), (0, "-35", 0, -1), (1, "-7", 0, -1), (1, "-1", 0, 2),
                 (1, "28", 1, -1), (2, "1", 0, 1), (2, "-3", 2, -1))),
    # a four-variable Roessler-type system: x' = -y - z, y' = x + 0.25 y + w,
    # z' = 3 + x z, w' = -0.5 z + 0.05 w
    "rossler4": (4, ((0, "-1", 1, -1), (0, "-1", 2, -1), (1, "1", 0, -1), (1, "0.25", 1, -1),
                     (1, "1", 3, -1), (2, "3", -1, -1), (2, "1", 0, 2), (3, "-0.5", 2, -1),
                     (3, "0.05", 3, -1))),
    # closed forms: x' = x^2 (x(t) = x0 / (1 - x0 t)), x' = -x, and the
    # harmonic oscillator x' = -y, y' = x
    "square": (1, ((0, "1", 0, 0),)),
    "decay": (1, ((0, "-1", 0, -1),)),
    "oscillator": (2, ((0, "-1", 1, -1), (1, "1", 0, -1))),
}

POLY_X0 = {
    "lorenz": BENCH_X0,
    "rossler": ("1", "1", "1"),
    "chen": ("-10", "0", "37"),
    "rossler4": ("-10", "-6", "0", "10"),
    "square": ("1/8",),
    "decay": ("1",),
    "oscillator": ("1", "0"),
}

# The polynomial-system ensemble: Roessler trajectories at K=300 digits,
# N=90, from seeded states x0 + uniform [-1, 1]^3 (float64, exact)
POLY_ENSEMBLE = dict(system="rossler", K=300, N=90, count=64, nsteps=100, seed=5)


def poly_states(seed: int, count: int, system: str = "rossler") -> List[Tuple[str, ...]]:
    """`count` initial states of `system`: its base state plus float64
    offsets uniform in [-1, 1], as exact rational strings."""
    from fractions import Fraction
    rng = np.random.default_rng(seed)
    base = POLY_X0[system]
    d = rng.uniform(-1.0, 1.0, (count, len(base)))
    out = []
    for t in range(count):
        row = []
        for b, x in zip(base, d[t]):
            q = Fraction(b) + Fraction(float(x))
            row.append(f"{q.numerator}/{q.denominator}")
        out.append(tuple(row))
    return out
