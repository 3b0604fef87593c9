"""Writes the regression fixtures of this folder from the oracle alone.

The paper prints no numerical solution values (its performance runs report
times only, Section 5), so nothing here is a value from the paper: these
files are the oracle's own states, kept so that a later change to the
oracle's arithmetic shows up as a diff, and so that the GPU tests can compare
against stored values as well as against a live oracle run.

    python tests/golden/make_golden.py

lorenz_k100_n40_states.txt: the K=100-digit, N=40, tau=1/100 trajectory
from x0 = (-15.8, -17.48, 35.64) (each coordinate rounded once to p bits),
the exact (sign, mantissa, exponent) of x, y, z after the listed steps.
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import lorenz as lz  # noqa: E402

X0 = ("-15.8", "-17.48", "35.64")
STEPS = (0, 1, 2, 10, 50, 100)


def main():
    ctx = lz.make_context(K_digits=100, N=40)
    x0 = lz.state_from_strings(ctx, X0)
    _, states = lz.integrate(ctx, x0, max(STEPS), keep_states=True)
    path = os.path.join(HERE, "lorenz_k100_n40_states.txt")
    with open(path, "w") as f:
        f.write("# oracle states of the K=100, N=40, tau=1/100 trajectory from\n")
        f.write("# x0 = (-15.8, -17.48, 35.64); written by make_golden.py (oracle only)\n")
        f.write("# step component sign mantissa(hex) exponent\n")
        for n in STEPS:
            for c, v in zip("xyz", states[n]):
                f.write(f"{n} {c} {v.s} {v.m:x} {v.e}\n")
    print(path)


if __name__ == "__main__":
    main()
