"""The stored oracle states in tests/golden (CPU).

The paper prints no numerical solution values, so the fixture is the
oracle's own output (written by tests/golden/make_golden.py, which calls only
oracle/): recomputing it catches any later change to the oracle's
arithmetic.  Its first steps are also checked against the independent
Fraction statement of the step (tests/fraction_reference.py).
"""
import os
from fractions import Fraction

import fraction_reference as fr
from oracle import lorenz as lz
from oracle.bigfloat import BF

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lorenz_k100_n40_states.txt")
X0 = ("-15.8", "-17.48", "35.64")


def load_states():
    """{(step, component): (sign, mantissa, exponent)} from the fixture."""
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            n, c, s, m, e = line.split()
            out[(int(n), c)] = (int(s), int(m, 16), int(e))
    return out


def test_stored_states_are_the_oracle_s():
    stored = load_states()
    ctx = lz.make_context(K_digits=100, N=40)
    x0 = lz.state_from_strings(ctx, X0)
    last = max(n for n, _ in stored)
    _, states = lz.integrate(ctx, x0, last, keep_states=True)
    for (n, c), v in stored.items():
        assert tuple(states[n]["xyz".index(c)]) == v, (n, c)


def test_first_steps_match_the_fraction_statement():
    stored = load_states()
    p = 32 * 12  # K = 100 digits -> 12 limbs
    state = tuple(fr.rne(Fraction(x), p) for x in X0)
    for n in range(3):
        for k, c in enumerate("xyz"):
            assert BF(*stored[(n, c)]).frac() == state[k], (n, c)
        state = fr.step(state, 40, p)
