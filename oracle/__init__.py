"""Plain, slow, exact CPU oracle for the multiple-precision Taylor series method
for the Lorenz system (Dimova et al., "OpenMP parallelization of multiple
precision Taylor series method", Sections 2 and 4, equations (1)-(3)).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package; only the test suite, the smoke check and
the CPU-baseline leg of the benchmark use it.  It shares no code, tables or
helpers with the HIP implementation.

Arithmetic is done in CPython integers (exact) and fractions.Fraction; every
rounding is round-to-nearest, ties-to-even, to p = 32*L bits.  The rounding
points are the project semantics:

  * each Cauchy-product sum of equation (3) is the exact sum of exact
    products, rounded once;
  * each new Taylor coefficient of equation (3) is its exact numerator
    divided by (i+1), rounded once;
  * each Horner step h <- h*tau + c_i of the series of equation (2) is
    rounded once (fused multiply-add).

Modules:
  bigfloat  -- the number type, exact sums, rounding, parsing, FP64 export
  lorenz    -- context, Taylor coefficients (eq. 3), Horner step (eq. 2),
               integration with per-step checkpoints
  adjoint   -- reverse-mode derivative of one step and of a whole run
"""
import sys as _sys

# Decimal printing of 10^4-digit integers needs the CPython limit lifted.
if hasattr(_sys, "set_int_max_str_digits"):
    _sys.set_int_max_str_digits(0)

from .bigfloat import BF, ZERO  # noqa: E402,F401
