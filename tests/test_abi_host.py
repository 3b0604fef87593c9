"""The C-ABI library loads, exports every symbol include/mpts.h declares, and
its host-side number handling (exact parse + one RNE rounding, FP64 export)
agrees with the oracle.  CPU only: no kernel is launched."""
import re
from fractions import Fraction
import os

import pytest

from oracle.bigfloat import parse, from_fraction, to_double, BF
from oracle.lorenz import make_context
from workloads import BENCH_X0

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1908_09301_amd import mpts
    return mpts


def test_every_declared_symbol_is_exported():
    mpts = _lib()
    header = open(os.path.join(ROOT, "include", "mpts.h")).read()
    declared = set(re.findall(r"\b(mpts_[a-z_0-9]+)\s*\(", header))
    declared -= {"mpts_bf"}
    assert declared == set(mpts.SYMBOLS)
    assert sorted(mpts.exported_symbols()) == sorted(declared)


@pytest.mark.parametrize("K", [100, 2000, 300])
def test_limb_rule_matches_oracle(K):
    mpts = _lib()
    p = mpts.Lorenz(K=K, N=10)
    assert p.L == make_context(K_digits=K, N=10).L


@pytest.mark.parametrize("L", [1, 2, 12, 208])
def test_parse_matches_oracle(L):
    mpts = _lib()
    p = mpts.Lorenz(L=L, N=3)
    for s in BENCH_X0 + ("8/3", "1/100", "-1e-30", "123456789.987654321e-7", "0", "-7/3"):
        o = parse(s, 32 * L)
        assert p.from_str(s) == tuple(o), s
    assert p.param(0) == tuple(parse("10", 32 * L))
    assert p.param(1) == tuple(parse("28", 32 * L))
    assert p.param(2) == tuple(parse("8/3", 32 * L))
    assert p.param(3) == tuple(parse("1/100", 32 * L))


def test_double_round_trip_and_export():
    mpts = _lib()
    p = mpts.Lorenz(L=12, N=3)
    for v in (0.1, -15.8, 1e-300, 5e-324, 1.7976931348623157e308, -2.5):
        bf = p.from_double(v)
        assert bf == tuple(from_fraction(Fraction(v), 384))
        assert p.to_double(bf) == v
    for s in ("1/3", "-2/7", "1e-310", "3e-324", "2e-324"):
        o = parse(s, 384)
        assert p.to_double(tuple(o)) == to_double(o), s


def test_invalid_arguments_fail_cleanly():
    mpts = _lib()
    with pytest.raises(mpts.MptsError):
        mpts.Lorenz(K=0, N=4)
    with pytest.raises(mpts.MptsError):
        mpts.Lorenz(K=10, N=0)
    with pytest.raises(mpts.MptsError):
        mpts.Lorenz(K=10, N=4, b="eight/3")
    p = mpts.Lorenz(L=4, N=3)
    with pytest.raises(mpts.MptsError):
        p.from_str("1/0")


def test_agreement_digits_exact():
    """The clean-numerical-simulation comparison of two states: -log10 of the
    largest relative difference, on the exact values."""
    from paper_1908_09301_amd.cns import agreement_digits
    one = (1, 1 << 63, -63)             # 1
    near = (1, (1 << 63) + 1, -63)      # 1 + 2^-63
    two = (1, 1 << 63, -62)             # 2
    assert agreement_digits([one, one, one], [one, one, one], 40.0) == 40.0
    d = agreement_digits([near, one, two], [one, one, two], 40.0)
    assert abs(d - 63 * 0.30102999566398120) < 1e-9
    assert agreement_digits([two, one, one], [one, one, one], 40.0) == 0.0


def test_error_paths_before_any_device_work():
    """Bad arguments are refused on the host with their codes: strings, sizes,
    unnormalised big-floats, a workspace smaller than the call needs."""
    import ctypes
    mpts = _lib()
    lib = mpts._lib
    h = ctypes.c_void_p()
    assert lib.mpts_create(b"10", b"28", b"8/3", 0, 40, b"1/100", ctypes.byref(h)) == mpts.MPTS_EINVAL
    assert lib.mpts_create(b"10", b"28", b"8/3", 100, 0, b"1/100", ctypes.byref(h)) == mpts.MPTS_EINVAL
    assert lib.mpts_create(b"1o", b"28", b"8/3", 100, 40, b"1/100", ctypes.byref(h)) == mpts.MPTS_EINVAL
    assert lib.mpts_create(b"10", b"28", b"8/0", 100, 40, b"1/100", ctypes.byref(h)) == mpts.MPTS_EINVAL
    p = mpts.Lorenz(K=100, N=40)
    x = mpts.BFArray(3, p.L)
    for j, v in enumerate(BENCH_X0):
        x.set(j, p.from_str(v))
    out = mpts.BFArray(3, p.L)
    need = p.workspace_bytes(10)
    # workspace one byte short: refused before any device call
    st = lib.mpts_integrate(p.handle, x.ptr(), 10, out.ptr(), None, ctypes.c_void_p(1 << 20),
                            need - 1, None, 0)
    assert st == mpts.MPTS_ENOSPC
    assert b"workspace" in lib.mpts_last_error(p.handle)
    # negative step count
    st = lib.mpts_integrate(p.handle, x.ptr(), -1, out.ptr(), None, ctypes.c_void_p(1 << 20),
                            need, None, 0)
    assert st == mpts.MPTS_EINVAL
    # an unnormalised mantissa (top bit clear) and a bad sign
    s, m, e = p.from_str("1.5")
    x.set(0, (s, m >> 1, e + 1))
    st = lib.mpts_integrate(p.handle, x.ptr(), 1, out.ptr(), None, ctypes.c_void_p(1 << 20),
                            need, None, 0)
    assert st == mpts.MPTS_EINVAL
    x.set(0, (s, m, e))
    x.arr[0].sign = 2
    st = lib.mpts_integrate(p.handle, x.ptr(), 1, out.ptr(), None, ctypes.c_void_p(1 << 20),
                            need, None, 0)
    assert st == mpts.MPTS_EINVAL
    # checkpoints without the flag, an unknown loss
    ck = mpts.BFArray(3 * 2, p.L)
    st = lib.mpts_integrate(p.handle, x.ptr(), 1, out.ptr(), ck.ptr(), ctypes.c_void_p(1 << 20),
                            need, None, 0)
    assert st == mpts.MPTS_EINVAL
    g = (ctypes.c_double * 6)()
    st = lib.mpts_grad(p.handle, x.ptr(), 1, 7, g, None, None, None, ctypes.c_void_p(1 << 20),
                       need, None)
    assert st == mpts.MPTS_EINVAL


def test_polynomial_systems_are_checked_on_the_host():
    """mpts_poly_create refuses bad terms and sizes and systems past its
    limits before any device work; a system's coefficients parse exactly
    like the oracle's."""
    from oracle.bigfloat import parse
    from workloads import POLY_SYSTEMS
    mpts = _lib()
    nvar, terms = POLY_SYSTEMS["rossler"]
    p = mpts.Poly(nvar, terms, L=4, N=10)
    for text in ("0.2", "-5.7", "1/3"):
        assert p.from_str(text) == tuple(parse(text, p.p))
    bad = [
        (3, [(3, "1", 0, -1)]),        # equation out of range
        (3, [(0, "1", 3, -1)]),        # variable out of range
        (3, [(0, "1", -1, 1)]),        # w without u
        (3, [(0, "x", 0, -1)]),        # not a number
        (0, []),                       # no variable
    ]
    for nv, ts in bad:
        with pytest.raises(mpts.MptsError) as ei:
            mpts.Poly(nv, ts, L=4, N=10)
        assert ei.value.code == mpts.MPTS_EINVAL, (nv, ts)
    limits = [
        (5, [(0, "1", 0, -1)]),                                                  # five variables
        (4, [(0, "1", u, w) for u in range(4) for w in range(u, 4)][:6]),        # six product pairs
        (1, [(0, "1", -1, -1), (0, "2", -1, -1)]),                               # two constants
        (2, [(0, c, 0, -1) for c in ("2", "3", "5", "7", "11")]),                # five non-unit products
    ]
    for nv, ts in limits:
        with pytest.raises(mpts.MptsError) as ei:
            mpts.Poly(nv, ts, L=4, N=10)
        assert ei.value.code == mpts.MPTS_EUNSUPPORTED, (nv, ts)
