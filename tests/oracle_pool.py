"""Oracle checks fanned out over the host's cores.

The GPU tests hand the oracle many independent checks: whole Taylor steps
F(s_n) == s_{n+1} (equations (2)-(3)), single index transitions of the
recursion (equation (3)) and Horner sums (equation (2)) of coefficients the
GPU returned.  Each check is a pure function of its inputs, so they run in
spawned worker processes (fresh interpreters that never touch the GPU), at
most one per host core and never more than 16.  Inputs that several checks
share (the coefficient lists of a step) go to a temporary pickle file that
each worker loads once.

Only tests use this module; it calls nothing but the oracle.
"""
import os
import pickle
import sys
import tempfile
from concurrent.futures import ProcessPoolExecutor
from multiprocessing import get_context

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MAX_WORKERS = 16


def n_workers() -> int:
    return max(1, min(MAX_WORKERS, os.cpu_count() or 1))


def _init(root):
    if root not in sys.path:
        sys.path.insert(0, root)
    if hasattr(sys, "set_int_max_str_digits"):
        sys.set_int_max_str_digits(0)


def make_pool(workers: int = 0) -> ProcessPoolExecutor:
    return ProcessPoolExecutor(max_workers=workers or n_workers(), mp_context=get_context("spawn"),
                               initializer=_init, initargs=(ROOT,))


_CTX = {}
_DATA = {}


def _ctx(L, N):
    from oracle import lorenz as lz
    if (L, N) not in _CTX:
        _CTX[(L, N)] = lz.make_context(L=L, N=N)
    return _CTX[(L, N)]


def _load(path):
    if path not in _DATA:
        with open(path, "rb") as f:
            _DATA.clear()
            _DATA[path] = pickle.load(f)
    return _DATA[path]


def _bf(v):
    from oracle.bigfloat import BF
    return BF(*v)


def step_task(L, N, n, state, expected):
    """n if the oracle's step from `state` differs from `expected`, else None."""
    from oracle import lorenz as lz
    ctx = _ctx(L, N)
    got = lz.step(ctx, tuple(_bf(v) for v in state))
    return None if [tuple(v) for v in got] == [tuple(v) for v in expected] else n


def transitions_task(L, N, path, indices):
    """The indices i (of `indices`) whose transition alpha, beta, gamma_{i+1}
    from the stored coefficients 0..i differs from the stored i+1."""
    from oracle import lorenz as lz
    ctx = _ctx(L, N)
    a, b, g = _load(path)
    bad = []
    for i in indices:
        ref = lz.next_coefficients(ctx, a, b, g, i)
        if (tuple(ref[0]), tuple(ref[1]), tuple(ref[2])) != (tuple(a[i + 1]), tuple(b[i + 1]),
                                                             tuple(g[i + 1])):
            bad.append(i)
    return bad


def horner_task(L, N, path, comp, expected):
    """True if the Horner sum of the stored coefficients of component comp
    (0 alpha, 1 beta, 2 gamma) equals `expected`."""
    from oracle import lorenz as lz
    ctx = _ctx(L, N)
    c = _load(path)[comp]
    return tuple(lz.horner(ctx, c)) == tuple(expected)


def store_coefficients(coefs) -> str:
    """Pickle (alpha, beta, gamma), lists of (s, m, e) tuples, to a temporary
    file and return its path (the caller deletes it)."""
    from oracle.bigfloat import BF
    data = tuple([BF(*v) for v in c] for c in coefs)
    fd, path = tempfile.mkstemp(suffix=".pkl", prefix="mpts_coefs_")
    with os.fdopen(fd, "wb") as f:
        pickle.dump(data, f, protocol=pickle.HIGHEST_PROTOCOL)
    return path


def chunked(seq, parts):
    """`seq` dealt round-robin into `parts` lists (costs grow with the index,
    so every list gets cheap and dear items)."""
    out = [[] for _ in range(parts)]
    for k, v in enumerate(seq):
        out[k % parts].append(v)
    return [o for o in out if o]


def run_task(L, N, x0, nsteps):
    """The oracle's final state after nsteps steps from x0 ((s, m, e) tuples)."""
    from oracle import lorenz as lz
    ctx = _ctx(L, N)
    fin = lz.integrate(ctx, tuple(_bf(v) for v in x0), nsteps)
    return [tuple(v) for v in fin]


def adjoint_task(L, N, x0, nsteps, loss="sqnorm"):
    """The oracle's final state and six p-bit gradients of `loss`."""
    from oracle import adjoint as oad
    ctx = _ctx(L, N)
    xT, g = oad.grad(ctx, tuple(_bf(v) for v in x0), nsteps, loss)
    return [tuple(v) for v in xT], [tuple(v) for v in g]
