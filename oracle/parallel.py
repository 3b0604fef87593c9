"""The oracle's coefficient recursion with the Cauchy sums split over worker
processes, the way the paper parallelises them (Section 4): every worker
owns a contiguous share of the terms k of each sum and returns its exact
partial sum (the paper's per-thread containers), and the master adds the
partials and rounds once.  Because the partials are exact, the bits are the
single-process oracle's (oracle.lorenz.coefficients) for any worker count;
the paper's own scheme rounds every GMP operation, which makes its results
depend on the thread count (Section 4), and that is not reproduced.

TEST INFRASTRUCTURE ONLY (the oracle's all-core timing on the host): nothing
in the product path uses it.
"""
import multiprocessing as mp
import os
import sys
from typing import List, Tuple

from .bigfloat import BF, exact_mul, exact_sum, round_exact
from .lorenz import Context, tails

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _worker(conn, root):
    if root not in sys.path:
        sys.path.insert(0, root)
    if hasattr(sys, "set_int_max_str_digits"):
        sys.set_int_max_str_digits(0)
    a: List[BF] = []
    b: List[BF] = []
    g: List[BF] = []
    while True:
        msg = conn.recv()
        op = msg[0]
        if op == "reset":
            a, b, g = [msg[1]], [msg[2]], [msg[3]]
        elif op == "append":
            a.append(msg[1])
            b.append(msg[2])
            g.append(msg[3])
        elif op == "sums":
            # exact partial sums over k in [k0, k1) of index i
            _, i, k0, k1 = msg
            p1 = exact_sum([exact_mul(a[i - k], g[k]) for k in range(k0, k1)])
            p2 = exact_sum([exact_mul(a[i - k], b[k]) for k in range(k0, k1)])
            conn.send((p1, p2))
        else:
            conn.close()
            return


class ParallelOracle:
    """Coefficients of one step (equation (3)) with each Cauchy sum split
    over `workers` processes (spawned fresh; they never touch a GPU)."""

    def __init__(self, ctx: Context, workers: int):
        self.ctx = ctx
        self.workers = max(1, workers)
        mpc = mp.get_context("spawn")
        self.conns, self.procs = [], []
        for _ in range(self.workers):
            here, there = mpc.Pipe()
            proc = mpc.Process(target=_worker, args=(there, _ROOT), daemon=True)
            proc.start()
            self.conns.append(here)
            self.procs.append(proc)

    def close(self):
        for c in self.conns:
            try:
                c.send(("stop",))
            except (BrokenPipeError, OSError):
                pass
        for p in self.procs:
            p.join(timeout=5)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _sums(self, i: int) -> Tuple[BF, BF]:
        """s1_i, s2_i: the workers' exact partials over near-equal k-chunks
        (the paper's schedule of the loop over k), added and rounded once."""
        n = i + 1
        parts = []
        for w, c in enumerate(self.conns):
            k0, k1 = n * w // self.workers, n * (w + 1) // self.workers
            if k1 > k0:
                c.send(("sums", i, k0, k1))
                parts.append(c)
        got = [c.recv() for c in parts]
        p = self.ctx.p
        s1 = round_exact(exact_sum([q[0] for q in got]), p)
        s2 = round_exact(exact_sum([q[1] for q in got]), p)
        return s1, s2

    def coefficients(self, state, upto: int = None):
        """alpha, beta, gamma for indices 0..upto (default N) from `state`."""
        ctx = self.ctx
        N = ctx.N if upto is None else upto
        a, b, g = [state[0]], [state[1]], [state[2]]
        for c in self.conns:
            c.send(("reset", state[0], state[1], state[2]))
        for i in range(N):
            s1, s2 = self._sums(i)
            an, bn, gn = tails(ctx, a, b, g, i, s1, s2)
            a.append(an)
            b.append(bn)
            g.append(gn)
            for c in self.conns:
                c.send(("append", an, bn, gn))
        return a, b, g
