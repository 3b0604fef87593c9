"""ctypes binding of libmpts.so (C ABI declared in include/mpts.h).

Argument marshalling only: numbers cross as (sign, mantissa, exponent)
Python integers with value sign * mantissa * 2**exponent; device memory comes
from PyTorch tensors and the stream is PyTorch's current stream.  Every step
of the computation runs in the HIP library; importing this module fails
loudly when the library is missing.
"""
import atexit
import ctypes
import os
from typing import List, Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpts.so")

MPTS_OK = 0
MPTS_EINVAL = -1
MPTS_ENOSPC = -2
MPTS_EHIP = -3
MPTS_ERANGE = -4
MPTS_EARCH = -5
MPTS_EUNSUPPORTED = -6
MPTS_CHECKPOINTS = 1
MPTS_GRAPH = 2
MPTS_AUTOTUNE = 4
MPTS_LOSS_SQNORM = 0
MPTS_LOSS_X = 1
MPTS_LOSS_Y = 2
MPTS_LOSS_Z = 3
LOSSES = {"sqnorm": MPTS_LOSS_SQNORM, "x": MPTS_LOSS_X, "y": MPTS_LOSS_Y, "z": MPTS_LOSS_Z}

# every symbol include/mpts.h declares
SYMBOLS = (
    "mpts_create", "mpts_create_limbs", "mpts_destroy", "mpts_limbs", "mpts_param",
    "mpts_bf_from_str", "mpts_bf_from_double", "mpts_bf_to_double", "mpts_set_schedule",
    "mpts_workspace_bytes", "mpts_state_bytes", "mpts_pack_state", "mpts_unpack_state",
    "mpts_integrate", "mpts_integrate_dev", "mpts_check", "mpts_coefficients",
    "mpts_batch_workspace_bytes", "mpts_integrate_batch", "mpts_grad",
    "mpts_grad_batch_workspace_bytes", "mpts_grad_batch", "mpts_release_caches",
    "mpts_probe_rate", "mpts_integrate_dev_noalloc", "mpts_strerror", "mpts_last_error",
    "mpts_poly_create", "mpts_poly_destroy", "mpts_poly_bf_from_str", "mpts_poly_integrate",
    "mpts_poly_coefficients", "mpts_poly_last_error",
)

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1908_09301_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)


class mpts_bf(ctypes.Structure):
    _fields_ = [("sign", ctypes.c_int32), ("exp", ctypes.c_int32),
                ("limbs", ctypes.POINTER(ctypes.c_uint32))]


_P = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u32 = ctypes.c_uint32
_sz = ctypes.c_size_t
_BFP = ctypes.POINTER(mpts_bf)

_lib.mpts_create.argtypes = [ctypes.c_char_p] * 3 + [_i32, _i32, ctypes.c_char_p, ctypes.POINTER(_P)]
_lib.mpts_create_limbs.argtypes = [ctypes.c_char_p] * 3 + [_i32, _i32, ctypes.c_char_p, ctypes.POINTER(_P)]
_lib.mpts_destroy.argtypes = [_P]
_lib.mpts_destroy.restype = None
_lib.mpts_limbs.argtypes = [_P, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32)]
_lib.mpts_param.argtypes = [_P, _i32, _BFP]
_lib.mpts_bf_from_str.argtypes = [_P, ctypes.c_char_p, _BFP]
_lib.mpts_bf_from_double.argtypes = [_P, ctypes.c_double, _BFP]
_lib.mpts_bf_to_double.argtypes = [_P, _BFP, ctypes.POINTER(ctypes.c_double)]
_lib.mpts_set_schedule.argtypes = [_P, _i32]
_lib.mpts_workspace_bytes.argtypes = [_P, _i64, _u32, ctypes.POINTER(_sz)]
_lib.mpts_state_bytes.argtypes = [_P, ctypes.POINTER(_sz)]
_lib.mpts_pack_state.argtypes = [_P, _BFP, _P]
_lib.mpts_unpack_state.argtypes = [_P, _P, _BFP]
_lib.mpts_integrate.argtypes = [_P, _BFP, _i64, _BFP, _BFP, _P, _sz, _P, _u32]
_lib.mpts_integrate_dev.argtypes = [_P, _P, _i64, _P, _P, _P, _sz, _P]
_lib.mpts_check.argtypes = [_P, _P, _P]
_lib.mpts_coefficients.argtypes = [_P, _BFP, _BFP, _BFP, _BFP, _P, _sz, _P]
_lib.mpts_batch_workspace_bytes.argtypes = [ctypes.POINTER(_P), _i32, ctypes.POINTER(_i64), _u32,
                                            ctypes.POINTER(_sz)]
_lib.mpts_integrate_batch.argtypes = [ctypes.POINTER(_P), _i32, _BFP, ctypes.POINTER(_i64), _BFP,
                                      _P, _sz, _P, _u32]
_DP = ctypes.POINTER(ctypes.c_double)
_lib.mpts_grad.argtypes = [_P, _BFP, _i64, _i32, _DP, _DP, _BFP, _BFP, _P, _sz, _P]
_lib.mpts_grad_batch_workspace_bytes.argtypes = [ctypes.POINTER(_P), _i32, ctypes.POINTER(_i64),
                                                 ctypes.POINTER(_sz)]
_lib.mpts_grad_batch.argtypes = [ctypes.POINTER(_P), _i32, _BFP, ctypes.POINTER(_i64), _i32, _DP,
                                 _DP, _BFP, _P, _sz, _P]
_lib.mpts_release_caches.argtypes = []
_lib.mpts_probe_rate.argtypes = [_i32, _DP, _P, _sz, _P]
_lib.mpts_integrate_dev_noalloc.argtypes = [_P, _P, _i64, _P, _P, _P]
_lib.mpts_strerror.argtypes = [_i32]
_lib.mpts_strerror.restype = ctypes.c_char_p
_lib.mpts_last_error.argtypes = [_P]
_lib.mpts_last_error.restype = ctypes.c_char_p


class mpts_poly_term(ctypes.Structure):
    _fields_ = [("eq", ctypes.c_int32), ("u", ctypes.c_int32), ("w", ctypes.c_int32),
                ("coef", ctypes.c_char_p)]


_lib.mpts_poly_create.argtypes = [_i32, ctypes.POINTER(mpts_poly_term), _i32, _i32, _i32,
                                  ctypes.c_char_p, ctypes.POINTER(_P)]
_lib.mpts_poly_destroy.argtypes = [_P]
_lib.mpts_poly_destroy.restype = None
_lib.mpts_poly_bf_from_str.argtypes = [_P, ctypes.c_char_p, _BFP]
_lib.mpts_poly_integrate.argtypes = [_P, _i32, _BFP, _i64, _BFP, _P]
_lib.mpts_poly_coefficients.argtypes = [_P, _BFP, _BFP, _P]
_lib.mpts_poly_last_error.argtypes = [_P]
_lib.mpts_poly_last_error.restype = ctypes.c_char_p


# Orderly shutdown: at interpreter exit, before the HIP runtime and the
# library's code objects are torn down, the cached batch graphs are
# destroyed; from then on no context destructor calls into the library.  The
# state is bound into Lorenz.__del__ as a default argument, so it is still
# reachable while the interpreter clears this module's globals.
_STATE = {"closed": False, "lib": _lib}


def _shutdown(state=_STATE):
    state["lib"].mpts_release_caches()
    state["closed"] = True


atexit.register(_shutdown)


class MptsError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        self.code = code
        text = _lib.mpts_strerror(code).decode()
        super().__init__(f"{text} ({code})" + (f": {msg}" if msg else ""))


def exported_symbols() -> List[str]:
    return [s for s in SYMBOLS if hasattr(_lib, s)]


def _bytes(s) -> bytes:
    return str(s).encode()


class BFArray:
    """Caller-owned storage for n big-floats of L limbs each."""

    def __init__(self, n: int, L: int):
        self.n, self.L = n, L
        self.store = (ctypes.c_uint32 * (n * L))()
        self.arr = (mpts_bf * n)()
        base = ctypes.addressof(self.store)
        for j in range(n):
            self.arr[j].limbs = ctypes.cast(base + 4 * L * j, ctypes.POINTER(ctypes.c_uint32))

    def set(self, j: int, v: Tuple[int, int, int]):
        s, m, e = v
        self.arr[j].sign = s
        self.arr[j].exp = e if s else 0
        for k in range(self.L):
            self.store[j * self.L + k] = (m >> (32 * k)) & 0xFFFFFFFF

    def get(self, j: int) -> Tuple[int, int, int]:
        b = self.arr[j]
        m = 0
        for k in range(self.L - 1, -1, -1):
            m = (m << 32) | self.store[j * self.L + k]
        if b.sign == 0:
            return (0, 0, 0)
        return (int(b.sign), m, int(b.exp))

    def ptr(self, j: int = 0):
        return ctypes.cast(ctypes.byref(self.arr, j * ctypes.sizeof(mpts_bf)), _BFP)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _workspace(nbytes: int):
    import torch
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda")


class Lorenz:
    """One problem definition: Lorenz parameters (equation (1)), Taylor
    order N and step tau (equation (2)), precision K decimal digits or L
    limbs."""

    def __init__(self, K: Optional[int] = None, N: int = 40, L: Optional[int] = None,
                 sigma: str = "10", R: str = "28", b: str = "8/3", tau: str = "1/100"):
        h = _P()
        if L is not None:
            st = _lib.mpts_create_limbs(_bytes(sigma), _bytes(R), _bytes(b), L, N, _bytes(tau),
                                        ctypes.byref(h))
        else:
            st = _lib.mpts_create(_bytes(sigma), _bytes(R), _bytes(b), K, N, _bytes(tau),
                                  ctypes.byref(h))
        if st != MPTS_OK:
            raise MptsError(st)
        self._h = h
        Lc, pc, Nc = _i32(), _i32(), _i32()
        _lib.mpts_limbs(h, ctypes.byref(Lc), ctypes.byref(pc), ctypes.byref(Nc))
        self.L, self.p, self.N = Lc.value, pc.value, Nc.value
        self._ws = None

    def __del__(self, _state=_STATE):
        h = getattr(self, "_h", None)
        self._h = None
        if h and not _state["closed"]:
            _state["lib"].mpts_destroy(h)

    @property
    def handle(self):
        return self._h

    def _check(self, st: int):
        if st != MPTS_OK:
            raise MptsError(st, _lib.mpts_last_error(self._h).decode())

    # -- numbers ----------------------------------------------------------
    def param(self, which: int) -> Tuple[int, int, int]:
        a = BFArray(1, self.L)
        self._check(_lib.mpts_param(self._h, which, a.ptr()))
        return a.get(0)

    def from_str(self, s: str) -> Tuple[int, int, int]:
        a = BFArray(1, self.L)
        self._check(_lib.mpts_bf_from_str(self._h, _bytes(s), a.ptr()))
        return a.get(0)

    def from_double(self, v: float) -> Tuple[int, int, int]:
        a = BFArray(1, self.L)
        self._check(_lib.mpts_bf_from_double(self._h, ctypes.c_double(v), a.ptr()))
        return a.get(0)

    def to_double(self, v: Tuple[int, int, int]) -> float:
        a = BFArray(1, self.L)
        a.set(0, v)
        out = ctypes.c_double()
        self._check(_lib.mpts_bf_to_double(self._h, a.ptr(), ctypes.byref(out)))
        return out.value

    def set_schedule(self, workgroups: int):
        self._check(_lib.mpts_set_schedule(self._h, workgroups))

    # -- device -----------------------------------------------------------
    def workspace_bytes(self, nsteps: int, flags: int = 0) -> int:
        n = _sz()
        self._check(_lib.mpts_workspace_bytes(self._h, nsteps, flags, ctypes.byref(n)))
        return n.value

    def workspace(self, nsteps: int, flags: int = 0):
        need = self.workspace_bytes(nsteps, flags)
        if self._ws is None or self._ws.numel() < need:
            self._ws = _workspace(need)
        return self._ws

    def state_bytes(self) -> int:
        n = _sz()
        self._check(_lib.mpts_state_bytes(self._h, ctypes.byref(n)))
        return n.value

    def pack_state(self, x: Sequence[Tuple[int, int, int]]):
        """Packed device-format state as a CPU int32 tensor."""
        import torch
        a = BFArray(3, self.L)
        for j in range(3):
            a.set(j, x[j])
        t = torch.zeros(self.state_bytes() // 4, dtype=torch.int32)
        self._check(_lib.mpts_pack_state(self._h, a.ptr(), ctypes.c_void_p(t.data_ptr())))
        return t

    def unpack_state(self, t) -> List[Tuple[int, int, int]]:
        t = t.cpu().contiguous()
        a = BFArray(3, self.L)
        self._check(_lib.mpts_unpack_state(self._h, ctypes.c_void_p(t.data_ptr()), a.ptr()))
        return [a.get(j) for j in range(3)]

    def integrate(self, x0, nsteps: int, checkpoints: bool = False):
        """Final state after nsteps Taylor steps (and all states with
        checkpoints=True)."""
        flags = MPTS_CHECKPOINTS if checkpoints else 0
        ws = self.workspace(nsteps, flags)
        a = BFArray(3, self.L)
        for j in range(3):
            a.set(j, x0[j])
        out = BFArray(3, self.L)
        ck = BFArray(3 * (nsteps + 1), self.L) if checkpoints else None
        self._check(_lib.mpts_integrate(self._h, a.ptr(), nsteps, out.ptr(),
                                        ck.ptr() if ck else None,
                                        ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(), flags))
        res = [out.get(j) for j in range(3)]
        if checkpoints:
            states = [[ck.get(3 * n + j) for j in range(3)] for n in range(nsteps + 1)]
            return res, states
        return res

    def integrate_dev(self, x0_dev, nsteps: int, xout_dev, ckpt_dev=None, ws=None):
        """Asynchronous device-resident run on the current stream; x0_dev and
        xout_dev are int32 CUDA tensors in the packed state format."""
        if ws is None:
            ws = self.workspace(nsteps)
        self._check(_lib.mpts_integrate_dev(
            self._h, ctypes.c_void_p(x0_dev.data_ptr()), nsteps, ctypes.c_void_p(xout_dev.data_ptr()),
            ctypes.c_void_p(ckpt_dev.data_ptr()) if ckpt_dev is not None else None,
            ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
        return ws

    def integrate_dev_noalloc(self, x0_dev, nsteps: int, xout_dev, ckpt_dev=None):
        """As integrate_dev with the library's own device scratch array as
        the workspace (no allocation); errors from the device through
        check(None)."""
        self._check(_lib.mpts_integrate_dev_noalloc(
            self._h, ctypes.c_void_p(x0_dev.data_ptr()), nsteps, ctypes.c_void_p(xout_dev.data_ptr()),
            ctypes.c_void_p(ckpt_dev.data_ptr()) if ckpt_dev is not None else None, _stream()))

    def check(self, ws):
        """Device status of the last call on workspace ws (None: of the last
        allocation-free call on this device)."""
        self._check(_lib.mpts_check(self._h, ctypes.c_void_p(ws.data_ptr()) if ws is not None
                                    else None, _stream()))

    def coefficients(self, x0):
        """Taylor coefficients (alpha, beta, gamma), each N+1 values, of one
        step from x0."""
        ws = self.workspace(1)
        a = BFArray(3, self.L)
        for j in range(3):
            a.set(j, x0[j])
        outs = [BFArray(self.N + 1, self.L) for _ in range(3)]
        self._check(_lib.mpts_coefficients(self._h, a.ptr(), outs[0].ptr(), outs[1].ptr(),
                                           outs[2].ptr(), ctypes.c_void_p(ws.data_ptr()),
                                           ws.numel(), _stream()))
        return tuple([o.get(i) for i in range(self.N + 1)] for o in outs)

    def grad(self, x0, nsteps: int, loss: str = "sqnorm"):
        """Gradient of a loss of x(T) ("sqnorm": ||x(T)||^2; "x", "y", "z": one
        component) w.r.t. (x0, y0, z0, sigma, R, b): returns (6 doubles,
        6 big-floats, final state, loss as a double)."""
        ws = self.workspace(nsteps, MPTS_CHECKPOINTS)
        a = BFArray(3, self.L)
        for j in range(3):
            a.set(j, x0[j])
        g = (ctypes.c_double * 6)()
        lv = ctypes.c_double()
        gb = BFArray(6, self.L)
        out = BFArray(3, self.L)
        self._check(_lib.mpts_grad(self._h, a.ptr(), nsteps, LOSSES[loss], g, ctypes.byref(lv),
                                   gb.ptr(), out.ptr(), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                   _stream()))
        return list(g), [gb.get(j) for j in range(6)], [out.get(j) for j in range(3)], lv.value


MPTS_PROBE_VALU_MAD = 0
MPTS_PROBE_MFMA_I8 = 1


def probe_rate(unit: int) -> float:
    """Measured multiply-adds per second of one arithmetic unit
    (MPTS_PROBE_VALU_MAD or MPTS_PROBE_MFMA_I8) on the current device."""
    import torch
    n = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    out = _workspace(8 * 1024 * n)
    v = ctypes.c_double()
    st = _lib.mpts_probe_rate(unit, ctypes.byref(v), ctypes.c_void_p(out.data_ptr()), out.numel(),
                              _stream())
    if st != MPTS_OK:
        raise MptsError(st)
    return v.value


def _batch_bfs(problems, x0s):
    """mpts_bf arrays of the initial states and of room for the final states
    (each trajectory with its own limb count), and the storage they use."""
    n = len(problems)
    ins = (mpts_bf * (3 * n))()
    outs = (mpts_bf * (3 * n))()
    keep = []
    for t, p in enumerate(problems):
        for j in range(3):
            s, m, e = x0s[t][j]
            buf = (ctypes.c_uint32 * p.L)(*[(m >> (32 * k)) & 0xFFFFFFFF for k in range(p.L)])
            ob = (ctypes.c_uint32 * p.L)()
            keep += [buf, ob]
            ins[3 * t + j].sign, ins[3 * t + j].exp = s, (e if s else 0)
            ins[3 * t + j].limbs = ctypes.cast(buf, ctypes.POINTER(ctypes.c_uint32))
            outs[3 * t + j].limbs = ctypes.cast(ob, ctypes.POINTER(ctypes.c_uint32))
    return ins, outs, keep


def _batch_states(problems, outs):
    res = []
    for t, p in enumerate(problems):
        r = []
        for j in range(3):
            b = outs[3 * t + j]
            m = 0
            for k in range(p.L - 1, -1, -1):
                m = (m << 32) | b.limbs[k]
            r.append((int(b.sign), m, int(b.exp)) if b.sign else (0, 0, 0))
        res.append(r)
    return res


def _limbs_for_digits(K: int) -> int:
    """The library's limb count for K decimal digits (from a throwaway
    context; no device work)."""
    h = _P()
    st = _lib.mpts_create(b"10", b"28", b"8/3", K, 1, b"1/100", ctypes.byref(h))
    if st != MPTS_OK:
        raise MptsError(st)
    L = _i32()
    _lib.mpts_limbs(h, ctypes.byref(L), None, None)
    _lib.mpts_destroy(h)
    return L.value


class Poly:
    """A polynomial vector field of degree at most two: `nvar` variables and
    terms (eq, coef, u, w) meaning coef * x_u * x_w in dx_eq/dt (u, w = -1:
    absent); order N, step tau, precision K decimal digits or L limbs."""

    def __init__(self, nvar: int, terms, K: Optional[int] = None, N: int = 40,
                 L: Optional[int] = None, tau: str = "1/100"):
        if L is None:
            L = _limbs_for_digits(K)
        self.nvar, self.L, self.p, self.N = nvar, L, 32 * L, N
        self._coefs = [_bytes(t[1]) for t in terms]  # kept alive during the call
        arr = (mpts_poly_term * max(len(terms), 1))()
        for j, (eq, coef, u, w) in enumerate(terms):
            arr[j].eq, arr[j].u, arr[j].w, arr[j].coef = eq, u, w, self._coefs[j]
        h = _P()
        st = _lib.mpts_poly_create(nvar, arr, len(terms), L, N, _bytes(tau), ctypes.byref(h))
        if st != MPTS_OK:
            raise MptsError(st)
        self._h = h

    def __del__(self, _state=_STATE):
        h = getattr(self, "_h", None)
        self._h = None
        if h and not _state["closed"]:
            _state["lib"].mpts_poly_destroy(h)

    def _check(self, st: int):
        if st != MPTS_OK:
            raise MptsError(st, _lib.mpts_poly_last_error(self._h).decode())

    def from_str(self, s: str) -> Tuple[int, int, int]:
        a = BFArray(1, self.L)
        self._check(_lib.mpts_poly_bf_from_str(self._h, _bytes(s), a.ptr()))
        return a.get(0)

    def integrate(self, x0s, nsteps: int):
        """`nsteps` steps of every trajectory in x0s (a list of nvar-tuples
        of (sign, mantissa, exponent)) in one launch."""
        n = len(x0s)
        a = BFArray(n * self.nvar, self.L)
        out = BFArray(n * self.nvar, self.L)
        for t, x in enumerate(x0s):
            for v in range(self.nvar):
                a.set(t * self.nvar + v, x[v])
        self._check(_lib.mpts_poly_integrate(self._h, n, a.ptr(), nsteps, out.ptr(), _stream()))
        return [tuple(out.get(t * self.nvar + v) for v in range(self.nvar)) for t in range(n)]

    def coefficients(self, x0):
        """The Taylor coefficients of one step: nvar lists of N+1 values."""
        a = BFArray(self.nvar, self.L)
        for v in range(self.nvar):
            a.set(v, x0[v])
        c = BFArray(self.nvar * (self.N + 1), self.L)
        self._check(_lib.mpts_poly_coefficients(self._h, a.ptr(), c.ptr(), _stream()))
        return [[c.get(v * (self.N + 1) + i) for i in range(self.N + 1)] for v in range(self.nvar)]


def integrate_batch(problems: Sequence[Lorenz], x0s, nsteps: Sequence[int], flags: int = 0):
    """Run many trajectories (each with its own K, N) in one persistent
    launch; returns the final states."""
    n = len(problems)
    hs = (_P * n)(*[p.handle for p in problems])
    ns = (_i64 * n)(*nsteps)
    need = _sz()
    st = _lib.mpts_batch_workspace_bytes(hs, n, ns, flags, ctypes.byref(need))
    if st != MPTS_OK:
        raise MptsError(st)
    ws = _workspace(need.value)
    ins, outs, keep = _batch_bfs(problems, x0s)
    st = _lib.mpts_integrate_batch(hs, n, ins, ns, outs, ctypes.c_void_p(ws.data_ptr()),
                                   ws.numel(), _stream(), flags)
    if st != MPTS_OK:
        raise MptsError(st, _lib.mpts_last_error(problems[0].handle).decode())
    del keep
    return _batch_states(problems, outs)


def grad_batch(problems: Sequence[Lorenz], x0s, nsteps: Sequence[int], loss: str = "sqnorm"):
    """Gradients of many trajectories (each with its own K, N) in one forward
    and one reverse launch; returns (grads: count lists of 6 doubles,
    losses: count doubles, final states)."""
    n = len(problems)
    hs = (_P * n)(*[p.handle for p in problems])
    ns = (_i64 * n)(*nsteps)
    need = _sz()
    st = _lib.mpts_grad_batch_workspace_bytes(hs, n, ns, ctypes.byref(need))
    if st != MPTS_OK:
        raise MptsError(st)
    ws = _workspace(need.value)
    ins, outs, keep = _batch_bfs(problems, x0s)
    g = (ctypes.c_double * (6 * n))()
    lv = (ctypes.c_double * n)()
    st = _lib.mpts_grad_batch(hs, n, ins, ns, LOSSES[loss], g, lv, outs,
                              ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream())
    if st != MPTS_OK:
        raise MptsError(st, _lib.mpts_last_error(problems[0].handle).decode())
    del keep
    return ([list(g[6 * t:6 * t + 6]) for t in range(n)], list(lv),
            _batch_states(problems, outs))


def _make_sqnorm_function():
    import torch

    class LorenzSqNorm(torch.autograd.Function):
        """loss = ||x(T)||^2 after `nsteps` Taylor steps of `problem` from x0.

        Inputs: x0, a float64 tensor of 3 values (taken exactly), and params,
        a float64 tensor (sigma, R, b) that must equal the problem's own
        parameters to double precision; the arithmetic uses the problem's
        p-bit parameters (b = 8/3 rounded to p bits, not its double).  The
        forward value is the library's FP64 rounding of the exact loss of the
        p-bit state; backward returns grad_output times the p-bit gradient rounded
        to FP64, for x0 and for params (the b derivative taken at the p-bit b).
        """

        @staticmethod
        def forward(ctx, x0, params, problem, nsteps):
            xs = [problem.from_double(float(v)) for v in x0.detach().cpu().tolist()]
            want = [problem.to_double(problem.param(j)) for j in range(3)]
            got = [float(v) for v in params.detach().cpu().tolist()]
            if got != want:
                raise ValueError(f"params {got} differ from the problem's {want}")
            g64, _, _, loss = problem.grad(xs, nsteps, "sqnorm")
            ctx.save_for_backward(torch.tensor(g64, dtype=torch.float64))
            return torch.tensor(loss, dtype=torch.float64, device=x0.device)

        @staticmethod
        def backward(ctx, grad_out):
            (g,) = ctx.saved_tensors
            go = grad_out.detach().to("cpu", torch.float64)
            return (go * g[:3]).to(grad_out.device), (go * g[3:]).to(grad_out.device), None, None

    return LorenzSqNorm


class _Lazy:
    fn = None


def LorenzSqNorm():
    """The torch.autograd.Function for ||x(T)||^2 (created on first use)."""
    if _Lazy.fn is None:
        _Lazy.fn = _make_sqnorm_function()
    return _Lazy.fn
