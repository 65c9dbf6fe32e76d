"""Thin Python binding of libmdwf (the C ABI declared in include/mdwf.h).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  torch tensors provide device memory (``complex128``,
contiguous, user layout ``[rhs][s][t][z][y][x][spin][colour]``) and the
stream; torch does no arithmetic here.  If the library has not been built the
first call raises ``MDWFError`` -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
# MDWF_LIB_PATH selects another build of the library (e.g. a variant being compared)
LIB_PATH = os.environ.get("MDWF_LIB_PATH") or os.path.join(_HERE, "libmdwf.so")

# status codes
OK, EINVAL, ENOMEM, EHIP, ENOCONV, EBREAKDOWN, ENAN, EBUSY = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENOCONV", -5: "EBREAKDOWN",
                -6: "ENAN", -7: "EBUSY"}
# precisions
F64, F32, F16, BF16, I16 = 0, 1, 2, 3, 4
PREC = {"f64": F64, "f32": F32, "f16": F16, "bf16": BF16, "i16": I16}
# operators
(OP_D, OP_DDAG, OP_MHAT, OP_MHATDAG, OP_NORMAL, OP_HOP_EO, OP_HOP_OE, OP_HOP, OP_HOPDAG, OP_M5,
 OP_M5INV, OP_MPHI, OP_PREP) = range(13)
HOST, DEVICE = 0, 1
# profile classes
PROF_DSLASH_INNER, PROF_DSLASH_F64, PROF_BLAS, PROF_SCALAR, PROF_OTHER = range(5)


class MDWFError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Action(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4), ("L5", ctypes.c_int32), ("t_antiperiodic", ctypes.c_int32),
                ("b5", ctypes.c_double), ("c5", ctypes.c_double), ("M5", ctypes.c_double), ("mq", ctypes.c_double)]

    @classmethod
    def make(cls, L, L5, b5=1.5, c5=0.5, M5=1.3, mq=0.05, t_antiperiodic=1):
        a = cls()
        for i in range(4):
            a.L[i] = int(L[i])
        a.L5 = int(L5)
        a.t_antiperiodic = int(t_antiperiodic)
        a.b5, a.c5, a.M5, a.mq = float(b5), float(c5), float(M5), float(mq)
        return a

    @property
    def lattice(self):
        return tuple(self.L[i] for i in range(4))

    def spinor_shape(self, nrhs=None):
        Lx, Ly, Lz, Lt = self.lattice
        shape = (self.L5, Lt, Lz, Ly, Lx, 4, 3)
        return shape if nrhs is None else (nrhs,) + shape


class CGOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("delta", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("inner", ctypes.c_int32), ("use_initial_guess", ctypes.c_int32), ("check_every", ctypes.c_int32)]

    # reliable-update threshold by inner precision (measured on 16^3x32,
    # 24^3x64 and 32^3x64): an FP32 iteration keeps ~7 digits, and letting its
    # residual fall 3000x between FP64 updates leaves the iteration count
    # unchanged with 3-4 updates instead of 5 (+1-4 % solves/s over 100x);
    # FP16 and int16 storage (~3-4 digits) update every 10x; BF16 (~2 digits)
    # every 3x: at 10x its c3 solve needed 1253 iterations, at 3x 283
    DEFAULT_DELTA = {F64: 0.1, F32: 3e-4, F16: 0.1, BF16: 0.3, I16: 0.1}

    @classmethod
    def make(cls, tol=1e-10, inner=F64, delta=None, max_iter=100000, use_initial_guess=0, check_every=0):
        o = cls()
        o.inner = PREC[inner] if isinstance(inner, str) else int(inner)
        if delta is None:
            delta = cls.DEFAULT_DELTA.get(o.inner, 0.1)
        o.tol, o.delta, o.max_iter = float(tol), float(delta), int(max_iter)
        o.use_initial_guess, o.check_every = int(use_initial_guess), int(check_every)
        return o


class CGStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("converged", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("reliable_updates", ctypes.c_int32), ("rel_res_normal", ctypes.c_double),
                ("rel_res_full", ctypes.c_double), ("seconds", ctypes.c_double), ("bytes", ctypes.c_double),
                ("flops", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int32
_SIGS = {
    "mdwf_abi_version": (_I, []),
    "mdwf_check_action": (_I, [ctypes.POINTER(Action), ctypes.c_char_p, ctypes.c_size_t]),
    "mdwf_copy_bandwidth": (_I, [_P, _P, _P, ctypes.c_size_t, _I, ctypes.POINTER(ctypes.c_double)]),
    "mdwf_query_traversal": (_I, [ctypes.POINTER(Action), _I, _I, _I, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "mdwf_create": (_I, [_I, _P, ctypes.POINTER(_P)]),
    "mdwf_destroy": (_I, [_P]),
    "mdwf_trim": (_I, [_P]),
    "mdwf_last_error": (ctypes.c_char_p, [_P]),
    "mdwf_stream": (_P, [_P]),
    "mdwf_gauge_load": (_I, [_P, ctypes.POINTER(_I), _P, _I, ctypes.c_uint32, ctypes.POINTER(_P)]),
    "mdwf_gauge_free": (_I, [_P]),
    "mdwf_gauge_bytes": (ctypes.c_size_t, [_P]),
    "mdwf_source_point": (_I, [_P, ctypes.POINTER(Action), ctypes.POINTER(_I), _I, _I, _P]),
    "mdwf_source_z2": (_I, [_P, ctypes.POINTER(Action), ctypes.c_uint64, _I, _P]),
    "mdwf_propagator_4d": (_I, [_P, ctypes.POINTER(Action), _I, _P, _P]),
    "mdwf_dslash_noalloc": (_I, [_P, _P, ctypes.POINTER(Action), _I, _I, _I, _P, _P]),
    "mdwf_source_physical": (_I, [_P, _P, ctypes.POINTER(Action), _I, _I, _P, _P]),
    "mdwf_current_source": (_I, [_P, ctypes.POINTER(Action), _I, _I, _P, _P]),
    "mdwf_dslash": (_I, [_P, _P, ctypes.POINTER(Action), _I, _I, _I, _P, _P]),
    "mdwf_hop_split": (_I, [_P, _P, ctypes.POINTER(Action), _I, _I, _I, _P, _P, ctypes.POINTER(ctypes.c_double)]),
    "mdwf_solve": (_I, [_P, _P, ctypes.POINTER(Action), ctypes.POINTER(CGOpts), _I, _P, _P,
                        ctypes.POINTER(CGStats)]),
    "mdwf_job_footprint": (ctypes.c_size_t, [ctypes.POINTER(Action), ctypes.POINTER(CGOpts), _I]),
    "mdwf_job_begin": (_I, [_P, _P, ctypes.POINTER(Action), ctypes.POINTER(CGOpts), _I, _P, _P,
                            ctypes.POINTER(_P)]),
    "mdwf_job_step": (_I, [_P, ctypes.POINTER(_P), _I, _I]),
    "mdwf_job_poll": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(CGStats)]),
    "mdwf_job_end": (_I, [_P]),
    "mdwf_profile_enable": (_I, [_P, _I]),
    "mdwf_profile_reset": (_I, [_P]),
    "mdwf_profile_read": (_I, [_P, _I, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_double)]),
    "mdwf_tune_mode": (_I, [_P, _I]),
    "mdwf_tune_save": (_I, [_P, ctypes.c_char_p]),
    "mdwf_tune_load": (_I, [_P, ctypes.c_char_p]),
    "mdwf_tune_entries": (_I, [_P]),
}


def lib():
    """Load libmdwf.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MDWFError(EHIP, f"{LIB_PATH} is not built (python -m paper_1810_01609_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check_action(act: Action):
    """Host-only validation; returns (status, message)."""
    buf = ctypes.create_string_buffer(256)
    st = lib().mdwf_check_action(ctypes.byref(act), buf, len(buf))
    return st, buf.value.decode()


def query_traversal(act: Action, prec, nrhs: int = 1, cb_log2: int = 4):
    """Host-only: (Bt, y-bands) of the stencil traversal for this action,
    precision and RHS count (environment overrides applied)."""
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    bt, yb = _I(), _I()
    st = lib().mdwf_query_traversal(ctypes.byref(act), p, int(nrhs), int(cb_log2), ctypes.byref(bt), ctypes.byref(yb))
    if st != OK:
        raise MDWFError(st, "mdwf_query_traversal: bad argument")
    return bt.value, yb.value


def job_footprint(act: Action, opts: CGOpts, nrhs: int) -> int:
    return int(lib().mdwf_job_footprint(ctypes.byref(act), ctypes.byref(opts), int(nrhs)))


def _ptr(t, nbytes=None, what="tensor"):
    """Device pointer of a contiguous complex128 torch tensor (checked)."""
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{what} must live on the GPU")
    if t.dtype != torch.complex128:
        raise ValueError(f"{what} must be complex128")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if nbytes is not None and t.numel() * 16 != nbytes:
        raise ValueError(f"{what} has {t.numel() * 16} bytes, expected {nbytes}")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One device + one stream.  By default it adopts torch's current stream,
    so library work is ordered with the torch operations around it."""

    def __init__(self, device: int = 0, stream=None, use_torch_stream: bool = True):
        self._h = ctypes.c_void_p()
        if stream is None and use_torch_stream:
            import torch

            stream = torch.cuda.current_stream(device).cuda_stream
        st = lib().mdwf_create(int(device), ctypes.c_void_p(stream) if stream else None, ctypes.byref(self._h))
        if st != OK:
            raise MDWFError(st, f"mdwf_create(device={device}) failed")
        self.device = device

    @property
    def handle(self):
        return self._h

    def _check(self, st, what):
        if st != OK:
            msg = lib().mdwf_last_error(self._h)
            raise MDWFError(st, f"{what}: {msg.decode() if msg else ''}")

    def close(self):
        if self._h:
            lib().mdwf_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def trim(self):
        """Release the device memory the context keeps between calls."""
        self._check(lib().mdwf_trim(self._h), "mdwf_trim")

    def stream(self):
        return lib().mdwf_stream(self._h)

    # ---- gauge ----
    def gauge_load(self, L, links, precs=("f64",)):
        """links: numpy complex128 [t][z][y][x][mu][3][3] (host) or a torch tensor (device)."""
        import numpy as np

        mask = 0
        for p in precs:
            mask |= 1 << (PREC[p] if isinstance(p, str) else int(p))
        Larr = (ctypes.c_int32 * 4)(*[int(v) for v in L])
        h = ctypes.c_void_p()
        Lx, Ly, Lz, Lt = (int(v) for v in L)
        nbytes = Lx * Ly * Lz * Lt * 4 * 9 * 16
        if isinstance(links, np.ndarray):
            arr = np.ascontiguousarray(links, dtype=np.complex128)
            if arr.nbytes != nbytes:
                raise ValueError("links have the wrong size")
            st = lib().mdwf_gauge_load(self._h, Larr, arr.ctypes.data_as(ctypes.c_void_p), HOST, mask,
                                       ctypes.byref(h))
        else:
            st = lib().mdwf_gauge_load(self._h, Larr, _ptr(links, nbytes, "links"), DEVICE, mask, ctypes.byref(h))
        self._check(st, "mdwf_gauge_load")
        return Gauge(self, h, tuple(int(v) for v in L))

    # ---- sources ----
    def source_point(self, act: Action, x0, spin, colour, eta):
        x = (ctypes.c_int32 * 4)(*[int(v) for v in x0])
        nb = 16 * _numel(act)
        st = lib().mdwf_source_point(self._h, ctypes.byref(act), x, int(spin), int(colour), _ptr(eta, nb, "eta"))
        self._check(st, "mdwf_source_point")

    def source_z2(self, act: Action, seed, rhs_index, eta):
        nb = 16 * _numel(act)
        st = lib().mdwf_source_z2(self._h, ctypes.byref(act), ctypes.c_uint64(int(seed)), int(rhs_index),
                                  _ptr(eta, nb, "eta"))
        self._check(st, "mdwf_source_z2")

    # ---- Feynman-Hellmann sequential source ----
    def propagator_4d(self, act: Action, psi, q, nrhs: int = 1):
        """q = P- psi_0 + P+ psi_{L5-1} (device tensors: psi in the 5D user
        layout, q complex128 [rhs][t][z][y][x][4][3])."""
        n4 = _numel(act) // act.L5
        st = lib().mdwf_propagator_4d(self._h, ctypes.byref(act), int(nrhs), _ptr(psi, 16 * _numel(act) * nrhs, "psi"),
                                      _ptr(q, 16 * n4 * nrhs, "q"))
        self._check(st, "mdwf_propagator_4d")

    def current_source(self, act: Action, gamma_mask: int, q, eta, nrhs: int = 1):
        """eta = wall injection of Gamma q, Gamma = g_x^b0 g_y^b1 g_z^b2 g_t^b3."""
        n4 = _numel(act) // act.L5
        st = lib().mdwf_current_source(self._h, ctypes.byref(act), int(nrhs), int(gamma_mask),
                                       _ptr(q, 16 * n4 * nrhs, "q"), _ptr(eta, 16 * _numel(act) * nrhs, "eta"))
        self._check(st, "mdwf_current_source")

    def source_physical(self, gauge, act: Action, xi, eta, gamma_mask: int = 0, nrhs: int = 1):
        """eta = (1 - c5 D_W) inject(Gamma xi): the 5D source whose solution,
        read off the walls, is the physical 4D propagator S Gamma xi."""
        n4 = _numel(act) // act.L5
        st = lib().mdwf_source_physical(self._h, gauge.handle, ctypes.byref(act), int(nrhs), int(gamma_mask),
                                        _ptr(xi, 16 * n4 * nrhs, "xi"), _ptr(eta, 16 * _numel(act) * nrhs, "eta"))
        self._check(st, "mdwf_source_physical")

    # ---- operators ----
    def dslash(self, gauge, act: Action, op: int, prec, inp, out, nrhs: int = 1):
        p = PREC[prec] if isinstance(prec, str) else int(prec)
        nb = 16 * _numel(act) * nrhs
        st = lib().mdwf_dslash(self._h, gauge.handle, ctypes.byref(act), int(op), p, int(nrhs),
                               _ptr(inp, nb, "in"), _ptr(out, nb, "out"))
        self._check(st, "mdwf_dslash")

    def dslash_noalloc(self, gauge, act: Action, op: int, prec, inp, out, nrhs: int = 1):
        """mdwf_dslash_noalloc: the same operator with every temporary in the
        library's fixed per-GPU scratch (no device allocation)."""
        p = PREC[prec] if isinstance(prec, str) else int(prec)
        nb = 16 * _numel(act) * nrhs
        st = lib().mdwf_dslash_noalloc(self._h, gauge.handle, ctypes.byref(act), int(op), p, int(nrhs),
                                       _ptr(inp, nb, "in"), _ptr(out, nb, "out"))
        self._check(st, "mdwf_dslash_noalloc")

    def hop_split(self, gauge, act: Action, prec, split_mask: int, inp, out, nrhs: int = 1, timed: bool = False):
        """out_e = H_eo in_o as one rank of a domain-decomposed run computes it
        (pack faces, interior hop, exterior update; the lattice is its own
        neighbour in each split dimension).  With timed=True returns the GPU
        milliseconds of the three steps."""
        p = PREC[prec] if isinstance(prec, str) else int(prec)
        nb = 16 * _numel(act) * nrhs
        ms = (ctypes.c_double * 3)() if timed else None
        st = lib().mdwf_hop_split(self._h, gauge.handle, ctypes.byref(act), p, int(split_mask), int(nrhs),
                                  _ptr(inp, nb, "in"), _ptr(out, nb, "out"), ms)
        self._check(st, "mdwf_hop_split")
        return list(ms) if timed else None

    # ---- solve ----
    def solve(self, gauge, act: Action, opts: CGOpts, eta, psi, nrhs: int = 1, raise_on_fail=True):
        nb = 16 * _numel(act) * nrhs
        stats = (CGStats * nrhs)()
        st = lib().mdwf_solve(self._h, gauge.handle, ctypes.byref(act), ctypes.byref(opts), int(nrhs),
                              _ptr(eta, nb, "eta"), _ptr(psi, nb, "psi"), stats)
        out = [s.as_dict() for s in stats]
        if st != OK and raise_on_fail:
            self._check(st, "mdwf_solve")
        return out

    # ---- stepping interface ----
    def job_begin(self, gauge, act: Action, opts: CGOpts, eta, psi, nrhs: int = 1):
        nb = 16 * _numel(act) * nrhs
        h = ctypes.c_void_p()
        st = lib().mdwf_job_begin(self._h, gauge.handle, ctypes.byref(act), ctypes.byref(opts), int(nrhs),
                                  _ptr(eta, nb, "eta"), _ptr(psi, nb, "psi"), ctypes.byref(h))
        self._check(st, "mdwf_job_begin")
        return Job(self, h, nrhs, keep=(eta, psi))

    def job_step(self, jobs, iters: int):
        arr = (ctypes.c_void_p * len(jobs))(*[j.handle.value for j in jobs])
        return lib().mdwf_job_step(self._h, arr, len(jobs), int(iters))

    # ---- measurement ----
    def copy_bandwidth(self, src, dst, reps: int = 5) -> float:
        """GB/s (read + write) of the library's STREAM-style copy kernel
        moving src (a contiguous device tensor) into dst of the same size."""
        nb = src.numel() * src.element_size()
        if dst.numel() * dst.element_size() != nb:
            raise ValueError("copy_bandwidth: src and dst differ in size")
        g = ctypes.c_double()
        st = lib().mdwf_copy_bandwidth(self._h, _ptr(src, nb, "src"), _ptr(dst, nb, "dst"), nb, int(reps),
                                       ctypes.byref(g))
        self._check(st, "mdwf_copy_bandwidth")
        return g.value


    def profile_enable(self, on=True, sample: int = 1):
        """Kernel timing on/off; sample = N > 1 times one CG iteration in N."""
        mode = 0 if not on else max(int(sample), 1)
        self._check(lib().mdwf_profile_enable(self._h, mode), "mdwf_profile_enable")

    def profile_reset(self):
        self._check(lib().mdwf_profile_reset(self._h), "mdwf_profile_reset")

    def profile_read(self, cls: int):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        b = ctypes.c_double()
        self._check(lib().mdwf_profile_read(self._h, int(cls), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(b)),
                    "mdwf_profile_read")
        return {"launches": n.value, "ms": ms.value, "bytes": b.value}

    # ---- tuning ----
    def tune_mode(self, mode: int):
        self._check(lib().mdwf_tune_mode(self._h, int(mode)), "mdwf_tune_mode")

    def tune_save(self, path):
        self._check(lib().mdwf_tune_save(self._h, str(path).encode()), "mdwf_tune_save")

    def tune_load(self, path):
        self._check(lib().mdwf_tune_load(self._h, str(path).encode()), "mdwf_tune_load")

    def tune_entries(self) -> int:
        return int(lib().mdwf_tune_entries(self._h))


def _numel(act: Action) -> int:
    Lx, Ly, Lz, Lt = act.lattice
    return Lx * Ly * Lz * Lt * act.L5 * 12


@dataclass
class Gauge:
    ctx: Context
    _h: ctypes.c_void_p
    L: tuple

    @property
    def handle(self):
        return self._h

    @property
    def nbytes(self):
        return int(lib().mdwf_gauge_bytes(self._h))

    def free(self):
        if self._h:
            lib().mdwf_gauge_free(self._h)
            self._h = ctypes.c_void_p()


class Job:
    def __init__(self, ctx: Context, h, nrhs, keep=()):
        self.ctx = ctx
        self._h = h
        self.nrhs = nrhs
        self._keep = keep  # keep eta / psi tensors alive while the job runs

    @property
    def handle(self):
        return self._h

    def poll(self):
        done = ctypes.c_int32()
        stats = (CGStats * self.nrhs)()
        lib().mdwf_job_poll(self._h, ctypes.byref(done), stats)
        return bool(done.value), [s.as_dict() for s in stats]

    def end(self):
        if self._h:
            lib().mdwf_job_end(self._h)
            self._h = ctypes.c_void_p()
        self._keep = ()  # the job no longer reads eta or writes psi
