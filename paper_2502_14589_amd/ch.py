"""Python binding of libch (include/ch.h): argument marshalling only.

Fields are torch tensors on the GPU (float64, contiguous, n**dim values,
x fastest); every computation runs in the HIP kernels of libch.so.  There is
no CPU fallback: a missing library raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from ctypes import POINTER, byref, c_double, c_int, c_longlong, c_void_p
from dataclasses import dataclass

# CH_LIB_PATH selects another build of the same library (e.g. to compare two builds on one GPU).
LIB_PATH = os.environ.get("CH_LIB_PATH") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libch.so")

CH_OK, CH_EINVAL, CH_ENOMEM, CH_ENONFINITE, CH_ETAU_UNDERFLOW, CH_EBUSY, CH_ENOENT, CH_EDEVICE = 0, -1, -2, -3, -4, -5, -6, -7
CH_FP64, CH_FP32_MIXED = 0, 1
CH_BC_PERIODIC, CH_BC_NEUMANN = 0, 1
CH_PHI_SHRINK, CH_PHI_RESTART = 0, 1
CH_MMAX = 100
CH_PMAX = 4096
CH_NOALLOC_MAX_POINTS = 1 << 20

EXPORTED = (
    "ch_create", "ch_destroy", "ch_strerror", "ch_last_error_message",
    "ch_run_ee", "ch_step_ee", "ch_run_ee_batch", "ch_run_lim", "ch_run_lim_batch", "ch_step_lim", "ch_step_lim_noalloc", "ch_phiv",
    "ch_time_kernel", "ch_get_shape", "ch_set_shape", "ch_tune_shape", "ch_tune_batch_shapes",

    "ch_server_create", "ch_server_destroy", "ch_submit", "ch_poll",
)
CH_REQ_QUEUED, CH_REQ_RUNNING, CH_REQ_DONE, CH_REQ_FAILED = 0, 1, 2, 3
CH_METHOD_EE, CH_METHOD_LIM = 0, 1
CH_KERNEL_MGS, CH_KERNEL_MATVEC, CH_KERNEL_PHI = 0, 1, 2
CH_KERNEL_DC_MATVEC, CH_KERNEL_DC_UPDATE, CH_KERNEL_LIM_STAGE, CH_KERNEL_DC_ITER, CH_KERNEL_LIM_STAGE2 = 3, 4, 5, 6, 7
CH_ORTH_DCGS2, CH_ORTH_MGS = 0, 1


class ChProblem(ctypes.Structure):
    _fields_ = [("dim", c_int), ("n", c_int), ("eps", c_double), ("eyre", c_int), ("prec", c_int), ("bc", c_int),
                ("length", c_double), ("mobility", c_int), ("mob0", c_double), ("mob1", c_double)]


class ChShape(ctypes.Structure):
    _fields_ = [("vx", c_int), ("wblk", c_int), ("cblk", c_int)]


class ChEeOpts(ctypes.Structure):
    _fields_ = [("m_max", c_int), ("tol", c_double), ("tol_phi_fixed", c_double), ("tau_min", c_double),
                ("constant_step", c_int), ("orth", c_int), ("graph_chunk", c_int)]


class ChStepRecord(ctypes.Structure):
    _fields_ = [("t", c_double), ("tau", c_double), ("tau_next", c_double), ("est", c_double),
                ("tol_phi", c_double), ("beta", c_double), ("resnorm", c_double), ("lambda_max", c_double),
                ("j", c_int), ("cycles", c_int), ("traced", c_int), ("matvecs", c_int)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ChRunStats(ctypes.Structure):
    _fields_ = [("t", c_double), ("tau_next", c_double), ("steps", c_int), ("matvecs", c_longlong),
                ("restarts", c_int), ("traces", c_int), ("status", c_int)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ChBatchItem(ctypes.Structure):
    _fields_ = [("n", c_int), ("eps", c_double), ("y", c_void_p), ("tau0", c_double), ("T", c_double),
                ("max_steps", c_int)]


class ChRequest(ctypes.Structure):
    _fields_ = [("n", c_int), ("eps", c_double), ("y0", c_void_p), ("steps", c_int), ("tau0", c_double),
                ("method", c_int), ("T", c_double), ("tol", c_double), ("y0_on_host", c_int)]


class ChError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(message)
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libch.so and declare its signatures (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2502_14589_amd.build`")
    lib = ctypes.CDLL(path)
    P = POINTER
    lib.ch_create.argtypes = [P(c_void_p), c_int, c_void_p]
    lib.ch_destroy.argtypes = [c_void_p]
    lib.ch_strerror.argtypes = [c_int]
    lib.ch_strerror.restype = ctypes.c_char_p
    lib.ch_last_error_message.argtypes = [c_void_p]
    lib.ch_last_error_message.restype = ctypes.c_char_p
    lib.ch_run_ee.argtypes = [c_void_p, P(ChProblem), c_void_p, c_double, c_double, c_double, c_int, P(ChEeOpts),
                              P(ChRunStats), P(ChStepRecord)]
    lib.ch_step_ee.argtypes = [c_void_p, P(ChProblem), c_void_p, c_double, c_double, c_double, P(ChEeOpts),
                               P(ChStepRecord)]
    lib.ch_run_lim.argtypes = [c_void_p, P(ChProblem), c_void_p, c_double, c_double, c_double, c_int, c_double,
                               P(ChRunStats), P(ChStepRecord)]
    lib.ch_step_lim.argtypes = [c_void_p, P(ChProblem), c_void_p, c_double, c_double, c_double, c_double,
                                P(ChStepRecord)]
    lib.ch_step_lim_noalloc.argtypes = [c_void_p, P(ChProblem), c_void_p, c_double, c_double, c_double, c_double,
                                        P(ChStepRecord)]
    lib.ch_phiv.argtypes = [c_void_p, P(ChProblem), c_void_p, c_void_p, c_double, c_int, c_double, c_int,
                            P(ChStepRecord)]
    lib.ch_run_ee_batch.argtypes = [c_void_p, c_int, P(ChBatchItem), c_int, c_int, c_int, P(ChEeOpts),
                                    P(ChRunStats)]
    lib.ch_run_lim_batch.argtypes = [c_void_p, c_int, P(ChBatchItem), c_int, c_int, c_double, P(ChRunStats)]
    lib.ch_server_create.argtypes = [c_int, c_int, P(ChEeOpts), ctypes.c_size_t, c_int, P(c_void_p)]
    lib.ch_server_destroy.argtypes = [c_void_p]
    lib.ch_submit.argtypes = [c_void_p, P(ChRequest), P(ctypes.c_ulonglong)]
    lib.ch_poll.argtypes = [c_void_p, ctypes.c_ulonglong, P(c_int), c_void_p, P(ChRunStats), P(c_double)]
    lib.ch_time_kernel.argtypes = [c_void_p, P(ChProblem), c_int, c_int, P(c_int), c_int, P(c_double), P(c_double)]
    lib.ch_get_shape.argtypes = [c_void_p, c_int, c_int, c_int, P(ChShape)]
    lib.ch_set_shape.argtypes = [c_void_p, c_int, c_int, c_int, P(ChShape)]
    lib.ch_tune_shape.argtypes = [c_void_p, P(ChProblem), c_int, P(ChShape), P(c_double), P(c_double)]
    lib.ch_tune_batch_shapes.argtypes = [c_void_p, c_int, P(ChBatchItem), c_int, c_int, c_int, c_int, P(c_double),
                                         P(c_double)]
    for name in ("ch_create", "ch_destroy", "ch_run_ee", "ch_step_ee", "ch_run_ee_batch", "ch_run_lim", "ch_run_lim_batch",
                 "ch_step_lim", "ch_step_lim_noalloc", "ch_phiv", "ch_time_kernel", "ch_server_create", "ch_server_destroy", "ch_submit",
                 "ch_poll", "ch_get_shape", "ch_set_shape", "ch_tune_shape", "ch_tune_batch_shapes"):
        getattr(lib, name).restype = c_int
    _lib = lib
    return lib


@dataclass
class Problem:
    """Cahn-Hilliard grid: n**dim points on [0,L]^dim, h = L/n; periodic, or
    (bc = CH_BC_NEUMANN, 2-D) the cell-centred grid with Neumann boundaries.

    mobility=(m0, m1) selects the variable mobility M(c) = max(m0 + m1 (1 - c^2), 0)
    of Section 2, Remark 1 (2-D periodic grids); None is the constant M = 1."""

    dim: int
    n: int
    eps: float
    eyre: bool = False
    precision: int = CH_FP64
    bc: int = CH_BC_PERIODIC
    length: float = 1.0
    mobility: tuple | None = None

    def c(self) -> ChProblem:
        m0, m1 = self.mobility if self.mobility is not None else (0.0, 0.0)
        return ChProblem(self.dim, self.n, float(self.eps), int(bool(self.eyre)), int(self.precision), int(self.bc),
                         float(self.length), int(self.mobility is not None), float(m0), float(m1))

    @property
    def N(self) -> int:
        return self.n ** self.dim


def _check_field(y, N):
    import torch

    if not isinstance(y, torch.Tensor) or not y.is_cuda or y.dtype != torch.float64 or not y.is_contiguous():
        raise ValueError("fields must be contiguous float64 CUDA tensors")
    if y.numel() != N:
        raise ValueError(f"field has {y.numel()} values, the grid {N}")


class Context:
    """A libch context bound to one device and torch's current stream on it."""

    def __init__(self, device: int = 0):
        import torch

        self.lib = load_library()
        self.device = device
        with torch.cuda.device(device):
            stream = torch.cuda.current_stream(device).cuda_stream
        self._ptr = c_void_p()
        rc = self.lib.ch_create(byref(self._ptr), device, c_void_p(stream))
        if rc != CH_OK:
            raise ChError(rc, f"ch_create: {self.lib.ch_strerror(rc).decode()}")

    def close(self):
        if self._ptr:
            self.lib.ch_destroy(self._ptr)
            self._ptr = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _raise(self, rc, what, allow=()):
        if rc != CH_OK and rc not in allow:
            msg = self.lib.ch_strerror(rc).decode()
            detail = self.lib.ch_last_error_message(self._ptr).decode()
            raise ChError(rc, f"{what}: {msg}" + (f" ({detail})" if detail else ""))

    # -- EE2 ---------------------------------------------------------------
    def run_ee(self, prob: Problem, y, tau0: float, *, t0: float = 0.0, T: float = math.inf, max_steps: int = 0,
               m_max: int = 30, tol: float = 1e-4, tol_phi_fixed: float = 0.0, tau_min: float = 0.0,
               constant_step: bool = False, records: bool = False, raise_on_error: bool = True,
               orth: int = CH_ORTH_DCGS2, graph_chunk: int = 0):
        """Adaptive (Fig. 4) or constant-step EE2 run on y in place; returns (stats, records).
        graph_chunk > 0 replays the DCGS2 iterations as captured HIP graphs of that many iterations."""
        _check_field(y, prob.N)
        opts = ChEeOpts(int(m_max), float(tol), float(tol_phi_fixed), float(tau_min), int(bool(constant_step)),
                        int(orth), int(graph_chunk))
        st = ChRunStats()
        recs = (ChStepRecord * max_steps)() if (records and max_steps > 0) else None
        pb = prob.c()
        rc = self.lib.ch_run_ee(self._ptr, byref(pb), c_void_p(y.data_ptr()), float(tau0), float(t0), float(T),
                                int(max_steps), byref(opts), byref(st), recs)
        if raise_on_error:
            self._raise(rc, "ch_run_ee")
        out = st.as_dict()
        out["rc"] = rc
        return out, ([r.as_dict() for r in recs[: st.steps]] if recs is not None else None)

    def step_ee(self, prob: Problem, y, tau: float, *, t: float = 0.0, T: float = math.inf, m_max: int = 30,
                tol: float = 1e-4, tol_phi_fixed: float = 0.0, tau_min: float = 0.0, constant_step: bool = False,
                orth: int = CH_ORTH_DCGS2):
        _check_field(y, prob.N)
        opts = ChEeOpts(int(m_max), float(tol), float(tol_phi_fixed), float(tau_min), int(bool(constant_step)),
                        int(orth))
        rec = ChStepRecord()
        pb = prob.c()
        rc = self.lib.ch_step_ee(self._ptr, byref(pb), c_void_p(y.data_ptr()), float(tau), float(t), float(T),
                                 byref(opts), byref(rec))
        self._raise(rc, "ch_step_ee")
        return rec.as_dict()

    def run_ee_batch(self, fields, ns, eps, *, dim: int = 2, eyre: bool = False, precision: int = CH_FP64,
                     tau0=1e-3, T=math.inf, max_steps=50, m_max: int = 30, tol: float = 1e-4,
                     tol_phi_fixed: float = 0.0, tau_min: float = 0.0, raise_on_error: bool = True,
                     orth: int = CH_ORTH_DCGS2, graph_chunk: int = 0):
        """Adaptive EE2 on many instances at once (each field updated in place); returns per-instance stats."""
        count = len(fields)
        as_list = lambda v: list(v) if isinstance(v, (list, tuple)) else [v] * count
        tau0s, Ts, steps = as_list(tau0), as_list(T), as_list(max_steps)
        items = (ChBatchItem * count)()
        for i, y in enumerate(fields):
            _check_field(y, ns[i] ** dim)
            items[i] = ChBatchItem(int(ns[i]), float(eps[i]), c_void_p(y.data_ptr()), float(tau0s[i]),
                                   float(Ts[i]), int(steps[i]))
        opts = ChEeOpts(int(m_max), float(tol), float(tol_phi_fixed), float(tau_min), 0, int(orth), int(graph_chunk))
        st = (ChRunStats * count)()
        rc = self.lib.ch_run_ee_batch(self._ptr, count, items, int(dim), int(bool(eyre)), int(precision),
                                      byref(opts), st)
        if raise_on_error:
            self._raise(rc, "ch_run_ee_batch")
        return [s.as_dict() for s in st], rc

    # -- LIM ---------------------------------------------------------------
    def run_lim(self, prob: Problem, y, tau0: float, *, t0: float = 0.0, T: float = math.inf, max_steps: int = 0,
                tol: float = 0.0, records: bool = False, raise_on_error: bool = True):
        """Adaptive (Fig. 2, tol > 0) or constant-step LIM run on y in place."""
        _check_field(y, prob.N)
        st = ChRunStats()
        recs = (ChStepRecord * max_steps)() if (records and max_steps > 0) else None
        pb = prob.c()
        rc = self.lib.ch_run_lim(self._ptr, byref(pb), c_void_p(y.data_ptr()), float(tau0), float(t0), float(T),
                                 int(max_steps), float(tol), byref(st), recs)
        if raise_on_error:
            self._raise(rc, "ch_run_lim")
        out = st.as_dict()
        out["rc"] = rc
        return out, ([r.as_dict() for r in recs[: st.steps]] if recs is not None else None)

    def run_lim_batch(self, fields, ns, eps, *, dim: int = 2, eyre: bool = False, tau0=1e-6, T=math.inf,
                      max_steps=10, tol: float = 1e-4, raise_on_error: bool = True):
        """Adaptive (tol > 0) or constant-step LIM on many instances at once (fields updated in place)."""
        count = len(fields)
        as_list = lambda v: list(v) if isinstance(v, (list, tuple)) else [v] * count
        tau0s, Ts, steps = as_list(tau0), as_list(T), as_list(max_steps)
        items = (ChBatchItem * count)()
        for i, y in enumerate(fields):
            _check_field(y, ns[i] ** dim)
            items[i] = ChBatchItem(int(ns[i]), float(eps[i]), c_void_p(y.data_ptr()), float(tau0s[i]),
                                   float(Ts[i]), int(steps[i]))
        st = (ChRunStats * count)()
        rc = self.lib.ch_run_lim_batch(self._ptr, count, items, int(dim), int(bool(eyre)), float(tol), st)
        if raise_on_error:
            self._raise(rc, "ch_run_lim_batch")
        return [s.as_dict() for s in st], rc

    def step_lim(self, prob: Problem, y, tau: float, *, t: float = 0.0, T: float = math.inf, tol: float = 0.0):
        _check_field(y, prob.N)
        rec = ChStepRecord()
        pb = prob.c()
        rc = self.lib.ch_step_lim(self._ptr, byref(pb), c_void_p(y.data_ptr()), float(tau), float(t), float(T),
                                  float(tol), byref(rec))
        self._raise(rc, "ch_step_lim")
        return rec.as_dict()

    def step_lim_noalloc(self, prob: Problem, y, tau: float, *, t: float = 0.0, T: float = math.inf,
                         tol: float = 0.0, raise_on_error: bool = True):
        """ch_step_lim without device allocation (scratch in a static device array)."""
        _check_field(y, prob.N)
        rec = ChStepRecord()
        pb = prob.c()
        rc = self.lib.ch_step_lim_noalloc(self._ptr, byref(pb), c_void_p(y.data_ptr()), float(tau), float(t),
                                          float(T), float(tol), byref(rec))
        if raise_on_error:
            self._raise(rc, "ch_step_lim_noalloc")
        return rec.as_dict(), rc

    # -- phi action --------------------------------------------------------
    def phiv(self, prob: Problem, y, y_out, tau0: float, *, mode: int = CH_PHI_SHRINK, tol_phi: float = 1e-8,
             m_max: int = 30):
        """y_out = y + tau phi(-tau Ahat)(ghat - Ahat y) (eq. yt); returns the step record."""
        _check_field(y, prob.N)
        _check_field(y_out, prob.N)
        rec = ChStepRecord()
        pb = prob.c()
        rc = self.lib.ch_phiv(self._ptr, byref(pb), c_void_p(y.data_ptr()), c_void_p(y_out.data_ptr()),
                              float(tau0), int(mode), float(tol_phi), int(m_max), byref(rec))
        self._raise(rc, "ch_phiv")
        return rec.as_dict()

    # -- measurement aid -----------------------------------------------------
    def time_kernel(self, prob: Problem, kernel: int, m_max: int, iters=None, count: int = 0):
        """(elapsed microseconds, algorithmic bytes) of back-to-back launches of one kernel:
        one per entry of `iters` (Arnoldi iterations), or `count` LIM stages."""
        us, by = c_double(), c_double()
        pb = prob.c()
        if iters is None:
            arr, n = None, int(count)
        else:
            n = len(iters)
            arr = (c_int * n)(*[int(k) for k in iters])
        rc = self.lib.ch_time_kernel(self._ptr, byref(pb), int(kernel), int(m_max), arr, n, byref(us), byref(by))
        self._raise(rc, "ch_time_kernel")
        return us.value, by.value

    # -- launch shapes -------------------------------------------------------
    def get_shape(self, dim: int, n: int, precision: int = CH_FP64) -> dict:
        """The launch shape runs use for this grid: {'vx', 'wblk', 'cblk'}."""
        out = ChShape()
        self._raise(self.lib.ch_get_shape(self._ptr, int(dim), int(n), int(precision), byref(out)), "ch_get_shape")
        return {"vx": out.vx, "wblk": out.wblk, "cblk": out.cblk}

    def set_shape(self, dim: int, n: int, precision: int = CH_FP64, shape: dict | None = None):
        """Sets (or with None clears) the launch shape of this grid for later runs."""
        ptr = byref(ChShape(int(shape["vx"]), int(shape["wblk"]), int(shape["cblk"]))) if shape is not None else None
        self._raise(self.lib.ch_set_shape(self._ptr, int(dim), int(n), int(precision), ptr), "ch_set_shape")

    def tune_shape(self, prob: Problem, m_max: int = 30):
        """Times candidate launch shapes and keeps the fastest: (shape, best_us, default_us)."""
        out, b, d = ChShape(), c_double(), c_double()
        pb = prob.c()
        self._raise(self.lib.ch_tune_shape(self._ptr, byref(pb), int(m_max), byref(out), byref(b), byref(d)),
                    "ch_tune_shape")
        return {"vx": out.vx, "wblk": out.wblk, "cblk": out.cblk}, b.value, d.value

    def tune_batch_shapes(self, ns, eps, *, dim: int = 2, eyre: bool = False, precision: int = CH_FP64,
                          m_max: int = 30):
        """Tunes the launch shapes of a batch's grids together: (shapes by n, best_us, default_us)."""
        count = len(ns)
        items = (ChBatchItem * count)()
        for i in range(count):
            items[i] = ChBatchItem(int(ns[i]), float(eps[i]), None, 1.0, 1.0, 1)
        b, d = c_double(), c_double()
        self._raise(self.lib.ch_tune_batch_shapes(self._ptr, count, items, int(dim), int(bool(eyre)), int(precision),
                                                  int(m_max), byref(b), byref(d)), "ch_tune_batch_shapes")
        return {n: self.get_shape(dim, n, precision) for n in sorted(set(int(x) for x in ns))}, b.value, d.value


class Server:
    """Continuous-batching EE2 server (ch_server_create / ch_submit / ch_poll)."""

    def __init__(self, device: int = 0, precision: int = CH_FP64, m_max: int = 30, tol: float = 1e-4,
                 tol_phi_fixed: float = 0.0, hbm_budget: int = 8 << 30, max_slots: int = 64,
                 orth: int = CH_ORTH_DCGS2):
        self.lib = load_library()
        opts = ChEeOpts(int(m_max), float(tol), float(tol_phi_fixed), 0.0, 0, int(orth))
        self._ptr = c_void_p()
        rc = self.lib.ch_server_create(device, int(precision), byref(opts), int(hbm_budget), int(max_slots),
                                       byref(self._ptr))
        if rc != CH_OK:
            raise ChError(rc, f"ch_server_create: {self.lib.ch_strerror(rc).decode()}")

    def submit(self, y0, n: int, eps: float, steps: int = 0, tau0: float = 1e-3, *, method: int = CH_METHOD_EE,
               T: float = math.inf, tol: float = 0.0) -> int:
        """Queue a 2-D request (y0 is copied: a CUDA tensor, or a host numpy
        array); returns its ticket.  steps <= 0 runs until T."""
        import numpy as np
        import torch

        if isinstance(y0, np.ndarray):
            if y0.dtype != np.float64 or not y0.flags["C_CONTIGUOUS"] or y0.size != n * n:
                raise ValueError("host fields must be contiguous float64 arrays of n*n values")
            ptr, host = c_void_p(y0.ctypes.data), 1
        else:
            _check_field(y0, n * n)
            torch.cuda.current_stream(y0.device).synchronize()   # the library copies y0 on its own stream
            ptr, host = c_void_p(y0.data_ptr()), 0
        req = ChRequest(int(n), float(eps), ptr, int(steps), float(tau0), int(method), float(T), float(tol), host)
        t = ctypes.c_ulonglong()
        rc = self.lib.ch_submit(self._ptr, byref(req), byref(t))
        if rc != CH_OK:
            raise ChError(rc, f"ch_submit: {self.lib.ch_strerror(rc).decode()}")
        return t.value

    def poll(self, ticket: int, y_out=None):
        """(state, status, stats, (queue, service, total) latency in s); copies the result when done."""
        state = c_int()
        st = ChRunStats()
        lat = (c_double * 3)()
        ptr = c_void_p(y_out.data_ptr()) if y_out is not None else None
        rc = self.lib.ch_poll(self._ptr, ctypes.c_ulonglong(ticket), byref(state), ptr, byref(st), lat)
        return state.value, rc, st.as_dict(), tuple(lat)

    def close(self):
        if self._ptr:
            self.lib.ch_server_destroy(self._ptr)
            self._ptr = c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
