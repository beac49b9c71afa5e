"""ctypes binding of libprop.so (the C ABI in include/prop.h).

Argument marshalling only: every step of propagation runs in the HIP
kernels behind the C ABI.  PyTorch is used, when the caller wants it, only
to hand over device memory and a stream.  There is no fallback: if the
library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libprop.so")

CONVERGED, INFEASIBLE, MAX_ROUNDS = 0, 1, 2
STATUS_NAMES = {CONVERGED: "CONVERGED", INFEASIBLE: "INFEASIBLE", MAX_ROUNDS: "MAX_ROUNDS"}
OK, EINVAL, ENOMEM, EDEVICE, EBUSY = 0, -1, -2, -3, -4
LOOP_PERSISTENT, LOOP_STREAM, LOOP_HOST, LOOP_GRAPH, LOOP_GRAPH_ALL = 0, 1, 2, 3, 4
LOOP_NAMES = {"persistent": LOOP_PERSISTENT, "stream": LOOP_STREAM, "host": LOOP_HOST,
              "graph": LOOP_GRAPH, "graph_all": LOOP_GRAPH_ALL}
STORE_F64, STORE_F32 = 64, 32

# every function the header declares
EXPORTED = ("prop_create", "prop_autotune", "prop_run", "prop_run_device", "prop_run_batch",
            "prop_run_batch_device", "prop_run_batch_device_static",
            "prop_set_loop", "prop_set_marking", "prop_set_parent", "prop_set_store",
            "prop_get_info",
            "prop_last_timing", "prop_set_kernel_timing", "prop_last_kernel_timing",
            "prop_destroy", "prop_last_error",
            "prop_srv_create", "prop_srv_add_instance", "prop_srv_submit", "prop_srv_poll",
            "prop_srv_wait", "prop_srv_get_stats", "prop_srv_reset_stats", "prop_srv_destroy")


class PropError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"prop error {code}: {msg}")
        self.code = code


class _Csr(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("vals", ctypes.c_void_p)]


class _Params(ctypes.Structure):
    _fields_ = [("eps_int", ctypes.c_double), ("cont_rel_tol", ctypes.c_double),
                ("feas_tol", ctypes.c_double), ("steps", ctypes.c_int32),
                ("layout", ctypes.c_int32)]


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("rounds", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("nnz_stored", ctypes.c_int64), ("n_chunks", ctypes.c_int32),
                ("n_long_rows", ctypes.c_int32), ("n_segments", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("device_bytes", ctypes.c_int64),
                ("alg_bytes_round", ctypes.c_int64), ("steps", ctypes.c_int32),
                ("layout", ctypes.c_int32)]


class _SrvConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int32),
                ("rounds_per_step", ctypes.c_int32), ("max_pending", ctypes.c_int32),
                ("marking", ctypes.c_int32)]


class _SrvStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("running", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("peak_device_bytes", ctypes.c_int64),
                ("steps", ctypes.c_int64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("wall_s", ctypes.c_double),
                ("req_per_s", ctypes.c_double)]


def _load():
    # PyTorch ships its own HIP runtime (same soname as the system one).  Load
    # it first so that libprop binds to that copy: two HIP runtimes in one
    # process cannot both open the GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32 = ctypes.c_void_p, ctypes.c_int32
    lib.prop_create.argtypes = [ctypes.POINTER(_Csr), P, P, P, ctypes.POINTER(_Params),
                                ctypes.POINTER(P)]
    lib.prop_create.restype = ctypes.c_int
    lib.prop_autotune.argtypes = [ctypes.POINTER(_Csr), P, P, P, ctypes.POINTER(_Params), P, P, i32,
                                  ctypes.POINTER(i32)]
    lib.prop_autotune.restype = ctypes.c_int
    lib.prop_run.argtypes = [P, P, P, i32, ctypes.POINTER(_Result)]
    lib.prop_run.restype = ctypes.c_int
    lib.prop_run_device.argtypes = [P, P, P, i32, P, ctypes.POINTER(_Result)]
    lib.prop_run_device.restype = ctypes.c_int
    lib.prop_run_batch.argtypes = [P, i32, P, P, i32, ctypes.POINTER(_Result)]
    lib.prop_run_batch.restype = ctypes.c_int
    lib.prop_run_batch_device.argtypes = [P, i32, P, P, i32, P, ctypes.POINTER(_Result)]
    lib.prop_run_batch_device.restype = ctypes.c_int
    lib.prop_run_batch_device_static.argtypes = [P, i32, P, P, i32, P, ctypes.POINTER(_Result)]
    lib.prop_run_batch_device_static.restype = ctypes.c_int
    lib.prop_set_loop.argtypes = [P, i32]
    lib.prop_set_loop.restype = ctypes.c_int
    lib.prop_set_marking.argtypes = [P, i32]
    lib.prop_set_marking.restype = ctypes.c_int
    lib.prop_set_parent.argtypes = [P, P, P, P]
    lib.prop_set_store.argtypes = [P, i32]
    lib.prop_set_store.restype = ctypes.c_int
    lib.prop_set_parent.restype = ctypes.c_int
    lib.prop_get_info.argtypes = [P, ctypes.POINTER(_Info)]
    lib.prop_get_info.restype = ctypes.c_int
    lib.prop_last_timing.argtypes = [P, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
    lib.prop_last_timing.restype = ctypes.c_int
    lib.prop_set_kernel_timing.argtypes = [P, i32]
    lib.prop_set_kernel_timing.restype = ctypes.c_int
    lib.prop_last_kernel_timing.argtypes = [P, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_int32)]
    lib.prop_last_kernel_timing.restype = ctypes.c_int
    lib.prop_destroy.argtypes = [P]
    lib.prop_destroy.restype = None
    lib.prop_last_error.argtypes = []
    lib.prop_last_error.restype = ctypes.c_char_p
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.prop_srv_create.argtypes = [ctypes.POINTER(_SrvConfig), ctypes.POINTER(P)]
    lib.prop_srv_create.restype = ctypes.c_int
    lib.prop_srv_add_instance.argtypes = [P, P, ctypes.POINTER(i32)]
    lib.prop_srv_add_instance.restype = ctypes.c_int
    lib.prop_srv_submit.argtypes = [P, i32, P, P, i32, i64p]
    lib.prop_srv_submit.restype = ctypes.c_int
    lib.prop_srv_poll.argtypes = [P, ctypes.c_int64, ctypes.POINTER(_Result), P, P]
    lib.prop_srv_poll.restype = ctypes.c_int
    lib.prop_srv_wait.argtypes = [P, ctypes.c_int64, i32, ctypes.POINTER(_Result), P, P]
    lib.prop_srv_wait.restype = ctypes.c_int
    lib.prop_srv_get_stats.argtypes = [P, ctypes.POINTER(_SrvStats)]
    lib.prop_srv_get_stats.restype = ctypes.c_int
    lib.prop_srv_reset_stats.argtypes = [P]
    lib.prop_srv_reset_stats.restype = ctypes.c_int
    lib.prop_srv_destroy.argtypes = [P]
    lib.prop_srv_destroy.restype = None
    return lib


lib = _load()


def last_error() -> str:
    return lib.prop_last_error().decode()


def _check(rc: int):
    if rc != OK:
        raise PropError(rc, last_error())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class RunResult:
    status: int
    rounds: int

    @property
    def status_name(self) -> str:
        return STATUS_NAMES[self.status]


class Problem:
    """A constraint system resident on the current HIP device."""

    def __init__(self, m, n, row_ptr, col_idx, vals, lhs, rhs, vartype, eps_int=1e-6,
                 cont_rel_tol=1e-6, feas_tol=1e-6, steps=0, layout=0):
        """steps: layout entries per lane (4, 8, 16); 0 = the autotuned value
        for this matrix shape, else by size.  layout: 0 length-class chunks,
        1 nnz split (single runs only)."""
        self._h = None
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        va = np.ascontiguousarray(vals, dtype=np.float64)
        lh = np.ascontiguousarray(lhs, dtype=np.float64)
        rh = np.ascontiguousarray(rhs, dtype=np.float64)
        vt = np.ascontiguousarray(vartype, dtype=np.uint8)
        if rp.shape != (m + 1,) or lh.shape != (m,) or rh.shape != (m,) or vt.shape != (n,):
            raise ValueError("array shapes do not match m / n")
        if ci.shape != va.shape or ci.shape[0] != int(rp[-1]):
            raise ValueError("col_idx / vals do not match row_ptr")
        csr = _Csr(int(m), int(n), int(rp[-1]), _ptr(rp).value, _ptr(ci).value, _ptr(va).value)
        prm = _Params(float(eps_int), float(cont_rel_tol), float(feas_tol), int(steps), int(layout))
        h = ctypes.c_void_p()
        _check(lib.prop_create(ctypes.byref(csr), _ptr(lh), _ptr(rh), _ptr(vt), ctypes.byref(prm),
                               ctypes.byref(h)))
        self._h = h
        self.m, self.n = int(m), int(n)

    @classmethod
    def from_instance(cls, inst, **params):
        return cls(inst.m, inst.n, inst.row_ptr, inst.col_idx, inst.vals, inst.lhs, inst.rhs,
                   inst.vartype, **params)

    def close(self):
        if self._h is not None and self._h.value:
            lib.prop_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- runs ---------------------------------------------------------------
    def run(self, lb, ub, max_rounds: int = 100):
        """Host arrays in, (RunResult, lb, ub) out; the inputs are not modified."""
        lb = np.array(lb, dtype=np.float64, copy=True)
        ub = np.array(ub, dtype=np.float64, copy=True)
        if lb.shape != (self.n,) or ub.shape != (self.n,):
            raise ValueError("bounds must have shape (n,)")
        res = _Result()
        _check(lib.prop_run(self._h, _ptr(lb), _ptr(ub), int(max_rounds), ctypes.byref(res)))
        return RunResult(res.status, res.rounds), lb, ub

    def run_device(self, d_lb, d_ub, max_rounds: int = 100, stream=None) -> RunResult:
        """Device tensors (float64, contiguous, length n) updated in place.
        `stream` is a torch.cuda.Stream or a raw hipStream_t integer; default:
        torch's current stream."""
        for t in (d_lb, d_ub):
            if not (t.is_cuda and t.dtype.is_floating_point and t.element_size() == 8
                    and t.is_contiguous() and t.numel() == self.n):
                raise ValueError("bounds must be contiguous float64 device tensors of length n")
        if stream is None:
            import torch

            stream = torch.cuda.current_stream(d_lb.device)
        raw = getattr(stream, "cuda_stream", stream)
        res = _Result()
        _check(lib.prop_run_device(self._h, ctypes.c_void_p(d_lb.data_ptr()),
                                   ctypes.c_void_p(d_ub.data_ptr()), int(max_rounds),
                                   ctypes.c_void_p(int(raw) if raw else 0), ctypes.byref(res)))
        return RunResult(res.status, res.rounds)

    def run_batch(self, lbs, ubs, max_rounds: int = 100):
        """Batched nodes on host arrays of shape (nodes, n): (list of
        RunResult, lbs, ubs) out; the inputs are not modified."""
        lbs = np.array(lbs, dtype=np.float64, copy=True, order="C")
        ubs = np.array(ubs, dtype=np.float64, copy=True, order="C")
        if lbs.ndim != 2 or lbs.shape[1] != self.n or ubs.shape != lbs.shape:
            raise ValueError("bounds must have shape (nodes, n), the same for lb and ub")
        nodes = int(lbs.shape[0])
        if nodes < 1:
            raise ValueError("at least one node")
        res = (_Result * nodes)()
        _check(lib.prop_run_batch(self._h, nodes, _ptr(lbs), _ptr(ubs), int(max_rounds), res))
        return [RunResult(r.status, r.rounds) for r in res], lbs, ubs

    def run_batch_device(self, d_lb, d_ub, max_rounds: int = 100, stream=None,
                         static: bool = False):
        """Batched nodes: device tensors of shape (nodes, n), float64, updated
        in place.  Returns one RunResult per node.  With `static`, the
        library's fixed workspace array is used and nothing is allocated
        (prop_run_batch_device_static)."""
        for t in (d_lb, d_ub):
            if not (t.is_cuda and t.dtype.is_floating_point and t.element_size() == 8
                    and t.is_contiguous() and t.dim() == 2 and t.shape[1] == self.n):
                raise ValueError("bounds must be contiguous float64 device tensors (nodes, n)")
        nodes = int(d_lb.shape[0])
        if d_ub.shape[0] != nodes:
            raise ValueError("lb and ub hold different node counts")
        if stream is None:
            import torch

            stream = torch.cuda.current_stream(d_lb.device)
        raw = getattr(stream, "cuda_stream", stream)
        res = (_Result * nodes)()
        fn = lib.prop_run_batch_device_static if static else lib.prop_run_batch_device
        _check(fn(self._h, nodes, ctypes.c_void_p(d_lb.data_ptr()),
                  ctypes.c_void_p(d_ub.data_ptr()), int(max_rounds),
                  ctypes.c_void_p(int(raw) if raw else 0), res))
        return [RunResult(r.status, r.rounds) for r in res]

    def set_loop(self, mode):
        if isinstance(mode, str):
            mode = LOOP_NAMES[mode]
        _check(lib.prop_set_loop(self._h, int(mode)))

    def set_marking(self, enable: bool):
        """Marked rounds: skip rows none of whose variables changed in the
        previous round (results unchanged)."""
        _check(lib.prop_set_marking(self._h, 1 if enable else 0))

    def set_parent(self, d_lb=None, d_ub=None, stream=None):
        """Parent fixed point for marked runs (device tensors of n float64),
        or None to clear it: round 1 then processes only the rows of
        variables whose start bounds differ from the parent's."""
        if d_lb is None and d_ub is None:
            _check(lib.prop_set_parent(self._h, None, None, None))
            return
        for t in (d_lb, d_ub):
            if not (t.is_cuda and t.dtype.is_floating_point and t.element_size() == 8
                    and t.is_contiguous() and t.numel() == self.n):
                raise ValueError("parent bounds must be contiguous float64 device tensors (n,)")
        if stream is None:
            import torch

            stream = torch.cuda.current_stream(d_lb.device)
        raw = getattr(stream, "cuda_stream", stream)
        _check(lib.prop_set_parent(self._h, ctypes.c_void_p(d_lb.data_ptr()),
                                   ctypes.c_void_p(d_ub.data_ptr()),
                                   ctypes.c_void_p(int(raw) if raw else 0)))

    def set_store(self, bits: int):
        """Bound store of later single runs: 64 (doubles) or 32 (single
        precision, rounded outward; FP64 arithmetic)."""
        _check(lib.prop_set_store(self._h, int(bits)))

    def info(self) -> dict:
        inf = _Info()
        _check(lib.prop_get_info(self._h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in _Info._fields_}

    def set_kernel_timing(self, enable: bool):
        _check(lib.prop_set_kernel_timing(self._h, 1 if enable else 0))

    def last_kernel_timing(self):
        """(summed ms, launches) of the per-round matrix kernel in the last run."""
        ms, n = ctypes.c_double(), ctypes.c_int32()
        _check(lib.prop_last_kernel_timing(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def last_timing(self):
        """(loop_ms, total_ms) of the last run, from HIP events on its stream."""
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(lib.prop_last_timing(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value


def autotune(inst, lb, ub, max_rounds: int = 100) -> int:
    """Times the layouts (steps 16, 8, 4) on full propagations from (lb, ub)
    and records the fastest for this matrix shape; returns its steps."""
    rp = np.ascontiguousarray(inst.row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(inst.col_idx, dtype=np.int32)
    va = np.ascontiguousarray(inst.vals, dtype=np.float64)
    lh = np.ascontiguousarray(inst.lhs, dtype=np.float64)
    rh = np.ascontiguousarray(inst.rhs, dtype=np.float64)
    vt = np.ascontiguousarray(inst.vartype, dtype=np.uint8)
    lb = np.ascontiguousarray(lb, dtype=np.float64)
    ub = np.ascontiguousarray(ub, dtype=np.float64)
    csr = _Csr(int(inst.m), int(inst.n), int(rp[-1]), _ptr(rp).value, _ptr(ci).value,
               _ptr(va).value)
    out = ctypes.c_int32()
    _check(lib.prop_autotune(ctypes.byref(csr), _ptr(lh), _ptr(rh), _ptr(vt), None, _ptr(lb),
                             _ptr(ub), int(max_rounds), ctypes.byref(out)))
    return out.value


def create_raw(csr_args, lhs, rhs, vartype, params=None):
    """Calls prop_create with explicit arrays; returns (rc, handle).  For tests
    of the validation path, which runs before any device call."""
    m, n, rp, ci, va = csr_args
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    va = np.ascontiguousarray(va, dtype=np.float64)
    lh = np.ascontiguousarray(lhs, dtype=np.float64)
    rh = np.ascontiguousarray(rhs, dtype=np.float64)
    vt = np.ascontiguousarray(vartype, dtype=np.uint8)
    csr = _Csr(int(m), int(n), int(rp[-1]) if rp.size else 0, _ptr(rp).value, _ptr(ci).value,
               _ptr(va).value)
    prm = _Params(*((tuple(params) + (0, 0))[:5] if params else (1e-6, 1e-6, 1e-6, 0, 0)))
    h = ctypes.c_void_p()
    rc = lib.prop_create(ctypes.byref(csr), _ptr(lh), _ptr(rh), _ptr(vt), ctypes.byref(prm),
                         ctypes.byref(h))
    return rc, h


class Server:
    """Continuous-batching server over problems resident on the device
    (prop_srv_* in the C ABI).  Problems added must outlive the server."""

    def __init__(self, budget_bytes: int, max_slots: int = 0, rounds_per_step: int = 0,
                 max_pending: int = 0, marking: bool = False):
        self._h = None
        cfg = _SrvConfig(int(budget_bytes), int(max_slots), int(rounds_per_step),
                         int(max_pending), 1 if marking else 0)
        h = ctypes.c_void_p()
        _check(lib.prop_srv_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._n = []          # n of each added problem
        self._problems = []   # keeps the problems alive while the server is

    def close(self):
        if self._h is not None and self._h.value:
            lib.prop_srv_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def add_instance(self, problem: Problem) -> int:
        i = ctypes.c_int32()
        _check(lib.prop_srv_add_instance(self._h, problem._h, ctypes.byref(i)))
        self._n.append(problem.n)
        self._problems.append(problem)
        return i.value

    def submit(self, inst: int, lb, ub, max_rounds: int = 100) -> int:
        lb = np.ascontiguousarray(lb, dtype=np.float64)
        ub = np.ascontiguousarray(ub, dtype=np.float64)
        n = self._n[inst] if 0 <= inst < len(self._n) else -1
        if lb.shape != (n,) or ub.shape != (n,):
            if n >= 0:
                raise ValueError("bounds must have shape (n,) of the instance")
        t = ctypes.c_int64()
        _check(lib.prop_srv_submit(self._h, int(inst), _ptr(lb), _ptr(ub), int(max_rounds),
                                   ctypes.byref(t)))
        return t.value

    def _take(self, fn, ticket, *extra, n, bounds=True):
        lb = np.empty(n) if bounds else None
        ub = np.empty(n) if bounds else None
        res = _Result()
        rc = fn(self._h, ctypes.c_int64(ticket), *extra, ctypes.byref(res),
                _ptr(lb) if bounds else None, _ptr(ub) if bounds else None)
        if rc < 0:
            raise PropError(rc, last_error())
        if rc == 0:
            return None
        return RunResult(res.status, res.rounds), lb, ub

    def poll(self, ticket: int, n: int, bounds: bool = True):
        """(RunResult, lb, ub) once finished (releasing the ticket), else None.
        n is the instance's variable count; with bounds=False the bounds are
        not copied (lb, ub are None)."""
        return self._take(lib.prop_srv_poll, ticket, n=n, bounds=bounds)

    def wait(self, ticket: int, n: int, timeout_ms: int = -1, bounds: bool = True):
        return self._take(lib.prop_srv_wait, ticket, ctypes.c_int32(int(timeout_ms)), n=n,
                          bounds=bounds)

    def stats(self) -> dict:
        st = _SrvStats()
        _check(lib.prop_srv_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in _SrvStats._fields_}

    def reset_stats(self):
        _check(lib.prop_srv_reset_stats(self._h))


def srv_create_raw(budget_bytes, max_slots=0, rounds_per_step=0, max_pending=0):
    """Calls prop_srv_create; returns (rc, handle).  For tests of argument
    checks, which need no device."""
    cfg = _SrvConfig(int(budget_bytes), int(max_slots), int(rounds_per_step), int(max_pending))
    h = ctypes.c_void_p()
    rc = lib.prop_srv_create(ctypes.byref(cfg), ctypes.byref(h))
    return rc, h
