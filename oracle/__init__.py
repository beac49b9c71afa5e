"""Sequential CPU oracle for activity-based domain propagation.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  The GPU library never
imports, links or executes anything here, and nothing here imports the GPU
library.

The arithmetic lives in ``prop_oracle.c`` (plain C, compiled with
``-ffp-contract=off``); this module builds it with gcc and wraps it with
ctypes.  See the header of ``prop_oracle.c`` for the passages of the paper
each step follows and for the readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "prop_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
SEQ_SOURCE = os.path.join(_HERE, "cpu_seq.c")
_SEQ_LIB_PATH = os.path.join(_HERE, "libcpuseq.so")

CONVERGED, INFEASIBLE, MAX_ROUNDS = 0, 1, 2
STATUS_NAMES = {CONVERGED: "CONVERGED", INFEASIBLE: "INFEASIBLE", MAX_ROUNDS: "MAX_ROUNDS"}

DEFAULT_EPS_INT = 1e-6
DEFAULT_CONT_REL_TOL = 1e-6
DEFAULT_FEAS_TOL = 1e-6

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=gnu11",
          "-Wall"]


def compile_library(src: str, out: str) -> str:
    """Compile an oracle source file into a shared library with gcc."""
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle library and the sequential baseline (no GPU code
    involved)."""
    if force or not os.path.exists(_LIB_PATH):
        compile_library(SOURCE, _LIB_PATH)
    if force or not os.path.exists(_SEQ_LIB_PATH):
        compile_library(SEQ_SOURCE, _SEQ_LIB_PATH)
    return _LIB_PATH


@dataclass
class Params:
    eps_int: float = DEFAULT_EPS_INT
    cont_rel_tol: float = DEFAULT_CONT_REL_TOL
    feas_tol: float = DEFAULT_FEAS_TOL


@dataclass
class Result:
    status: int
    rounds: int
    lb: np.ndarray
    ub: np.ndarray
    flags: int = 0


class OracleError(RuntimeError):
    pass


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _problem_arrays(inst):
    rp = np.ascontiguousarray(inst.row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(inst.col_idx, dtype=np.int32)
    va = np.ascontiguousarray(inst.vals, dtype=np.float64)
    lh = np.ascontiguousarray(inst.lhs, dtype=np.float64)
    rh = np.ascontiguousarray(inst.rhs, dtype=np.float64)
    vt = np.ascontiguousarray(inst.vartype, dtype=np.uint8)
    if rp.shape != (inst.m + 1,) or lh.shape != (inst.m,) or rh.shape != (inst.m,):
        raise ValueError("row arrays do not match m")
    if vt.shape != (inst.n,):
        raise ValueError("vartype does not match n")
    if ci.shape != va.shape or ci.shape[0] != rp[-1]:
        raise ValueError("col_idx / vals do not match row_ptr")
    return rp, ci, va, lh, rh, vt


class Oracle:
    """ctypes wrapper around one build of the oracle library."""

    def __init__(self, lib_path: str):
        lib = ctypes.CDLL(lib_path)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        lib.orc_exact_dot.argtypes = [P, P, i64]
        lib.orc_exact_dot.restype = f64
        lib.orc_activities.argtypes = [i32, i32, P, P, P, P, P, P, P, P, P]
        lib.orc_activities.restype = ctypes.c_int
        lib.orc_round.argtypes = [i32, i32, P, P, P, P, P, P, f64, f64, f64, P, P, P, P, P, P, P]
        lib.orc_round.restype = ctypes.c_int
        lib.orc_run.argtypes = [i32, i32, P, P, P, P, P, P, f64, f64, f64, P, P, i32, P, P, P]
        lib.orc_run.restype = ctypes.c_int
        lib.orc_run_seq.argtypes = [i32, i32, P, P, P, P, P, P, f64, f64, f64, P, P, i32, P, P]
        lib.orc_run_seq.restype = ctypes.c_int
        lib.orc_run_store.argtypes = [i32, i32, P, P, P, P, P, P, f64, f64, f64, i32, P, P, i32,
                                      P, P, P]
        lib.orc_run_store.restype = ctypes.c_int
        lib.orc_store_down.argtypes = [f64]
        lib.orc_store_down.restype = f64
        lib.orc_store_up.argtypes = [f64]
        lib.orc_store_up.restype = f64
        self.lib = lib
        self.path = lib_path

    def exact_dot(self, a, b) -> float:
        """Exact sum of a[i]*b[i], rounded once to the nearest double."""
        a = np.ascontiguousarray(a, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        assert a.shape == b.shape
        return float(self.lib.orc_exact_dot(_ptr(a), _ptr(b), a.size))

    def activities(self, inst, L, U):
        """Per row: (min finite part, min infinity count, max finite part, max count)."""
        rp, ci, va, _, _, _ = _problem_arrays(inst)
        L = np.ascontiguousarray(L, dtype=np.float64)
        U = np.ascontiguousarray(U, dtype=np.float64)
        m = inst.m
        mnf, mxf = np.zeros(m), np.zeros(m)
        mni, mxi = np.zeros(m, np.int64), np.zeros(m, np.int64)
        rc = self.lib.orc_activities(m, inst.n, _ptr(rp), _ptr(ci), _ptr(va), _ptr(L), _ptr(U),
                                     _ptr(mnf), _ptr(mni), _ptr(mxf), _ptr(mxi))
        if rc:
            raise OracleError(f"orc_activities failed: {rc}")
        return mnf, mni, mxf, mxi

    def round_(self, inst, L, U, params: Params | None = None):
        """One synchronous round from (L, U): (Ln, Un, changed, infeasible, flags)."""
        p = params or Params()
        rp, ci, va, lh, rh, vt = _problem_arrays(inst)
        L = np.ascontiguousarray(L, dtype=np.float64)
        U = np.ascontiguousarray(U, dtype=np.float64)
        Ln, Un = np.empty(inst.n), np.empty(inst.n)
        ch, inf = ctypes.c_int32(0), ctypes.c_int32(0)
        fl = ctypes.c_int64(0)
        rc = self.lib.orc_round(inst.m, inst.n, _ptr(rp), _ptr(ci), _ptr(va), _ptr(lh),
                                _ptr(rh), _ptr(vt), p.eps_int, p.cont_rel_tol, p.feas_tol,
                                _ptr(L), _ptr(U), _ptr(Ln), _ptr(Un), ctypes.byref(ch),
                                ctypes.byref(inf), ctypes.byref(fl))
        if rc:
            raise OracleError(f"orc_round failed: {rc}")
        return Ln, Un, bool(ch.value), bool(inf.value), int(fl.value)

    def run(self, inst, lb, ub, max_rounds: int = 100, params: Params | None = None,
            store: int = 64) -> Result:
        """Full synchronous propagation: status, rounds and the bounds.
        ``store=32`` keeps the bounds in single precision, rounded outward
        (reading R12 of ``prop_oracle.c``)."""
        p = params or Params()
        rp, ci, va, lh, rh, vt = _problem_arrays(inst)
        lb = np.array(lb, dtype=np.float64, copy=True)
        ub = np.array(ub, dtype=np.float64, copy=True)
        st, rd = ctypes.c_int32(0), ctypes.c_int32(0)
        fl = ctypes.c_int64(0)
        if store == 64:
            rc = self.lib.orc_run(inst.m, inst.n, _ptr(rp), _ptr(ci), _ptr(va), _ptr(lh),
                                  _ptr(rh), _ptr(vt), p.eps_int, p.cont_rel_tol, p.feas_tol,
                                  _ptr(lb), _ptr(ub), int(max_rounds), ctypes.byref(st),
                                  ctypes.byref(rd), ctypes.byref(fl))
        else:
            rc = self.lib.orc_run_store(inst.m, inst.n, _ptr(rp), _ptr(ci), _ptr(va), _ptr(lh),
                                        _ptr(rh), _ptr(vt), p.eps_int, p.cont_rel_tol,
                                        p.feas_tol, int(store), _ptr(lb), _ptr(ub),
                                        int(max_rounds), ctypes.byref(st), ctypes.byref(rd),
                                        ctypes.byref(fl))
        if rc:
            raise OracleError(f"orc_run failed: {rc}")
        return Result(st.value, rd.value, lb, ub, int(fl.value))

    def store_down(self, x: float) -> float:
        """Largest member of the single-precision store's grid not above x."""
        return float(self.lib.orc_store_down(float(x)))

    def store_up(self, x: float) -> float:
        """Smallest member of the single-precision store's grid not below x."""
        return float(self.lib.orc_store_up(float(x)))

    def run_seq(self, inst, lb, ub, max_sweeps: int = 1000,
                params: Params | None = None) -> Result:
        """Sequential propagation with constraint marking (rows in order)."""
        p = params or Params()
        rp, ci, va, lh, rh, vt = _problem_arrays(inst)
        lb = np.array(lb, dtype=np.float64, copy=True)
        ub = np.array(ub, dtype=np.float64, copy=True)
        st, sw = ctypes.c_int32(0), ctypes.c_int32(0)
        rc = self.lib.orc_run_seq(inst.m, inst.n, _ptr(rp), _ptr(ci), _ptr(va), _ptr(lh),
                                  _ptr(rh), _ptr(vt), p.eps_int, p.cont_rel_tol, p.feas_tol,
                                  _ptr(lb), _ptr(ub), int(max_sweeps), ctypes.byref(st),
                                  ctypes.byref(sw))
        if rc:
            raise OracleError(f"orc_run_seq failed: {rc}")
        return Result(st.value, sw.value, lb, ub)


_default: Oracle | None = None


def default() -> Oracle:
    global _default
    if _default is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        _default = Oracle(_LIB_PATH)
    return _default


def exact_dot(a, b) -> float:
    return default().exact_dot(a, b)


def activities(inst, L, U):
    return default().activities(inst, L, U)


def round_(inst, L, U, params: Params | None = None):
    return default().round_(inst, L, U, params)


def run(inst, lb, ub, max_rounds: int = 100, params: Params | None = None,
        store: int = 64) -> Result:
    return default().run(inst, lb, ub, max_rounds, params, store)


def run_seq(inst, lb, ub, max_sweeps: int = 1000, params: Params | None = None) -> Result:
    return default().run_seq(inst, lb, ub, max_sweeps, params)


class CpuSeq:
    """The paper's sequential baseline (Algorithm 1 with constraint marking,
    plain double sums in CSR order; ``cpu_seq.c``).  The column view is
    built once here; ``run`` times the propagation alone, single-threaded."""

    _lib = None

    def __init__(self, inst):
        if CpuSeq._lib is None:
            if not os.path.exists(_SEQ_LIB_PATH):
                compile_library(SEQ_SOURCE, _SEQ_LIB_PATH)
            lib = ctypes.CDLL(_SEQ_LIB_PATH)
            P = ctypes.c_void_p
            i32, f64 = ctypes.c_int32, ctypes.c_double
            lib.cs_create.argtypes = [i32, i32, P, P, P, P, P, P]
            lib.cs_create.restype = P
            lib.cs_destroy.argtypes = [P]
            lib.cs_destroy.restype = None
            lib.cs_run.argtypes = [P, f64, f64, f64, P, P, i32, P, P]
            lib.cs_run.restype = ctypes.c_int
            CpuSeq._lib = lib
        self._arrays = _problem_arrays(inst)  # kept alive: the C side borrows them
        rp, ci, va, lh, rh, vt = self._arrays
        self.n = inst.n
        self._h = CpuSeq._lib.cs_create(inst.m, inst.n, _ptr(rp), _ptr(ci), _ptr(va), _ptr(lh),
                                        _ptr(rh), _ptr(vt))
        if not self._h:
            raise OracleError("cs_create failed")

    def run(self, lb, ub, max_sweeps: int = 1000, params: Params | None = None):
        """(Result, seconds of the propagation itself)."""
        import time

        p = params or Params()
        lb = np.array(lb, dtype=np.float64, copy=True)
        ub = np.array(ub, dtype=np.float64, copy=True)
        st, sw = ctypes.c_int32(0), ctypes.c_int32(0)
        t0 = time.perf_counter()
        rc = CpuSeq._lib.cs_run(self._h, p.eps_int, p.cont_rel_tol, p.feas_tol, _ptr(lb),
                                _ptr(ub), int(max_sweeps), ctypes.byref(st), ctypes.byref(sw))
        dt = time.perf_counter() - t0
        if rc:
            raise OracleError(f"cs_run failed: {rc}")
        return Result(st.value, sw.value, lb, ub), dt

    def close(self):
        if self._h:
            CpuSeq._lib.cs_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

