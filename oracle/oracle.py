"""ctypes binding of the FP64 CPU oracle (``smo_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  It shares no
code with the HIP library; both are fed by ``paper_1406_5161_amd.datagen``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "smo_oracle.c")
LIB = os.path.join(HERE, "libsmo_oracle.so")

OK, NOT_CONVERGED, EINVAL, EONECLASS, ENONFINITE = 0, 1, -1, -2, -3


def build(force: bool = True) -> str:
    """Compile the oracle with plain gcc (-O2, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", "-fopenmp",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def _default_threads() -> int:
    """ORACLE_THREADS if set, else every core this process may run on."""
    v = os.environ.get("ORACLE_THREADS")
    if v:
        return max(1, int(v))
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return max(1, os.cpu_count() or 1)


def set_threads(t: int) -> int:
    """Threads for the oracle's per-sample loops; results do not depend on it."""
    return lib().orc_set_threads(int(t))


def get_threads() -> int:
    return lib().orc_get_threads()


class _Data(C.Structure):
    _fields_ = [("n", C.c_int32), ("d", C.c_int32), ("is_csr", C.c_int32),
                ("x", C.c_void_p), ("row_ptr", C.c_void_p), ("col", C.c_void_p),
                ("val", C.c_void_p), ("y", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("C", C.c_double), ("gamma", C.c_double), ("eps", C.c_double),
                ("shrink_mode", C.c_int32), ("shrink_kind", C.c_int32), ("shrink_param", C.c_double),
                ("max_iter", C.c_int64), ("dual_fresh", C.c_int32), ("pad", C.c_int32)]


class _Result(C.Structure):
    _fields_ = [("beta", C.c_double), ("b_up", C.c_double), ("b_low", C.c_double),
                ("dual_obj", C.c_double), ("iterations", C.c_int64), ("n_sv", C.c_int32),
                ("n_bsv", C.c_int32), ("n_recon", C.c_int32), ("status", C.c_int32),
                ("shrink_passes", C.c_int64), ("shrunk_total", C.c_int64)]


class _Trace(C.Structure):
    _fields_ = [("cap", C.c_int64), ("count", C.c_int64), ("i_up", C.c_void_p), ("i_low", C.c_void_p),
                ("b_up", C.c_void_p), ("b_low", C.c_void_p), ("obj", C.c_void_p), ("n_active", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = C.CDLL(LIB)
        P = C.POINTER
        L.orc_train.argtypes = [P(_Data), P(_Params), C.c_void_p, C.c_void_p, P(_Result), P(_Trace)]
        L.orc_train.restype = C.c_int
        L.orc_kernel.argtypes = [P(_Data), C.c_int64, P(_Data), C.c_int64, C.c_double]
        L.orc_kernel.restype = C.c_double
        L.orc_f_full.argtypes = [P(_Data), C.c_void_p, C.c_double, C.c_void_p]
        L.orc_dual.argtypes = [P(_Data), C.c_void_p, C.c_double]
        L.orc_dual.restype = C.c_double
        L.orc_decision.argtypes = [P(_Data), C.c_void_p, C.c_double, C.c_double, P(_Data), C.c_void_p]
        L.orc_select.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                 P(C.c_double), P(C.c_int32), P(C.c_double), P(C.c_int32)]
        L.orc_pair_update.argtypes = [C.c_double, C.c_double, C.c_int8, C.c_int8, C.c_double, C.c_double,
                                      C.c_double, C.c_double, C.c_double, C.c_double,
                                      P(C.c_double), P(C.c_double)]
        L.orc_set_id.argtypes = [C.c_int8, C.c_double, C.c_double]
        L.orc_set_id.restype = C.c_int32
        L.orc_validate.argtypes = [P(_Data), P(_Params)]
        L.orc_validate.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = C.c_int
        L.orc_get_threads.restype = C.c_int
        L.orc_max_threads.restype = C.c_int
        _lib = L
        L.orc_set_threads(_default_threads())
    return _lib


class OracleData:
    """FP64 copy of an SvmData (values are float32-representable, read exactly)."""

    def __init__(self, data, y: Optional[np.ndarray] = None):
        self.n, self.d = int(data.n), int(data.d)
        self.is_csr = data.layout == "csr"
        yy = data.y if y is None else y
        self.y = np.ascontiguousarray(yy, dtype=np.int8) if yy is not None else None
        if self.is_csr:
            self.row_ptr = np.ascontiguousarray(data.row_ptr, dtype=np.int32)
            self.col = np.ascontiguousarray(data.col, dtype=np.int32)
            self.val = np.ascontiguousarray(data.val, dtype=np.float64)
            self.x = None
        else:
            self.x = np.ascontiguousarray(data.x, dtype=np.float64)
            self.row_ptr = self.col = self.val = None
        self.s = _Data(self.n, self.d, int(self.is_csr),
                       self.x.ctypes.data if self.x is not None else None,
                       self.row_ptr.ctypes.data if self.is_csr else None,
                       self.col.ctypes.data if self.is_csr else None,
                       self.val.ctypes.data if self.is_csr else None,
                       self.y.ctypes.data if self.y is not None else None)


def _params(C_, gamma, eps, shrink_mode=0, shrink_kind=0, shrink_param=0.0, max_iter=10**12, dual_fresh=0):
    return _Params(float(C_), float(gamma), float(eps), int(shrink_mode), int(shrink_kind),
                   float(shrink_param), int(max_iter), int(dual_fresh), 0)


@dataclass
class OracleResult:
    rc: int
    alpha: np.ndarray
    f: np.ndarray
    beta: float
    b_up: float
    b_low: float
    dual_obj: float
    iterations: int
    n_sv: int
    n_bsv: int
    n_recon: int
    status: int
    shrink_passes: int
    shrunk_total: int
    trace: Optional[dict] = None


def train(data, C_, gamma, eps=1e-3, shrink_mode=0, shrink_kind=0, shrink_param=0.0,
          max_iter=10**12, dual_fresh=False, trace_cap=0, trace_obj=False) -> OracleResult:
    od = data if isinstance(data, OracleData) else OracleData(data)
    p = _params(C_, gamma, eps, shrink_mode, shrink_kind, shrink_param, max_iter, int(dual_fresh))
    alpha = np.zeros(od.n)
    f = np.zeros(od.n)
    r = _Result()
    tr = None
    arrs = None
    if trace_cap:
        arrs = dict(i_up=np.zeros(trace_cap, np.int32), i_low=np.zeros(trace_cap, np.int32),
                    b_up=np.zeros(trace_cap), b_low=np.zeros(trace_cap),
                    n_active=np.zeros(trace_cap, np.int32))
        if trace_obj:
            arrs["obj"] = np.zeros(trace_cap)
        tr = _Trace(trace_cap, 0, arrs["i_up"].ctypes.data, arrs["i_low"].ctypes.data,
                    arrs["b_up"].ctypes.data, arrs["b_low"].ctypes.data,
                    arrs["obj"].ctypes.data if trace_obj else None, arrs["n_active"].ctypes.data)
    rc = lib().orc_train(C.byref(od.s), C.byref(p), alpha.ctypes.data, f.ctypes.data, C.byref(r),
                         C.byref(tr) if tr is not None else None)
    trace = None
    if tr is not None:
        trace = {k: v[:tr.count].copy() for k, v in arrs.items()}
    return OracleResult(rc, alpha, f, r.beta, r.b_up, r.b_low, r.dual_obj, r.iterations, r.n_sv, r.n_bsv,
                        r.n_recon, r.status, r.shrink_passes, r.shrunk_total, trace)


def train_config(cfg, **kw) -> OracleResult:
    kw.setdefault("max_iter", cfg.max_iter)
    return train(cfg.data, cfg.C, cfg.gamma, cfg.eps, cfg.shrink_mode, cfg.shrink_kind, cfg.shrink_param, **kw)


def validate(data, C_=1.0, gamma=1.0, eps=1e-3, shrink_mode=0, shrink_param=0.0) -> int:
    od = data if isinstance(data, OracleData) else OracleData(data)
    p = _params(C_, gamma, eps, shrink_mode, 0, shrink_param)
    return lib().orc_validate(C.byref(od.s), C.byref(p))


def kernel(A, i, B, j, gamma) -> float:
    oa = A if isinstance(A, OracleData) else OracleData(A)
    ob = B if isinstance(B, OracleData) else OracleData(B)
    return lib().orc_kernel(C.byref(oa.s), int(i), C.byref(ob.s), int(j), float(gamma))


def f_full(data, alpha, gamma) -> np.ndarray:
    od = data if isinstance(data, OracleData) else OracleData(data)
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    out = np.zeros(od.n)
    lib().orc_f_full(C.byref(od.s), a.ctypes.data, float(gamma), out.ctypes.data)
    return out


def dual(data, alpha, gamma) -> float:
    od = data if isinstance(data, OracleData) else OracleData(data)
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    return lib().orc_dual(C.byref(od.s), a.ctypes.data, float(gamma))


def decision(train_data, alpha, beta, gamma, queries) -> np.ndarray:
    ot = train_data if isinstance(train_data, OracleData) else OracleData(train_data)
    oq = queries if isinstance(queries, OracleData) else OracleData(queries, y=np.zeros(queries.n, np.int8))
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    out = np.zeros(oq.n)
    lib().orc_decision(C.byref(ot.s), a.ctypes.data, float(beta), float(gamma), C.byref(oq.s), out.ctypes.data)
    return out


def select(S, f, alpha, y, C_):
    S = np.ascontiguousarray(S, dtype=np.int32)
    f = np.ascontiguousarray(f, dtype=np.float64)
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.int8)
    bu, bl = C.c_double(), C.c_double()
    iu, il = C.c_int32(), C.c_int32()
    lib().orc_select(len(S), S.ctypes.data, f.ctypes.data, alpha.ctypes.data, y.ctypes.data, float(C_),
                     C.byref(bu), C.byref(iu), C.byref(bl), C.byref(il))
    return bu.value, iu.value, bl.value, il.value


def pair_update(a_up, a_low, y_up, y_low, f_up, f_low, K_uu, K_ll, K_ul, C_):
    nu, nl = C.c_double(), C.c_double()
    lib().orc_pair_update(float(a_up), float(a_low), int(y_up), int(y_low), float(f_up), float(f_low),
                          float(K_uu), float(K_ll), float(K_ul), float(C_), C.byref(nu), C.byref(nl))
    return nu.value, nl.value


def set_id(y, a, C_) -> int:
    return lib().orc_set_id(int(y), float(a), float(C_))
