"""Thin ctypes binding of libsvmhip.so: the C-ABI entry points under the same
names, plus helpers that marshal torch device tensors into the C structs.
Every step of training and classification runs in the library's HIP kernels;
this module only moves pointers.  Importing it fails loudly if the library has
not been built."""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsvmhip.so")

SVM_OK, SVM_NOT_CONVERGED = 0, 1
SVM_EINVAL, SVM_EONECLASS, SVM_ENONFINITE, SVM_EWORKSPACE, SVM_EHIP = -1, -2, -3, -4, -5
SVM_EUNSUPPORTED, SVM_ENOMEM, SVM_EBUSY, SVM_EABORT, SVM_ESCRATCH = -6, -7, -8, -9, -10
SVM_DENSE_ROW_MAJOR, SVM_DENSE_FEATURE_MAJOR, SVM_CSR = 0, 1, 2
SVM_KERNEL_FP32, SVM_KERNEL_FP64 = 0, 1
SVM_FLAG_WARM_START, SVM_FLAG_NO_FINAL_RECOMPUTE = 1, 2
SVM_FLAG_NO_LDS_PAYLOAD, SVM_FLAG_NO_LDS_STATE, SVM_FLAG_NO_BITSETS = 4, 8, 16
SVM_FLAG_KERNEL_MATRIX = 32

EXPORTS = ["svm_train_workspace_size", "svm_train", "svm_train_shared_workspace_size", "svm_train_shared",
           "svm_decision_workspace_size", "svm_decision",
           "svm_decision_noalloc", "svm_train_batch", "svm_autotune", "svm_autotune_reset", "svm_server_create",
           "svm_server_submit", "svm_server_poll", "svm_server_drain", "svm_server_stats", "svm_server_destroy",
           "svm_strerror", "svm_version", "svm_debug_select", "svm_debug_set_trace", "svm_debug_set_profile",
           "svm_debug_step_info"]


class svm_problem_t(C.Structure):
    _fields_ = [("n", C.c_int32), ("d", C.c_int32), ("layout", C.c_int32), ("reserved", C.c_int32),
                ("x", C.c_void_p), ("ldx", C.c_int64), ("row_ptr", C.c_void_p), ("col", C.c_void_p),
                ("val", C.c_void_p), ("y", C.c_void_p)]


class svm_params_t(C.Structure):
    _fields_ = [("C", C.c_double), ("gamma", C.c_double), ("eps", C.c_double), ("shrink_mode", C.c_int32),
                ("shrink_kind", C.c_int32), ("shrink_param", C.c_double), ("max_iter", C.c_int64),
                ("kernel_precision", C.c_int32), ("flags", C.c_uint32), ("grid_blocks", C.c_int32),
                ("lanes_per_row", C.c_int32), ("head_cols", C.c_int32), ("cache_mb", C.c_int32)]


SVM_TUNE_GRID, SVM_TUNE_TEAM = 0, 1


class svm_tune_t(C.Structure):
    _fields_ = [("target", C.c_int32), ("chosen", C.c_int32), ("n_candidates", C.c_int32), ("reserved", C.c_int32),
                ("shape", C.c_int32 * 8), ("us_per_iter", C.c_double * 8)]

    def as_dict(self):
        k = self.n_candidates
        return {"target": self.target, "chosen": self.chosen,
                "candidates": [{"shape": self.shape[i], "us_per_iter": self.us_per_iter[i]} for i in range(k)]}


class svm_result_t(C.Structure):
    _fields_ = [("beta", C.c_double), ("b_up", C.c_double), ("b_low", C.c_double), ("dual_obj", C.c_double),
                ("iterations", C.c_int64), ("n_sv", C.c_int32), ("n_bsv", C.c_int32), ("n_recon", C.c_int32),
                ("status", C.c_int32), ("shrink_passes", C.c_int64), ("shrunk_total", C.c_int64),
                ("n_launches", C.c_int32), ("grid_blocks", C.c_int32), ("ms_total", C.c_double),
                ("ms_step", C.c_double), ("ms_recon", C.c_double), ("rows_streamed", C.c_int64),
                ("nnz_streamed", C.c_int64), ("pattern_only", C.c_int32), ("lanes_per_row", C.c_int32),
                ("ksum_mfma", C.c_int32), ("ms_ksum", C.c_double), ("recon_pairs", C.c_int64),
                ("head_cols", C.c_int32), ("cache_rows", C.c_int32), ("rows_read", C.c_int64),
                ("cache_values", C.c_int64), ("cache_both", C.c_int64), ("kernel_matrix", C.c_int32),
                ("reserved", C.c_int32), ("ms_kmatrix", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsvmhip.so is not built: run __graft_entry__.build() "
                               "(hipcc --offload-arch=gfx950) first")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.svm_train_workspace_size.argtypes = [P(svm_problem_t), P(svm_params_t)]
        L.svm_train_workspace_size.restype = C.c_size_t
        L.svm_train.argtypes = [P(svm_problem_t), P(svm_params_t), C.c_void_p, C.c_void_p, P(svm_result_t),
                                C.c_void_p, C.c_size_t, C.c_void_p]
        L.svm_train_shared_workspace_size.argtypes = [P(svm_problem_t), C.c_int32, P(C.c_void_p), P(svm_params_t)]
        L.svm_train_shared_workspace_size.restype = C.c_size_t
        L.svm_train_shared.argtypes = [P(svm_problem_t), C.c_int32, P(C.c_void_p), P(svm_params_t), P(C.c_void_p),
                                       P(C.c_void_p), P(svm_result_t), C.c_void_p, C.c_size_t, C.c_void_p]
        L.svm_decision_workspace_size.argtypes = [P(svm_problem_t), P(svm_problem_t), C.c_int32]
        L.svm_decision_workspace_size.restype = C.c_size_t
        L.svm_decision.argtypes = [P(svm_problem_t), C.c_void_p, C.c_double, C.c_double, P(svm_problem_t),
                                   C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p]
        L.svm_decision_noalloc.argtypes = [P(svm_problem_t), C.c_void_p, C.c_double, C.c_double, P(svm_problem_t),
                                           C.c_void_p, C.c_int32, C.c_void_p]
        L.svm_autotune.argtypes = [P(svm_problem_t), P(svm_params_t), C.c_int32, P(svm_tune_t), C.c_void_p]
        L.svm_train_batch.argtypes = [C.c_int32, P(svm_problem_t), P(svm_params_t), P(C.c_void_p), P(C.c_void_p),
                                      P(svm_result_t), C.c_void_p]
        L.svm_server_create.argtypes = [C.c_size_t, C.c_int32, P(C.c_void_p)]
        L.svm_server_submit.argtypes = [C.c_void_p, P(svm_problem_t), P(svm_params_t), C.c_void_p,
                                        P(C.c_int64)]
        L.svm_server_poll.argtypes = [C.c_void_p, C.c_int64, P(svm_result_t)]
        L.svm_server_drain.argtypes = [C.c_void_p]
        L.svm_server_stats.argtypes = [C.c_void_p, P(C.c_int64), P(C.c_int64), P(C.c_int64), P(C.c_int64)]
        L.svm_server_destroy.argtypes = [C.c_void_p]
        L.svm_strerror.argtypes = [C.c_int]
        L.svm_strerror.restype = C.c_char_p
        L.svm_debug_select.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                       C.c_int32, P(C.c_double), P(C.c_int32), P(C.c_double), P(C.c_int32),
                                       C.c_void_p]
        L.svm_debug_set_trace.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.svm_debug_set_profile.argtypes = [C.c_void_p]
        L.svm_debug_step_info.argtypes = [P(C.c_int32), P(C.c_int32), P(C.c_int32)]
        _lib = L
    return _lib


def strerror(rc: int) -> str:
    return lib().svm_strerror(int(rc)).decode()


# ------------------------------------------------------------------ torch marshalling

def _torch():
    import torch
    return torch


@dataclass
class DeviceProblem:
    """A sample set resident in device memory plus its svm_problem_t view."""
    s: svm_problem_t
    keep: tuple
    n: int
    d: int


def to_device(data, device="cuda", layout: Optional[int] = None, with_labels: bool = True) -> DeviceProblem:
    """Copy an ``SvmData`` (dense float32 rows or CSR) to the device."""
    torch = _torch()
    y = torch.from_numpy(np.ascontiguousarray(data.y, np.int8)).to(device) if (with_labels and data.y is not None) \
        else None
    if data.layout == "csr":
        rp = torch.from_numpy(np.ascontiguousarray(data.row_ptr, np.int32)).to(device)
        col = torch.from_numpy(np.ascontiguousarray(data.col, np.int32)).to(device)
        val = torch.from_numpy(np.ascontiguousarray(data.val, np.float32)).to(device)
        s = svm_problem_t(data.n, data.d, SVM_CSR, 0, None, 0, rp.data_ptr(), col.data_ptr(),
                          val.data_ptr(), y.data_ptr() if y is not None else None)
        keep = (rp, col, val, y)
    else:
        lay = SVM_DENSE_ROW_MAJOR if layout is None else layout
        xh = np.ascontiguousarray(data.x, np.float32)
        if lay == SVM_DENSE_FEATURE_MAJOR:
            x = torch.from_numpy(np.ascontiguousarray(xh.T)).to(device)
            ldx = data.n
        else:
            x = torch.from_numpy(xh).to(device)
            ldx = data.d
        s = svm_problem_t(data.n, data.d, lay, 0, x.data_ptr(), ldx, None, None, None,
                          y.data_ptr() if y is not None else None)
        keep = (x, y)
    return DeviceProblem(s, keep, data.n, data.d)


def make_params(C_, gamma, eps=1e-3, shrink_mode=0, shrink_kind=0, shrink_param=0.0, max_iter=10**9,
                kernel_precision=SVM_KERNEL_FP32, flags=0, grid_blocks=0, lanes_per_row=0,
                head_cols=0, cache_mb=0) -> svm_params_t:
    return svm_params_t(float(C_), float(gamma), float(eps), int(shrink_mode), int(shrink_kind), float(shrink_param),
                        int(max_iter), int(kernel_precision), int(flags), int(grid_blocks), int(lanes_per_row),
                        int(head_cols), int(cache_mb))


def params_for(cfg, **kw) -> svm_params_t:
    kw.setdefault("max_iter", cfg.max_iter)
    return make_params(cfg.C, cfg.gamma, cfg.eps, cfg.shrink_mode, cfg.shrink_kind, cfg.shrink_param, **kw)


def current_stream_ptr():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------------ entry points (same names as the C-ABI)

def svm_train_workspace_size(prob: DeviceProblem, params: svm_params_t) -> int:
    return int(lib().svm_train_workspace_size(C.byref(prob.s), C.byref(params)))


def svm_train(prob: DeviceProblem, params: svm_params_t, alpha, f=None, workspace=None, stream=None):
    """alpha, f: float64 device tensors of length n (f may be None); workspace: uint8 device
    tensor or None.  Returns (rc, svm_result_t)."""
    res = svm_result_t()
    ws_ptr, ws_bytes = (None, 0) if workspace is None else (workspace.data_ptr(), workspace.numel())
    rc = lib().svm_train(C.byref(prob.s), C.byref(params), alpha.data_ptr(),
                         f.data_ptr() if f is not None else None, C.byref(res), ws_ptr, ws_bytes,
                         stream if stream is not None else current_stream_ptr())
    return rc, res


def svm_train_shared(prob: DeviceProblem, ys, params, alphas, fs=None, workspace=None, stream=None):
    """Several problems over the samples of `prob` (its labels unused): ys[p] int8 device
    labels, params[p] svm_params_t, alphas[p] / fs[p] float64 device tensors.  Returns (rc,
    [svm_result_t])."""
    k = len(ys)
    yarr = (C.c_void_p * k)(*[t.data_ptr() for t in ys])
    qarr = (svm_params_t * k)(*params)
    aarr = (C.c_void_p * k)(*[a.data_ptr() for a in alphas])
    farr = (C.c_void_p * k)(*[(f.data_ptr() if f is not None else None) for f in (fs or [None] * k)])
    res = (svm_result_t * k)()
    ws_ptr, ws_bytes = (None, 0) if workspace is None else (workspace.data_ptr(), workspace.numel())
    rc = lib().svm_train_shared(C.byref(prob.s), k, yarr, qarr, aarr, farr, res, ws_ptr, ws_bytes,
                                stream if stream is not None else current_stream_ptr())
    return rc, [res[i] for i in range(k)]


def svm_train_shared_workspace_size(prob: DeviceProblem, ys, params) -> int:
    k = len(ys)
    yarr = (C.c_void_p * k)(*[t.data_ptr() for t in ys])
    qarr = (svm_params_t * k)(*params)
    return int(lib().svm_train_shared_workspace_size(C.byref(prob.s), k, yarr, qarr))


def svm_decision_workspace_size(train: DeviceProblem, queries: DeviceProblem,
                                kernel_precision=SVM_KERNEL_FP32) -> int:
    return int(lib().svm_decision_workspace_size(C.byref(train.s), C.byref(queries.s), int(kernel_precision)))


def svm_decision(train: DeviceProblem, alpha, beta: float, gamma: float, queries: DeviceProblem, out,
                 kernel_precision=SVM_KERNEL_FP32, workspace=None, stream=None) -> int:
    """workspace: uint8 device tensor of at least svm_decision_workspace_size() bytes, or None
    (the library then allocates its scratch on the stream)."""
    ws_ptr, ws_bytes = (None, 0) if workspace is None else (workspace.data_ptr(), workspace.numel())
    return lib().svm_decision(C.byref(train.s), alpha.data_ptr(), float(beta), float(gamma), C.byref(queries.s),
                              out.data_ptr(), int(kernel_precision), ws_ptr, ws_bytes,
                              stream if stream is not None else current_stream_ptr())


def svm_decision_noalloc(train: DeviceProblem, alpha, beta: float, gamma: float, queries: DeviceProblem, out,
                         kernel_precision=SVM_KERNEL_FP32, stream=None) -> int:
    """svm_decision on the library's built-in scratch (no allocation)."""
    return lib().svm_decision_noalloc(C.byref(train.s), alpha.data_ptr(), float(beta), float(gamma),
                                      C.byref(queries.s), out.data_ptr(), int(kernel_precision),
                                      stream if stream is not None else current_stream_ptr())


def svm_autotune(prob: DeviceProblem, params: svm_params_t, target: int, stream=None):
    """Returns (rc, dict of the candidates timed and the shape chosen)."""
    t = svm_tune_t()
    rc = lib().svm_autotune(C.byref(prob.s), C.byref(params), int(target), C.byref(t),
                            stream if stream is not None else current_stream_ptr())
    return rc, t.as_dict()


def svm_autotune_reset() -> int:
    return lib().svm_autotune_reset()


def svm_debug_select(active, f, alpha, y, C_, num_blocks=0, stream=None):
    bu, bl = C.c_double(), C.c_double()
    iu, il = C.c_int32(), C.c_int32()
    rc = lib().svm_debug_select(int(active.numel()), active.data_ptr(), f.data_ptr(), alpha.data_ptr(),
                                y.data_ptr(), float(C_), int(num_blocks), C.byref(bu), C.byref(iu), C.byref(bl),
                                C.byref(il), stream if stream is not None else current_stream_ptr())
    return rc, (bu.value, iu.value, bl.value, il.value)


def svm_debug_set_trace(cap, i_up=None, i_low=None, b_up=None, b_low=None) -> int:
    if not cap:
        return lib().svm_debug_set_trace(0, None, None, None, None)
    return lib().svm_debug_set_trace(int(cap), i_up.data_ptr(), i_low.data_ptr(), b_up.data_ptr(),
                                     b_low.data_ptr())


def svm_debug_set_profile(slots) -> int:
    """slots: uint64/int64 device tensor of 8 entries, or None to switch the timer off."""
    return lib().svm_debug_set_profile(slots.data_ptr() if slots is not None else None)


def svm_debug_step_info():
    m, g, l = C.c_int32(), C.c_int32(), C.c_int32()
    lib().svm_debug_step_info(C.byref(m), C.byref(g), C.byref(l))
    return m.value, g.value, l.value


def svm_train_batch(probs, params, alphas, fs=None, stream=None):
    k = len(probs)
    parr = (svm_problem_t * k)(*[p.s for p in probs])
    qarr = (svm_params_t * k)(*params)
    aarr = (C.c_void_p * k)(*[a.data_ptr() for a in alphas])
    farr = (C.c_void_p * k)(*[(f.data_ptr() if f is not None else None) for f in (fs or [None] * k)])
    res = (svm_result_t * k)()
    rc = lib().svm_train_batch(k, parr, qarr, aarr, farr, res, stream if stream is not None else current_stream_ptr())
    return rc, [res[i] for i in range(k)]


# ------------------------------------------------------------------ convenience

@dataclass
class TrainOutput:
    rc: int
    alpha: np.ndarray
    f: np.ndarray
    result: dict


def train_data(data, C_, gamma, eps=1e-3, device="cuda", **kw) -> TrainOutput:
    """Train on an ``SvmData`` held on the host (copied to the device first)."""
    torch = _torch()
    dp = to_device(data, device)
    params = make_params(C_, gamma, eps, **kw)
    alpha = torch.zeros(data.n, dtype=torch.float64, device=device)
    f = torch.zeros(data.n, dtype=torch.float64, device=device)
    rc, res = svm_train(dp, params, alpha, f)
    torch.cuda.synchronize()
    return TrainOutput(rc, alpha.cpu().numpy(), f.cpu().numpy(), res.as_dict())


def train_config(cfg, device="cuda", **kw) -> TrainOutput:
    kw.setdefault("max_iter", cfg.max_iter)
    return train_data(cfg.data, cfg.C, cfg.gamma, cfg.eps, device, shrink_mode=cfg.shrink_mode,
                      shrink_kind=cfg.shrink_kind, shrink_param=cfg.shrink_param, **kw)


def decision_data(train, alpha: np.ndarray, beta: float, gamma: float, queries, device="cuda",
                  kernel_precision=SVM_KERNEL_FP32) -> np.ndarray:
    torch = _torch()
    tp = to_device(train, device)
    qp = to_device(queries, device, with_labels=False)
    a = torch.from_numpy(np.ascontiguousarray(alpha, np.float64)).to(device)
    out = torch.zeros(queries.n, dtype=torch.float64, device=device)
    rc = svm_decision(tp, a, beta, gamma, qp, out, kernel_precision)
    if rc != SVM_OK:
        raise RuntimeError("svm_decision failed: %s" % strerror(rc))
    torch.cuda.synchronize()
    return out.cpu().numpy()


# ------------------------------------------------------------------ serving

class Server:
    """Continuous-batching server of training problems (svm_server_* of the C-ABI)."""

    def __init__(self, hbm_budget: int, max_slots: int):
        h = C.c_void_p()
        rc = lib().svm_server_create(int(hbm_budget), int(max_slots), C.byref(h))
        if rc != SVM_OK:
            raise RuntimeError("svm_server_create failed: %s" % strerror(rc))
        self.h = h
        self.keep = {}

    def submit(self, prob: DeviceProblem, params: svm_params_t, alpha) -> int:
        t = C.c_int64()
        rc = lib().svm_server_submit(self.h, C.byref(prob.s), C.byref(params), alpha.data_ptr(), C.byref(t))
        if rc != SVM_OK:
            raise RuntimeError("svm_server_submit failed: %s" % strerror(rc))
        self.keep[t.value] = (prob, alpha)
        return t.value

    def poll(self, ticket: int):
        res = svm_result_t()
        rc = lib().svm_server_poll(self.h, int(ticket), C.byref(res))
        if rc == SVM_EBUSY:
            return None
        self.keep.pop(ticket, None)
        return rc, res

    def drain(self) -> int:
        return lib().svm_server_drain(self.h)

    def stats(self) -> dict:
        a, d, c, f = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        lib().svm_server_stats(self.h, C.byref(a), C.byref(d), C.byref(c), C.byref(f))
        return {"admitted": a.value, "deferred": d.value, "completed": c.value, "in_flight": f.value}

    def close(self):
        if self.h:
            lib().svm_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
