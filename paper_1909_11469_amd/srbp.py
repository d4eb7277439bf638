"""ctypes binding of libsrbp (include/srbp.h): serial residual belief
propagation on the host CPU, the serial baseline the paper's speedups are
measured against.  Argument marshalling only."""
import ctypes
import os

import numpy as np

from . import bp as _bp

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsrbp.so")

EXPORTED = ["srbp_solve", "srbp_last_error"]


class srbp_stats(ctypes.Structure):
    _fields_ = [("updates", ctypes.c_int64), ("converged", ctypes.c_int32),
                ("timed_out", ctypes.c_int32), ("max_residual", ctypes.c_double),
                ("seconds", ctypes.c_double), ("evaluations", ctypes.c_int64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.srbp_solve.argtypes = [ctypes.POINTER(_bp.bp_graph_desc), ctypes.c_double, ctypes.c_int64,
                               ctypes.c_double, P, P, P, ctypes.c_int64,
                               ctypes.POINTER(srbp_stats)]
    lib.srbp_solve.restype = ctypes.c_int
    lib.srbp_last_error.argtypes = []
    lib.srbp_last_error.restype = ctypes.c_char_p
    return lib


lib = _load()


def srbp_solve(problem, eps=1e-4, max_updates=10 ** 9, time_limit_s=0.0, msgs=False,
               trace_len=0):
    """Serial residual BP on `problem` (the dict of inputs.py).  Returns a dict
    with marginals [N, K] FP64, the statistics, and optionally the final
    messages [E, K] and the first trace_len committed message ids."""
    d, keep = _bp._make_desc(problem)
    N, K = int(problem["N"]), int(problem["K"])
    E = 2 * int(np.asarray(problem["edges"]).reshape(-1, 2).shape[0])
    marg = np.zeros((N, K), np.float64)
    m = np.zeros((E, K), np.float64) if msgs else None
    tr = np.zeros(max(int(trace_len), 1), np.int64) if trace_len else None
    st = srbp_stats()
    rc = lib.srbp_solve(ctypes.byref(d), float(eps), int(max_updates), float(time_limit_s),
                        marg.ctypes.data_as(ctypes.c_void_p),
                        None if m is None else m.ctypes.data_as(ctypes.c_void_p),
                        None if tr is None else tr.ctypes.data_as(ctypes.c_void_p),
                        int(trace_len), ctypes.byref(st))
    del keep
    if rc < 0:
        raise _bp.BpError(rc, lib.srbp_last_error().decode())
    out = {f: getattr(st, f) for f, _ in st._fields_}
    out["converged"] = bool(out["converged"])
    out["timed_out"] = bool(out["timed_out"])
    out["marginals"] = marg
    if m is not None:
        out["msgs"] = m
    if tr is not None:
        out["trace"] = tr[:min(int(trace_len), out["updates"])]
    return out
