"""ctypes loader for the oracle's C/OpenMP stage 5 (test infrastructure only).

The shared object is compiled from oracle/cstage5.c by `build_cstage5()` (gcc, -O2,
-fopenmp); the graft entry's build() calls it.  Paper passage: Algorithm 1, stage 5.
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cstage5.c")
_SO = os.path.join(_HERE, "_cstage5.so")
_KINDS = {"exp": 0, "sqexp": 1, "exp_l1": 2, "const": 3, "lin": 4}
_lib = None


def build_cstage5():
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", _SO, "-lm"])
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build_cstage5()
        lib = ctypes.CDLL(_SO)
        lib.oracle_stage5_rows.restype = ctypes.c_int
        lib.oracle_stage5_rows.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int,
                                           ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                           ctypes.c_void_p]
        _lib = lib
    return _lib


def stage5(prob, Yp, rows=None, threads=0):
    """Z' = Gamma Y' for the oracle Problem `prob`, computed by the C/OpenMP loop.
    rows = (r0, r1) computes only those rows of Z' (a bounded timing sample); threads > 0
    fixes the number of OpenMP threads."""
    lib = _load()
    X = np.ascontiguousarray(prob.X, dtype=np.float64)
    one = Yp.ndim == 1
    Y = np.ascontiguousarray(Yp.reshape(len(Yp), -1), dtype=np.float64)
    r0, r1 = (0, X.shape[0]) if rows is None else (int(rows[0]), int(rows[1]))
    Z = np.empty((r1 - r0, Y.shape[1]), dtype=np.float64)
    d = X.shape[1]
    ell = np.ascontiguousarray(np.asarray(prob.cov.get("corr_len", [1.0] * d), dtype=np.float64)[:d])
    rc = lib.oracle_stage5_rows(d, X.shape[0], X.ctypes.data, Y.shape[1], Y.ctypes.data,
                                _KINDS[prob.cov["kind"]], float(prob.cov.get("sigma2", 1.0)),
                                ell.ctypes.data, r0, r1, int(threads), Z.ctypes.data)
    if rc != 0:
        raise RuntimeError("oracle_stage5 failed")
    return Z.reshape(-1) if one else Z
