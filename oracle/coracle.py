"""ctypes binding of the C oracle (``oracle/c/oracle.c``).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  ``build()`` compiles
``oracle/c/liboracle.so`` with gcc -O2 -fopenmp; ``load()`` returns the
library, building it if it is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "c", "oracle.c")
LIB = os.path.join(HERE, "c", "liboracle.so")

_lib = None


def build() -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-ffp-contract=off",
           SRC, "-o", LIB, "-lm"]
    subprocess.run(cmd, check=True)
    return LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    lib = ctypes.CDLL(LIB)
    i64, i32, p = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
    lib.orc_threads.restype = i32
    lib.orc_exact_entries.argtypes = [i32, i64, i64, i64, p, p, i64, p, p, p, p, p, p]
    lib.orc_exact_entries.restype = i32
    lib.orc_exponents.argtypes = [i64, i64, p, i64, i64, p, p]
    lib.orc_exponents.restype = i32
    lib.orc_method_entries.argtypes = [i32, i64, i64, i64, p, p, i32, i32, i32, i64, p, i64, p,
                                       p, p, p, p]
    lib.orc_method_entries.restype = i32
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def threads() -> int:
    return int(load().orc_threads())


def exact_entries(A: np.ndarray, B: np.ndarray, ii, jj, Cq=None):
    """Exact layer at entries (ii[e], jj[e]).

    Returns (Crn (nent, m): greedy RN words of C*, absab (nent,): RN of
    (|A||B|)_ij, err (nent,) or None: RN(C*_ij - sum of the words of Cq[e])).
    """
    lib = load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    m, M, K = A.shape
    N = B.shape[2]
    ii = np.ascontiguousarray(ii, dtype=np.int64)
    jj = np.ascontiguousarray(jj, dtype=np.int64)
    n = ii.shape[0]
    Crn = np.zeros((n, m))
    absab = np.zeros(n)
    err = None
    cq_ptr = None
    if Cq is not None:
        Cq = np.ascontiguousarray(Cq, dtype=np.float64).reshape(n, m)
        err = np.zeros(n)
        cq_ptr = _ptr(Cq)
    rc = lib.orc_exact_entries(m, M, N, K, _ptr(A), _ptr(B), n, _ptr(ii), _ptr(jj), cq_ptr,
                               _ptr(Crn), _ptr(absab), _ptr(err) if err is not None else None)
    if rc:
        raise RuntimeError(f"orc_exact_entries failed ({rc})")
    return Crn, absab, err


def exponents(lead: np.ndarray, by_columns: bool):
    """(E, span) per row of ``lead`` (R, K), or per column if by_columns."""
    lib = load()
    lead = np.ascontiguousarray(lead, dtype=np.float64)
    R0, C0 = lead.shape
    if by_columns:
        R, K, sr, sk = C0, R0, 1, C0
    else:
        R, K, sr, sk = R0, C0, C0, 1
    E = np.zeros(R, dtype=np.int32)
    span = np.zeros(R, dtype=np.int32)
    lib.orc_exponents(R, K, _ptr(lead), sr, sk, _ptr(E), _ptr(span))
    return E, span


def method_entries(A: np.ndarray, B: np.ndarray, beta: int, S: int, rows, cols,
                   balanced: bool = False):
    """Method layer for rows x cols: (E, F, D (nr, nc, S), C (m, nr, nc));
    ``balanced``: the balanced 8-bit digits (beta = 8)."""
    lib = load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    m, M, K = A.shape
    N = B.shape[2]
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    nr, nc = rows.shape[0], cols.shape[0]
    E = np.zeros(M, dtype=np.int32)
    F = np.zeros(N, dtype=np.int32)
    D = np.zeros((nr, nc, S), dtype=np.int64)
    C = np.zeros((nr, nc, m))
    rc = lib.orc_method_entries(m, M, N, K, _ptr(A), _ptr(B), beta, S, int(balanced), nr, _ptr(rows), nc,
                                _ptr(cols), _ptr(E), _ptr(F), _ptr(D), _ptr(C))
    if rc:
        raise RuntimeError(f"orc_method_entries failed ({rc})")
    return E, F, D, np.ascontiguousarray(np.transpose(C, (2, 0, 1)))
