"""ORACLE — test infrastructure only.

Plain, slow, obviously correct CPU implementations that the GPU path is
checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package; the library under
``paper_2501_06872_amd`` never does, and it shares no code with it.

* ``transpose``       — Algorithm 1 (Atomic GT, Section II-B) run by one thread
                        (C, ``gt_oracle.c``): CSC lists in increasing CSR edge
                        position, i.e. ascending source, multi-edges in CSR order.
* ``transpose_slice`` — the same restricted to a destination range, for checks
                        of full-size outputs on chosen vertex ranges.
* ``transpose_py``    — the definition written out in pure Python (small cases).
* ``features``        — the degree-sampling pass and feature vector (numpy).
* ``mlp``             — fp64 forward/backward/Adam of the parameter-choice network.
* ``random_access``   — replay of the random-access microbenchmark (Fig. 3):
                        the indices every thread visits and what each access
                        kind leaves behind.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRCS = [os.path.join(_HERE, "gt_oracle.c")]

ORC_OK, ORC_EINVAL, ORC_EGRAPH, ORC_ENOMEM, ORC_EINTERNAL = 0, 1, 2, 3, 4


def build():
    """Compile the C oracle (plain gcc, no OpenMP, no SIMD intrinsics)."""
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-Wall", "-o", _SO] + _SRCS)


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or any(os.path.getmtime(_SO) < os.path.getmtime(s) for s in _SRCS):
            build()
        lib = ctypes.CDLL(_SO)
        i64, vp = ctypes.c_int64, ctypes.c_void_p
        lib.gt_oracle_validate.argtypes = [i64, i64, vp, vp]
        lib.gt_oracle_transpose.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp]
        lib.gt_oracle_transpose_slice.argtypes = [i64, i64, vp, vp, vp, i64, i64, vp, vp, vp]
        for f in (lib.gt_oracle_validate, lib.gt_oracle_transpose, lib.gt_oracle_transpose_slice):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _prep(O, D, P):
    O = np.ascontiguousarray(O, dtype=np.int64)
    D = np.ascontiguousarray(D, dtype=np.int32)
    if P is not None:
        P = np.ascontiguousarray(P).view(np.uint32)
    return O, D, P


class OracleError(ValueError):
    pass


def validate(O, D):
    O, D, _ = _prep(O, D, None)
    n, m = O.size - 1, D.size
    return _load().gt_oracle_validate(n, m, _p(O), _p(D))


def transpose(O, D, P=None):
    """Return (T int64[n+1], S int32[m], Q uint32[m] or None)."""
    O, D, P = _prep(O, D, P)
    n, m = O.size - 1, D.size
    T = np.empty(n + 1, dtype=np.int64)
    S = np.empty(m, dtype=np.int32)
    Q = np.empty(m, dtype=np.uint32) if P is not None else None
    rc = _load().gt_oracle_transpose(n, m, _p(O), _p(D), _p(P), _p(T), _p(S), _p(Q))
    if rc != ORC_OK:
        raise OracleError(f"oracle transpose failed ({rc})")
    return T, S, Q


def transpose_slice(O, D, P, lo, hi):
    """T[lo..hi] and the concatenated lists of the vertices [lo, hi)."""
    O, D, P = _prep(O, D, P)
    n, m = O.size - 1, D.size
    lib = _load()
    # the slice length is only known after counting: size S by a first count
    Tsl = np.empty(hi - lo + 1, dtype=np.int64)
    cnt = int(np.count_nonzero((D >= lo) & (D < hi)))
    S = np.empty(max(cnt, 1), dtype=np.int32)
    Q = np.empty(max(cnt, 1), dtype=np.uint32) if P is not None else None
    rc = lib.gt_oracle_transpose_slice(n, m, _p(O), _p(D), _p(P), lo, hi, _p(Tsl), _p(S), _p(Q))
    if rc != ORC_OK:
        raise OracleError(f"oracle slice failed ({rc})")
    return Tsl, S[:cnt], (Q[:cnt] if Q is not None else None)


def transpose_py(O, D, P=None):
    """Pure-Python statement of the definition (small inputs only):
    T[v] = #{e : D[e] < v}; the slots T[v]..T[v+1]-1 hold (src(e), P[e]) of
    the edges with D[e] = v in increasing e (Section II-A)."""
    O = [int(x) for x in O]
    D = [int(x) for x in D]
    n, m = len(O) - 1, len(D)
    src = []
    for u in range(n):
        for _ in range(O[u], O[u + 1]):
            src.append(u)
    T = [sum(1 for e in range(m) if D[e] < v) for v in range(n + 1)]
    S, Q = [], []
    for v in range(n):
        for e in range(m):
            if D[e] == v:
                S.append(src[e])
                if P is not None:
                    Q.append(int(P[e]))
    return T, S, (Q if P is not None else None)
