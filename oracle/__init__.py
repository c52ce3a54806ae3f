"""FP64 CPU oracle for Secant-Avoidance Projection -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``sap_oracle.c`` (plain C,
FP64, OpenMP) through ctypes and shares nothing with the HIP library.

Every function takes numpy arrays in the layouts of the workload generator:
X is N x n (float32 or float64; promoted exactly to float64 here), P is n x k
float64 with orthonormal columns.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "sap_oracle.c"
_LIB = _HERE / "libsap_oracle.so"

OK, EARG, ENOPAIRS, EDEGENERATE, ENOMEM = 0, 1, 2, 3, 4


class OracleError(RuntimeError):
    pass


class _MinT(C.Structure):
    _fields_ = [("r_min", C.c_double), ("i", C.c_int64), ("j", C.c_int64),
                ("r_second", C.c_double), ("i2", C.c_int64), ("j2", C.c_int64),
                ("r_max", C.c_double), ("n_pairs", C.c_int64),
                ("n_dropped", C.c_int64)]


def build(force: bool = True) -> Path:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp")
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                        "-fno-fast-math", "-std=c11", "-o", str(tmp), str(_SRC), "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
            build(force=True)
        lib = C.CDLL(str(_LIB))
        d, i32, i64, p = C.c_double, C.c_int32, C.c_int64, C.c_void_p
        lib.oracle_min_secant.argtypes = [p, i64, i32, p, i32, d, C.POINTER(_MinT)]
        lib.oracle_pair_r.argtypes = [p, i64, i32, p, i32, i64, i64,
                                      C.POINTER(d), C.POINTER(d)]
        lib.oracle_all_r.argtypes = [p, i64, i32, p, i32, d, p, p]
        lib.oracle_pairs_r.argtypes = [p, i64, i32, p, i32, p, i64, p]
        lib.oracle_step.argtypes = [p, i32, i32, p, d, i32, p, C.POINTER(i32)]
        lib.oracle_orth_error.argtypes = [p, i32, i32]
        lib.oracle_orth_error.restype = d
        lib.oracle_run.argtypes = [p, i64, i32, p, i32, d, d, i32, i32, p, p, p, p, p]
        lib.oracle_softmin.argtypes = [p, i64, i32, p, i32, d, d, C.POINTER(d), p,
                                       C.POINTER(d), C.POINTER(i64), C.POINTER(i64)]
        lib.oracle_secant_matrix.argtypes = [p, i64, i32, d, p, i64]
        lib.oracle_secant_matrix.restype = i64
        lib.oracle_unit_secant.argtypes = [p, i64, i32, i64, i64, p]
        lib.oracle_unit_secant.restype = d
        lib.oracle_pair_index.argtypes = [i64, i64, i64]
        lib.oracle_pair_index.restype = i64
        lib.oracle_num_threads.restype = C.c_int
        lib.oracle_set_threads.argtypes = [C.c_int]
        _lib = lib
    return _lib


def _X(X) -> np.ndarray:
    X = np.asarray(X)
    if X.ndim != 2:
        raise ValueError("X must be N x n")
    return np.ascontiguousarray(X, dtype=np.float64)


def _P(P) -> np.ndarray:
    P = np.asarray(P)
    if P.ndim != 2:
        raise ValueError("P must be n x k")
    return np.ascontiguousarray(P, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _check(st: int, what: str):
    if st != OK:
        raise OracleError(f"{what}: oracle status {st}")


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_threads(t: int) -> None:
    _load().oracle_set_threads(int(t))


def pair_index(N: int, i: int, j: int) -> int:
    return int(_load().oracle_pair_index(N, i, j))


def min_secant(X, P, min_len: float = 0.0) -> dict:
    X, P = _X(X), _P(P)
    out = _MinT()
    st = _load().oracle_min_secant(_ptr(X), X.shape[0], X.shape[1], _ptr(P),
                                   P.shape[1], float(min_len), C.byref(out))
    _check(st, "min_secant")
    return dict(r_min=out.r_min, i=out.i, j=out.j, r_second=out.r_second,
                i2=out.i2, j2=out.j2, r_max=out.r_max, n_pairs=out.n_pairs,
                n_dropped=out.n_dropped)


def pair_r(X, P, i: int, j: int) -> tuple[float, float]:
    X, P = _X(X), _P(P)
    r, d = C.c_double(), C.c_double()
    st = _load().oracle_pair_r(_ptr(X), X.shape[0], X.shape[1], _ptr(P), P.shape[1],
                               int(i), int(j), C.byref(r), C.byref(d))
    _check(st, "pair_r")
    return r.value, d.value


def pairs_r(X, P, ij) -> np.ndarray:
    """r of each pair in ij (count x 2 integer array)."""
    X, P = _X(X), _P(P)
    ij = np.ascontiguousarray(ij, dtype=np.int64).reshape(-1, 2)
    r = np.empty(ij.shape[0])
    st = _load().oracle_pairs_r(_ptr(X), X.shape[0], X.shape[1], _ptr(P), P.shape[1],
                                _ptr(ij), ij.shape[0], _ptr(r))
    _check(st, "pairs_r")
    return r


def all_r(X, P, min_len: float = 0.0) -> tuple[np.ndarray, np.ndarray]:
    X, P = _X(X), _P(P)
    N = X.shape[0]
    r = np.empty(N * (N - 1) // 2)
    d = np.empty_like(r)
    st = _load().oracle_all_r(_ptr(X), N, X.shape[1], _ptr(P), P.shape[1],
                              float(min_len), _ptr(r), _ptr(d))
    _check(st, "all_r")
    return r, d


def unit_secant(X, i: int, j: int) -> tuple[np.ndarray, float]:
    X = _X(X)
    s = np.empty(X.shape[1])
    d = _load().oracle_unit_secant(_ptr(X), X.shape[0], X.shape[1], int(i), int(j), _ptr(s))
    if d < 0:
        raise OracleError("unit_secant: bad pair")
    return s, d


def step(P, s, alpha: float = 0.01, rule: int = 0) -> tuple[np.ndarray, int]:
    P = _P(P)
    s = np.ascontiguousarray(s, dtype=np.float64)
    n, k = P.shape
    if s.shape != (n,):
        raise ValueError("s must have length n")
    out = np.empty_like(P)
    t = C.c_int32()
    st = _load().oracle_step(_ptr(P), n, k, _ptr(s), float(alpha), int(rule),
                             _ptr(out), C.byref(t))
    _check(st, "step")
    return out, int(t.value)


def orth_error(P) -> float:
    P = _P(P)
    return float(_load().oracle_orth_error(_ptr(P), P.shape[0], P.shape[1]))


def run(X, P0, iters: int, alpha: float = 0.01, min_len: float = 0.0,
        rule: int = 0) -> tuple[np.ndarray, dict]:
    X, P0 = _X(X), _P(P0)
    n, k = P0.shape
    Pout = np.empty_like(P0)
    m = iters + 1
    tmin, tsec, torth = np.empty(m), np.empty(m), np.empty(m)
    tij = np.empty(2 * m, dtype=np.int64)
    st = _load().oracle_run(_ptr(X), X.shape[0], n, _ptr(P0), k, float(alpha),
                            float(min_len), int(rule), int(iters), _ptr(Pout),
                            _ptr(tmin), _ptr(tij), _ptr(tsec), _ptr(torth))
    _check(st, "run")
    return Pout, dict(min=tmin, ij=tij.reshape(m, 2), second=tsec, orth=torth)


def softmin(X, P, tau: float, min_len: float = 0.0, grad: bool = True) -> dict:
    X, P = _X(X), _P(P)
    n, k = P.shape
    L = C.c_double()
    wsum = C.c_double()
    npairs, nzero = C.c_int64(), C.c_int64()
    G = np.zeros((n, k)) if grad else None
    st = _load().oracle_softmin(_ptr(X), X.shape[0], n, _ptr(P), k, float(tau),
                                float(min_len), C.byref(L),
                                _ptr(G) if grad else None, C.byref(wsum),
                                C.byref(npairs), C.byref(nzero))
    _check(st, "softmin")
    return dict(L=L.value, G=G, wsum=wsum.value, n_pairs=npairs.value,
                n_zero=nzero.value)


def secant_matrix(X, min_len: float = 0.0) -> np.ndarray:
    """S (n x |Pi|): the kept unit secants as columns, in pair-index order
    (Sec. 4, the secant matrix whose SVD initialises Algorithm 1)."""
    X = _X(X)
    N, n = X.shape
    cap = N * (N - 1) // 2
    S = np.empty((cap, n))
    q = _load().oracle_secant_matrix(_ptr(X), N, n, float(min_len), _ptr(S), cap)
    if q < 0:
        raise OracleError("secant_matrix: bad arguments")
    return np.ascontiguousarray(S[:q].T)


def pca_init(X, k: int, min_len: float = 0.0) -> tuple[np.ndarray, np.ndarray]:
    """Algorithm 1's initial projection (Sec. 4): the first k columns of U in
    S = U Sigma V^T, with S the explicit secant matrix.  Returns (P, sigma):
    P n x k with each column's largest-magnitude component positive (the
    first such component on ties), sigma the k largest singular values; the
    third value is every singular value.  The SVD is the library routine
    (numpy / LAPACK)."""
    S = secant_matrix(X, min_len)
    U, sv, _ = np.linalg.svd(S, full_matrices=False)
    P = U[:, :k].copy()
    for c in range(k):
        t = int(np.argmax(np.abs(P[:, c])))
        if P[t, c] < 0:
            P[:, c] = -P[:, c]
    return P, sv[:k].copy(), sv

