"""Exact-rational brute force for tiny secant sets -- TEST INFRASTRUCTURE ONLY.

For rational points X and a projection P whose columns are rational and
orthonormal, r_ij^2 = ||P^T (x_i - x_j)||^2 / ||x_i - x_j||^2 is a rational
number, so the minimum of the projected unit-secant norm (paper Sec. 4, the
objective; Algorithm 1, the argmin step) and its lexicographic (r, i, j)
argmin can be found with no rounding at all.  This pins the tie-break of the
FP64 oracle on constructed exact ties.  Pure Python; keep N <= 10.
"""
from __future__ import annotations

from fractions import Fraction
from typing import Sequence


def _f(v) -> Fraction:
    return v if isinstance(v, Fraction) else Fraction(v)


def r2_exact(X: Sequence[Sequence], P: Sequence[Sequence], i: int, j: int,
             min_len2: Fraction = Fraction(0)):
    """Exact r^2 of pair (i, j), or None if the pair is dropped
    (duplicate, or squared length below min_len^2)."""
    n = len(X[0])
    k = len(P[0])
    diff = [_f(X[i][l]) - _f(X[j][l]) for l in range(n)]
    d2 = sum(t * t for t in diff)
    if d2 == 0 or d2 < min_len2:
        return None
    c = [sum(_f(P[l][q]) * diff[l] for l in range(n)) for q in range(k)]
    return sum(t * t for t in c) / d2


def min_exact(X, P, min_len2: Fraction = Fraction(0)):
    """(r2_min, i, j, sorted list of (r2, i, j)) over all kept pairs."""
    N = len(X)
    allv = []
    for i in range(N):
        for j in range(i + 1, N):
            v = r2_exact(X, P, i, j, min_len2)
            if v is not None:
                allv.append((v, i, j))
    if not allv:
        raise ValueError("no pairs")
    allv.sort()
    v, i, j = allv[0]
    return v, i, j, allv


def is_orthonormal_exact(P) -> bool:
    n, k = len(P), len(P[0])
    for a in range(k):
        for b in range(k):
            s = sum(_f(P[l][a]) * _f(P[l][b]) for l in range(n))
            if s != (1 if a == b else 0):
                return False
    return True
