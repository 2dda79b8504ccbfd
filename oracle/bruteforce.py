"""Exhaustive l0 minimisation for tiny problems.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The problem statement of Sec. 1: min ||x||_0 subject to A x = y.  For n <= 16 every
support of size s = 0, 1, 2, ... is tried in turn; a support S is feasible when the
least-squares solution of A_S x_S = y leaves a residual below ``atol``.  The first size
with a feasible support is the l0 minimum; the function returns every minimiser of
that size so the caller can check uniqueness.
"""
from __future__ import annotations

import itertools

import numpy as np

__all__ = ["dense_matrix", "l0_minimisers"]


def dense_matrix(A_cols: np.ndarray, m: int) -> np.ndarray:
    n, d = A_cols.shape
    A = np.zeros((m, n), dtype=np.float64)
    for j in range(n):
        A[A_cols[j], j] = 1.0
    return A


def l0_minimisers(A: np.ndarray, y: np.ndarray, max_support: int, atol: float = 1e-9):
    m, n = A.shape
    if n > 16:
        raise ValueError("brute force is for n <= 16")
    y = np.asarray(y, dtype=np.float64)
    if np.linalg.norm(y) <= atol:
        return 0, [np.zeros(n)]
    for s in range(1, max_support + 1):
        sols = []
        for S in itertools.combinations(range(n), s):
            AS = A[:, S]
            xs, *_ = np.linalg.lstsq(AS, y, rcond=None)
            if np.linalg.norm(AS @ xs - y) <= atol and np.all(np.abs(xs) > atol):
                x = np.zeros(n)
                x[list(S)] = xs
                sols.append(x)
        if sols:
            return s, sols
    return None, []
