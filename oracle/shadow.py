"""fp64 shadow of the column test.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Alg. 1's column body evaluated in float64, with the posterior scores p_breve of
eq:breve computed from their series (log-sum-exp in oracle.posterior) instead of the
float32 tables of the contract path.  It returns each decision together with its
margin, the distance of every comparison the decision depends on from its threshold:
the outer test 1 - p_breve_z(r_i) >= t, the consensus test n_e - n_z >= alpha and the
l1 test.  A contract (float32, tabulated) decision that differs from the shadow's where
the margin exceeds the float32/table resolution is a mistake; where the margin is
smaller, the two may differ by rounding.

Readings (R7, R8, R9): one update per column, the passing row with the largest n_e
(ties to the smaller row); the l1 test is taken on the column's own rows; N(j) includes
the row itself.
"""
from __future__ import annotations

import math

from oracle import posterior as P


def column(v, t: float, alpha: float, d: int, rho: float, sigma: float, split: bool = False,
           quantised: bool = False):
    """One column with residual entries v (its d rows, ascending).  Returns
    (candidates, margin): candidates are the passing rows as (n_e, omega, row), margin
    the smallest distance of any comparison from its threshold (relative for the l1
    test).  With split, (candidates, outer margin, margin of the other tests).  With
    quantised the weights are the indicators 1{p_breve_z >= 1 - t} and 1{p_breve_e >= t}
    (Table "scores", middle column), whose distances from their levels count as margins."""
    pz = [float(P.p_breve("z", vi, d, rho, sigma)) for vi in v]
    other_m = math.inf
    if quantised:
        other_m = min(abs(p - (1.0 - t)) for p in pz)
        qz = [1.0 if p >= 1.0 - t else 0.0 for p in pz]
    else:
        qz = pz
    n_z = sum(qz)
    S1 = sum(abs(vi) for vi in v)
    cands = []
    outer_m = math.inf
    for i in range(d):
        outer = 1.0 - pz[i] - t
        outer_m = min(outer_m, abs(outer))
        if outer < 0:
            continue
        pe = [1.0 if l == i else float(P.p_breve("e", v[i] - v[l], d, rho, sigma)) for l in range(d)]
        if quantised:
            other_m = min([other_m] + [abs(pe[l] - t) for l in range(d) if l != i])
            qe = [1.0 if p >= t else 0.0 for p in pe]
        else:
            qe = pe
        n_e = sum(qe)
        omega = sum(v[l] * qe[l] for l in range(d)) / n_e
        L = sum(abs(v[l] - omega) for l in range(d))
        # quantised counts are exact integers in float32 too: their comparison has no margin
        other_m = min(other_m, math.inf if quantised else abs(n_e - n_z - alpha), abs(L - S1) / max(S1, 1e-30))
        if L <= S1 and n_e - n_z >= alpha:
            cands.append((n_e, omega, i))
    if split:
        return cands, outer_m, other_m
    return cands, min(outer_m, other_m)


def decision(v, t: float, alpha: float, d: int, rho: float, sigma: float, split: bool = False,
             quantised: bool = False):
    """(updated, row, omega, margin) of one column: the passing row with the largest
    n_e, ties to the smaller row.  With split the margin is two values, of the outer test
    and of the other tests."""
    cands, *margins = column(v, t, alpha, d, rho, sigma, split, quantised)
    if not cands:
        return (False, -1, 0.0, *margins)
    n_e, omega, row = max(cands, key=lambda c: (c[0], -c[2]))
    return (True, row, omega, *margins)
