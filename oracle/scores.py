"""Score functions, t-sweep schedule and stopping tolerance for Robust-l0.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Scores (Table "scores", continuous column): q_z(r | t) = p_breve_z(r) and
q_e(r1 - r2 | t) = p_breve_e(r1 - r2), with p_breve from eq:breve applied to
eq:pz_approx / eq:pe_approx (module ``posterior``).

The decoder makes every decision in float32 (the paper fixes no precision; float32 is
the precision of the GPU kernels, so both sides decide in it).  A score is therefore a
float32 function, fixed here as a tabulation of the fp64 posterior:

  * range R: with h0 = sqrt(v0)/8 (v0 = sn^2 for z, 2 sn^2 for e), R = q h0 for the
    smallest integer q >= 8 with p_breve(q h0) < 2^-27;
  * nodes  : T[i] = fl32(p_breve(i R / N)), i = 0..N, N = 4096 (T[0] = 1 exactly);
  * lookup : for a >= 0, u = fl32(a * inv_h) with inv_h = fl32(N / R); if u >= N the
             score is 0; else i = floor(u), f = u - i and the score is
             T[i] + f * (T[i+1] - T[i]), every operation rounded to float32 in that
             order, no fused multiply-add.
The tabulated score differs from p_breve by less than 1e-6 (pinned in the tests).

With sigma_n = 0 the posteriors degenerate to indicators and the scores become the
Parallel-l0 column of the table: q_z(r) = 1{r = 0}, q_e(r1 - r2) = 1{r1 = r2}.

Schedule (Alg. 1 and Sec. 4 "Selection of parameter c"): t starts at 1 and drops by c
after each iteration while t > 0, so iteration it runs at t_it = 1 - it c (evaluated
afresh in fp64 each time, then rounded to float32) and there are ceil(1/c) iterations.
Stopping (Sec. 4 "Stopping conditions"): the decoder has converged once
||r||_1 <= E||eta||_1 = m sigma_n sqrt(2/pi).
"""
from __future__ import annotations

import math

import numpy as np

from . import posterior

__all__ = [
    "TABLE_N",
    "Table",
    "build_table",
    "lookup",
    "c_rule",
    "n_iters",
    "t_of",
    "tolerance",
    "eta_l1_mean",
    "eta_l1_var",
]

TABLE_N = 4096
CUTOFF = 2.0 ** -27


class Table:
    """A tabulated score: nodes T (float32, N+1 entries), inv_h (float32), range R."""

    def __init__(self, T: np.ndarray, inv_h: np.float32, R: float, exact: bool = False):
        self.T = T
        self.inv_h = inv_h
        self.R = R
        self.exact = exact


def _odds_coefficients(kind, d, rho, sigma_n, sigma_s, ell):
    terms = posterior.approx_terms(kind, d, rho, sigma_n, sigma_s, ell)
    v0 = terms[0][1]
    coeffs = []
    for weight, var in terms[1:]:
        C = weight * math.sqrt(v0 / var)
        a = 0.5 * (1.0 / v0 - 1.0 / var)
        coeffs.append((C, a))
    return v0, coeffs


def _odds(w: float, coeffs) -> float:
    w2 = w * w
    s = 0.0
    for C, a in coeffs:
        s += C * math.exp(a * w2)
    return s


def build_table(kind: str, d: int, rho: float, sigma_n: float, sigma_s: float = 1.0,
                ell: int = 4, N: int = TABLE_N) -> Table:
    """Tabulate p_breve_z (kind "z") or p_breve_e (kind "e") as described above."""
    if sigma_n == 0.0:
        return Table(np.zeros(N + 1, np.float32), np.float32(0.0), 0.0, exact=True)
    v0, coeffs = _odds_coefficients(kind, d, rho, sigma_n, sigma_s, ell)
    one_plus_S0 = 1.0 + _odds(0.0, coeffs)

    def pb(w):
        return one_plus_S0 / (1.0 + _odds(w, coeffs))

    h0 = math.sqrt(v0) / 8.0
    q = 8
    while pb(q * h0) >= CUTOFF:
        q += 1
    R = q * h0
    T = np.empty(N + 1, dtype=np.float32)
    for i in range(N + 1):
        T[i] = np.float32(pb(i * R / N))
    T[0] = np.float32(1.0)
    return Table(T, np.float32(N / R), R)


def lookup(table: Table, a: np.ndarray) -> np.ndarray:
    """Evaluate the tabulated score at a >= 0 (float32 in, float32 out)."""
    a = np.asarray(a, dtype=np.float32)
    if table.exact:
        return (a == np.float32(0.0)).astype(np.float32)
    N = table.T.size - 1
    u = (a * table.inv_h).astype(np.float32)
    inside = u < np.float32(N)
    uc = np.where(inside, u, np.float32(0.0)).astype(np.float32)
    i = uc.astype(np.int64)
    f = (uc - i.astype(np.float32)).astype(np.float32)
    Ti = table.T[i]
    Ti1 = table.T[np.minimum(i + 1, N)]
    val = (Ti + f * (Ti1 - Ti)).astype(np.float32)
    return np.where(inside, val, np.float32(0.0)).astype(np.float32)


def c_rule(delta: float, rho: float = 0.0, quantised: bool = False) -> float:
    """eq:finetune_c_cont (continuous) and eq:finetune_c_quant (quantised)."""
    if delta <= 0.05:
        return 0.01
    if not quantised:
        return 0.025
    if rho <= 0.1:
        return 0.05
    if rho <= 0.2:
        return 0.075
    return 0.1


def n_iters(c: float) -> int:
    """Number of t values 1, 1-c, 1-2c, ... that stay > 0."""
    return int(math.ceil(1.0 / c - 1e-9))


def t_of(it: int, c: float) -> np.float32:
    return np.float32(1.0 - it * c)


def eta_l1_mean(m: int, sigma: float) -> float:
    """E||eta||_1 = m sigma sqrt(2/pi) for eta ~ N(0, sigma^2 I) (Sec. 4)."""
    return m * sigma * math.sqrt(2.0 / math.pi)


def eta_l1_var(m: int, sigma: float) -> float:
    """Var||eta||_1 = m sigma^2 (1 - 2/pi) (Sec. 4)."""
    return m * sigma * sigma * (1.0 - 2.0 / math.pi)


def tolerance(m: int, sigma: float) -> float:
    """Stopping tolerance on ||r||_1 used by the phase-transition runs (Sec. 4)."""
    return eta_l1_mean(m, sigma)
