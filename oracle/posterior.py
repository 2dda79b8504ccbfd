"""Posteriors p_z and p_e for centred Gaussian signal and noise, in fp64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Notation (Sec. 3 of the paper): rho = k/m, sigma_n the noise std, sigma_s the signal
std, phi(w | v) the centred Gaussian density of variance v.

* Full series (Sec. 3, "Explicit formulas for the centred Gaussian case",
  eq:pz_gaussian and eq:pe_gaussian):
      p_z(w) = phi(w | sn^2)   / sum_{q>=0} (d rho)^q/q!  phi(w | q ss^2 + sn^2)
      p_e(w) = phi(w | 2 sn^2) / sum_{q>=0} (2d rho)^q/q! phi(w | q ss^2 + 2 sn^2)
* Truncated series with a moment-matched Gaussian tail (Sec. 3, "Estimating the tails
  in the Gaussian case", eq:pz_approx and eq:pe_approx): the terms q = 0..ell are kept
  and the remainder sum_{q>ell} is replaced by R(ell) * phi(w | sigma_T^2) where
      R(ell)     = sum_{q>ell} lam^q / q!           (= e^lam - sum_{q<=ell} lam^q/q!)
      sigma_T^2  = (ss^2 lam R(ell-1) + v0 R(ell)) / R(ell)
  which is the variance of the normalised tail mixture (Lemma "Sums of centred density
  functions").  For p_z: lam = d rho, v0 = sn^2; for p_e: lam = 2 d rho, v0 = 2 sn^2.
* Normalisation (eq:breve): p_breve(w) = p(w) / max_s p(s).  Every term of the odds
  S(w) = sum_{q>=1} (weight_q / 1) phi(w|v_q)/phi(w|v0) grows with |w| because
  v_q > v0, so p = 1/(1+S) peaks at w = 0 and p_breve(w) = (1+S(0)) / (1+S(w)).

Readings of garbled passages (each listed in the design notes):
  - the variance of term q is q ss^2 + sn^2 (the printed "q ss^2 + sn" lacks a square);
  - the tail-variance sum runs over q = ell+1 .. infinity (printed upper limit ell);
  - for p_e the terms use q ss^2 + 2 sn^2 and R_e uses (2 d rho)^q, as in eq:pe_gaussian
    (the printed R_e and sigma_{q,e} reuse the z-form).
R(ell) is summed directly rather than as e^lam minus the partial sum: the two are the
same number, and the direct sum avoids cancellation when lam is small.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "rates",
    "series_terms",
    "tail_remainder",
    "approx_terms",
    "log_odds_terms",
    "p_full",
    "p_approx",
    "p_breve",
    "p_breve_full",
    "gaussian_pdf",
]


def gaussian_pdf(w, var):
    w = np.asarray(w, dtype=np.float64)
    return np.exp(-0.5 * w * w / var) / math.sqrt(2.0 * math.pi * var)


def rates(kind: str, d: int, rho: float, sigma_n: float):
    """(lam, v0) of the Poisson mixture: Thm. "Distribution of y_hat_i and ..."."""
    if kind == "z":
        return d * rho, sigma_n * sigma_n
    if kind == "e":
        return 2.0 * d * rho, 2.0 * sigma_n * sigma_n
    raise ValueError(kind)


def _poisson_weight(lam: float, q: int) -> float:
    # lam^q / q!
    return math.exp(q * math.log(lam) - math.lgamma(q + 1)) if lam > 0 else (1.0 if q == 0 else 0.0)


def tail_remainder(lam: float, ell: int) -> float:
    """R(ell) = sum_{q > ell} lam^q / q!, summed term by term until negligible."""
    if ell < -1:
        raise ValueError("ell >= -1")
    total = 0.0
    q = ell + 1
    term = _poisson_weight(lam, q)
    while True:
        total += term
        q += 1
        term = term * lam / q
        if term <= total * 1e-18 or q > ell + 400:
            break
    return total


def series_terms(kind: str, d: int, rho: float, sigma_n: float, sigma_s: float, qmax: int):
    """[(weight_q, var_q)] for q = 0..qmax of the full series (eq:pz_gaussian/eq:pe_gaussian)."""
    lam, v0 = rates(kind, d, rho, sigma_n)
    return [(_poisson_weight(lam, q), q * sigma_s * sigma_s + v0) for q in range(qmax + 1)]


def approx_terms(kind: str, d: int, rho: float, sigma_n: float, sigma_s: float, ell: int):
    """[(weight, var)] of eq:pz_approx / eq:pe_approx: q = 0..ell, then the Gaussian tail."""
    if ell < 1:
        raise ValueError("ell >= 1")
    lam, v0 = rates(kind, d, rho, sigma_n)
    terms = [(_poisson_weight(lam, q), q * sigma_s * sigma_s + v0) for q in range(ell + 1)]
    R_ell = tail_remainder(lam, ell)
    R_prev = tail_remainder(lam, ell - 1)
    if R_ell > 0.0:
        var_T = (sigma_s * sigma_s * lam * R_prev + v0 * R_ell) / R_ell
        terms.append((R_ell, var_T))
    return terms


def log_odds_terms(terms, v0: float):
    """Per term q >= 1: (log C_q, a_q) with phi(w|v_q)/phi(w|v0) * weight = C_q exp(a_q w^2).

    The q = 0 term has var v0 and weight 1; it is the numerator itself, so p = 1/(1+S)."""
    out = []
    for weight, var in terms[1:]:
        if weight <= 0.0:
            continue
        logC = math.log(weight) + 0.5 * math.log(v0 / var)
        a = 0.5 * (1.0 / v0 - 1.0 / var)
        out.append((logC, a))
    return out


def _log1p_odds(w, lt):
    """log(1 + S(w)) with S(w) = sum exp(logC + a w^2), by log-sum-exp."""
    w = np.asarray(w, dtype=np.float64)
    w2 = w * w
    expo = np.stack([np.zeros_like(w2)] + [logC + a * w2 for logC, a in lt])
    mx = expo.max(axis=0)
    return mx + np.log(np.exp(expo - mx).sum(axis=0))


def _terms(kind, d, rho, sigma_n, sigma_s, ell, qmax):
    if ell is None:
        return series_terms(kind, d, rho, sigma_n, sigma_s, qmax)
    return approx_terms(kind, d, rho, sigma_n, sigma_s, ell)


def p_full(kind, w, d, rho, sigma_n, sigma_s=1.0, qmax=200):
    """p_z or p_e from the full series, by direct density ratio (small |w| only)."""
    terms = series_terms(kind, d, rho, sigma_n, sigma_s, qmax)
    num = gaussian_pdf(w, terms[0][1])
    den = sum(wt * gaussian_pdf(w, var) for wt, var in terms)
    return num / den


def p_approx(kind, w, d, rho, sigma_n, sigma_s=1.0, ell=4):
    """eq:pz_approx / eq:pe_approx as 1/(1+S(w)), evaluated in the log domain."""
    terms = approx_terms(kind, d, rho, sigma_n, sigma_s, ell)
    lt = log_odds_terms(terms, terms[0][1])
    return np.exp(-_log1p_odds(w, lt))


def p_breve(kind, w, d, rho, sigma_n, sigma_s=1.0, ell=4):
    """eq:breve applied to eq:pz_approx / eq:pe_approx: (1+S(0))/(1+S(w))."""
    terms = approx_terms(kind, d, rho, sigma_n, sigma_s, ell)
    lt = log_odds_terms(terms, terms[0][1])
    return np.exp(_log1p_odds(0.0, lt) - _log1p_odds(w, lt))


def p_breve_full(kind, w, d, rho, sigma_n, sigma_s=1.0, qmax=120):
    """eq:breve applied to the full series eq:pz_gaussian / eq:pe_gaussian."""
    terms = series_terms(kind, d, rho, sigma_n, sigma_s, qmax)
    lt = log_odds_terms(terms, terms[0][1])
    return np.exp(_log1p_odds(0.0, lt) - _log1p_odds(w, lt))
