"""Posteriors and score tables for non-Gaussian signal and noise distributions.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Thm "Probabilities for general signal and noise distributions" (eq:pz_general,
eq:pe_general) gives, with lambda = d rho,

    p_z(w) = nu(w) / sum_{q >= 0} lambda^q / q! (nu * mu_q)(w),
    p_e(w) = nu~(w) / sum_{q >= 0} (2 lambda)^q / q! (nu~ * mu-bar_q)(w),

where mu_q is the q-fold convolution of mu (mu_0 the unit mass at 0, so the q = 0 term
is nu itself), nu~ = nu * nu^- is the law of the difference of two noise values and
mu-bar = (mu + mu^-) / 2 the symmetrised signal law (Definition "Measures").  This module
writes those sums out term by term in direct space: every convolution (nu * mu_q)(w) is
one adaptive quadrature (scipy.integrate.quad, breakpoints at the kinks of the densities)
of nu(w - x) mu_q(x), with mu_q in closed form, and the series runs until its terms no
longer change the sum in double precision.

Families (symmetric about 0, each given by its standard deviation s):
  gaussian  N(0, s^2); mu_q = N(0, q s^2); nu~ = N(0, 2 s^2);
  laplace   scale b = s / sqrt(2), density exp(-|x|/b) / (2b).  The sum of q independent
            such values has the density (a textbook result, the half-integer Bessel form
            of the variance-gamma law)
                f_q(x) = exp(-a) / (b 2^(2q-1) (q-1)!) sum_{j=0}^{q-1}
                         (2q-2-j)! / (j! (q-1-j)!) (2a)^j,     a = |x| / b,
            and nu~ = f_2.
Both families are symmetric, so mu-bar = mu and nu^- = nu.

Readings (the paper leaves them open):
  * the normalisation of eq:breve takes its maximum at w = 0, p_breve = p / p(0) (as R5
    for the Gaussian case); the tests check that p is non-increasing on the table range;
  * the tables follow scores.build_table: h0 = sqrt(v0)/8 with v0 the variance of nu (for
    z) or of nu~ = 2 Var(nu) (for e), R = q h0 for the smallest q >= 8 with
    p_breve(q h0) < 2^-27, T[i] = fl32(p_breve(i R / N)), T[0] = 1, inv_h = fl32(N / R);
  * the whole series is summed (no Gaussian tail approximation: that is eq:pz_approx's,
    for the Gaussian case only);
  * the stopping tolerance is m E|eta|: sigma sqrt(2/pi) for gaussian noise (Sec. 4), b for
    laplace noise.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate

from . import scores as _scores

__all__ = ["FAMILIES", "density", "sum_density", "diff_density", "posterior", "p_breve",
           "build_table", "noise_l1_mean"]

FAMILIES = ("gaussian", "laplace")
_SQRT2 = math.sqrt(2.0)


def _check(family: str) -> None:
    if family not in FAMILIES:
        raise ValueError(f"family must be one of {FAMILIES}")


def density(family: str, s: float, x: float) -> float:
    """The density of the family with standard deviation s at x."""
    _check(family)
    if family == "gaussian":
        return math.exp(-0.5 * (x / s) ** 2) / (s * math.sqrt(2.0 * math.pi))
    b = s / _SQRT2
    return math.exp(-abs(x) / b) / (2.0 * b)


def _laplace_sum_log_coeffs(q: int) -> list[float]:
    # log of (2q-2-j)! / (j! (q-1-j)! (q-1)! 2^(2q-1)), j = 0 .. q-1
    return [math.lgamma(2 * q - 1 - j) - math.lgamma(j + 1) - math.lgamma(q - j) - math.lgamma(q)
            - (2 * q - 1) * math.log(2.0) for j in range(q)]


def sum_density(family: str, s: float, q: int, x: float) -> float:
    """The density of the sum of q >= 1 independent values of the family at x."""
    _check(family)
    if q < 1:
        raise ValueError("q >= 1")
    if family == "gaussian":
        v = q * s * s
        return math.exp(-0.5 * x * x / v) / math.sqrt(2.0 * math.pi * v)
    b = s / _SQRT2
    a = abs(x) / b
    logc = _laplace_sum_log_coeffs(q)
    if a == 0.0:
        return math.exp(logc[0]) / b
    la = math.log(2.0 * a)
    return sum(math.exp(lc + j * la - a) for j, lc in enumerate(logc)) / b


def diff_density(family: str, s: float, x: float) -> float:
    """The density of the difference of two independent values of the family (nu~)."""
    if family == "gaussian":
        return density("gaussian", s * _SQRT2, x)
    return sum_density("laplace", s, 2, x)


def _conv(f, g, w: float, scale: float) -> float:
    """(f * g)(w) = int f(w - x) g(x) dx, f concentrated on a few multiples of `scale`
    around 0 (the noise), g wide (the signal sum); kinks at x = w and x = 0."""
    lo, hi = w - 60.0 * scale, w + 60.0 * scale
    pts = sorted({p for p in (0.0, w) if lo < p < hi})
    val, _ = integrate.quad(lambda x: f(w - x) * g(x), lo, hi, points=pts or None, limit=400,
                            epsabs=0.0, epsrel=1e-12)
    return val


def _denominator(kind: str, w: float, d: int, rho: float, mu: tuple, nu: tuple) -> tuple[float, float]:
    """(numerator, denominator) of eq:pz_general (kind "z") or eq:pe_general (kind "e")."""
    (fm, sm), (fn, sn) = mu, nu
    if kind == "z":
        lam = d * rho
        base = lambda x: density(fn, sn, x)  # noqa: E731
        scale = sn
    elif kind == "e":
        lam = 2.0 * d * rho
        base = lambda x: diff_density(fn, sn, x)  # noqa: E731
        scale = sn * _SQRT2
    else:
        raise ValueError("kind must be 'z' or 'e'")
    num = base(w)
    total = num
    weight = 1.0
    q = 0
    while True:
        q += 1
        weight *= lam / q
        peak = weight * sum_density(fm, sm, q, 0.0)      # the term's largest possible value
        if q > lam and peak < 1e-18 * total:
            break
        total += weight * _conv(base, lambda x, q=q: sum_density(fm, sm, q, x), w, scale)
        if q > 400:
            raise RuntimeError("series did not settle")
    return num, total


def posterior(kind: str, w: float, d: int, rho: float, mu: tuple, nu: tuple) -> float:
    """p_z(w) or p_e(w) of the theorem; mu, nu = (family, standard deviation)."""
    num, den = _denominator(kind, w, d, rho, mu, nu)
    return num / den


def p_breve(kind: str, w: float, d: int, rho: float, mu: tuple, nu: tuple, p0: float | None = None) -> float:
    """eq:breve with the maximum at 0: p(w) / p(0)."""
    if p0 is None:
        p0 = posterior(kind, 0.0, d, rho, mu, nu)
    return posterior(kind, w, d, rho, mu, nu) / p0


def build_table(kind: str, d: int, rho: float, mu: tuple, nu: tuple, N: int = _scores.TABLE_N,
                nodes=None) -> _scores.Table:
    """The score table of p_breve (module docstring).  With `nodes` (indices into 0..N)
    only those entries are evaluated; the others are left NaN (for spot checks)."""
    fn, sn = nu
    v0 = sn * sn * (1.0 if kind == "z" else 2.0)
    p0 = posterior(kind, 0.0, d, rho, mu, nu)
    pb = lambda w: posterior(kind, w, d, rho, mu, nu) / p0  # noqa: E731
    h0 = math.sqrt(v0) / 8.0
    q = 8
    while pb(q * h0) >= _scores.CUTOFF:
        q += 1
    R = q * h0
    T = np.full(N + 1, np.nan, dtype=np.float32)
    idx = range(N + 1) if nodes is None else nodes
    for i in idx:
        T[i] = np.float32(pb(i * R / N))
    T[0] = np.float32(1.0)
    return _scores.Table(T, np.float32(N / R), R)


def noise_l1_mean(m: int, nu: tuple) -> float:
    """E||eta||_1 = m E|eta_i|: the stopping tolerance (Sec. 4 for the Gaussian case)."""
    fn, sn = nu
    _check(fn)
    if fn == "gaussian":
        return m * sn * math.sqrt(2.0 / math.pi)
    return m * sn / _SQRT2
