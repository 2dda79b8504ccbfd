"""Pins for the oracle's posteriors under non-Gaussian signal and noise laws (Thm
"Probabilities for general signal and noise distributions"): the Gaussian case against the
closed-form Gaussian series, the Laplace q-fold densities against direct convolution and
their moments, the small-rate limit against the closed-form convolution of two Laplace
laws, and both posteriors against a Monte Carlo of the generating model itself."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import decoder as D
from oracle import general as G
from oracle import scores as S


def gaussian_series(kind, w, d, rho, ss, sn):
    lam, v0 = (d * rho, sn * sn) if kind == "z" else (2 * d * rho, 2 * sn * sn)
    num = math.exp(-w * w / (2 * v0)) / math.sqrt(2 * math.pi * v0)
    den, wt = 0.0, 1.0
    for q in range(300):
        if q:
            wt *= lam / q
        v = v0 + q * ss * ss
        den += wt * math.exp(-w * w / (2 * v)) / math.sqrt(2 * math.pi * v)
    return num / den


@pytest.mark.parametrize("kind", ["z", "e"])
@pytest.mark.parametrize("d,rho,ss,sn", [(7, 0.1, 1.0, 0.01), (3, 0.3, 2.0, 0.05), (12, 0.02, 1.0, 0.001)])
def test_gaussian_laws_give_the_closed_form_series(kind, d, rho, ss, sn):
    # the q-fold convolutions of N(0, ss^2) are N(0, q ss^2) and nu * N(0, v) = N(0, v + sn^2)
    for w in (0.0, 0.7 * sn, 2.5 * sn, 5.0 * sn):
        a = G.posterior(kind, w, d, rho, ("gaussian", ss), ("gaussian", sn))
        b = gaussian_series(kind, w, d, rho, ss, sn)
        assert abs(a - b) <= 1e-10 * b


@pytest.mark.parametrize("q", [1, 2, 3, 4, 7])
def test_laplace_sum_density_moments_and_convolution(q):
    s = 1.3
    mass = integrate.quad(lambda x: G.sum_density("laplace", s, q, x), -np.inf, np.inf, points=None)[0]
    var = 2.0 * integrate.quad(lambda x: x * x * G.sum_density("laplace", s, q, x), 0, np.inf)[0]
    assert abs(mass - 1.0) < 1e-9 and abs(var - q * s * s) < 1e-8 * q * s * s
    if q > 1:
        for x in (0.0, 0.4, 2.0, 5.0):
            conv = integrate.quad(lambda t: G.sum_density("laplace", s, q - 1, x - t) * G.density("laplace", s, t),
                                  -60, 60, points=[0.0, x], limit=400, epsabs=0.0, epsrel=1e-12)[0]
            assert abs(conv - G.sum_density("laplace", s, q, x)) <= 1e-9 * conv
    one, ref = G.sum_density("laplace", s, 1, 0.37), G.density("laplace", s, 0.37)
    assert abs(one - ref) <= 1e-14 * ref


@pytest.mark.parametrize("family", ["gaussian", "laplace"])
def test_difference_law_is_the_self_convolution(family):
    s = 0.2
    for x in (0.0, 0.1, 0.5):
        conv = integrate.quad(lambda t: G.density(family, s, x + t) * G.density(family, s, t), -20, 20,
                              points=[0.0, -x], limit=400, epsabs=0.0, epsrel=1e-12)[0]
        assert abs(conv - G.diff_density(family, s, x)) <= 1e-9 * conv


def test_small_rate_limit_is_one_laplace_convolution():
    # D(w) = nu(w) + lam (nu * mu)(w) + O(lam^2), and for two Laplace laws with scales bs, bn
    # (nu * mu)(x) = (bs exp(-|x|/bs) - bn exp(-|x|/bn)) / (2 (bs^2 - bn^2))
    ss, sn, d = 1.0, 0.05, 7
    bs, bn = ss / math.sqrt(2), sn / math.sqrt(2)
    rho = 1e-7
    lam = d * rho
    for w in (0.0, 0.03, 0.2):
        num, den = G._denominator("z", w, d, rho, ("laplace", ss), ("laplace", sn))
        closed = (bs * math.exp(-w / bs) - bn * math.exp(-w / bn)) / (2 * (bs * bs - bn * bn))
        assert num == G.density("laplace", sn, w)
        assert abs((den - num) / lam - closed) <= 1e-5 * closed


def _mc_rows(rng, count, lam, mu, nu):
    """Row values of the generating model: a Poisson(lam) number of signal values plus noise."""
    q = rng.poisson(lam, size=count)
    fam_m, sm = mu
    total = q.sum()
    draws = rng.laplace(0.0, sm / math.sqrt(2), size=total) if fam_m == "laplace" else rng.normal(0.0, sm, total)
    row = np.zeros(count)
    np.add.at(row, np.repeat(np.arange(count), q), draws)
    fam_n, sn = nu
    row += rng.laplace(0.0, sn / math.sqrt(2), size=count) if fam_n == "laplace" else rng.normal(0.0, sn, count)
    return q, row


@pytest.mark.parametrize("mu,nu", [(("laplace", 1.0), ("laplace", 0.25)), (("laplace", 1.0), ("gaussian", 0.25)),
                                   (("gaussian", 1.0), ("laplace", 0.25))])
def test_posteriors_match_a_monte_carlo_of_the_model(mu, nu):
    """p_z(w) = P(a row holds no signal | its value is w), with a Poisson(d rho) number of
    signal values per row (the limit of the theorem); p_e(w) = P(neither of two rows holds
    signal | their difference is w).  Each estimate is a bin of half-width 0.01 around w."""
    rng = np.random.Generator(np.random.PCG64(2024))
    d, rho = 7, 0.1
    lam = d * rho
    count = 4_000_000
    q1, r1 = _mc_rows(rng, count, lam, mu, nu)
    q2, r2 = _mc_rows(rng, count, lam, mu, nu)
    for kind, zero, val in (("z", q1 == 0, r1), ("e", (q1 == 0) & (q2 == 0), r1 - r2)):
        for w in (0.0, 0.15, 0.35, 0.6):
            sel = np.abs(np.abs(val) - w) < 0.01
            n = int(sel.sum())
            est = float(zero[sel].mean())
            p = G.posterior(kind, w, d, rho, mu, nu)
            se = math.sqrt(max(p * (1 - p), 1e-4) / n)
            assert n > 2000 and abs(est - p) < 5 * se + 0.01, (kind, w, est, p, n)


def test_noise_l1_mean_matches_the_law():
    rng = np.random.Generator(np.random.PCG64(3))
    for fam in ("gaussian", "laplace"):
        s = 0.3
        x = rng.laplace(0, s / math.sqrt(2), 2_000_000) if fam == "laplace" else rng.normal(0, s, 2_000_000)
        assert abs(G.noise_l1_mean(1, (fam, s)) - np.abs(x).mean()) < 2e-3 * s
    assert G.noise_l1_mean(1000, ("gaussian", 0.01)) == S.tolerance(1000, 0.01)


def test_table_follows_the_score_table_rules():
    mu, nu = ("laplace", 1.0), ("laplace", 0.01)
    nodes = list(range(0, 4097, 256)) + [4096]
    for kind in ("z", "e"):
        T = G.build_table(kind, 7, 0.1, mu, nu, nodes=nodes)
        v0 = 0.01 ** 2 * (1 if kind == "z" else 2)
        h0 = math.sqrt(v0) / 8
        p0 = G.posterior(kind, 0.0, 7, 0.1, mu, nu)
        assert T.T[0] == 1.0 and T.inv_h == np.float32(4096 / T.R)
        q = round(T.R / h0)
        assert abs(q * h0 - T.R) < 1e-15 and q >= 8
        assert G.posterior(kind, T.R, 7, 0.1, mu, nu) / p0 < S.CUTOFF
        assert G.posterior(kind, T.R - h0, 7, 0.1, mu, nu) / p0 >= S.CUTOFF or q == 8
        vals = T.T[nodes]
        assert np.all(np.diff(vals) <= 0)           # non-increasing: the maximum is at 0
        assert vals[-1] < 2 ** -27


def test_constants_take_general_laws_and_given_tables():
    n, m, d, k = 4096, 1024, 7, 80
    Tz = S.Table(np.linspace(1, 0, 4097).astype(np.float32), np.float32(4096 / 0.1), 0.1)
    Te = S.Table(np.linspace(1, 0, 4097).astype(np.float32) ** 2, np.float32(4096 / 0.2), 0.2)
    C = D.make_constants(n, m, d, k, 0.01, noise="laplace", tables=(Tz, Te))
    assert C.Tz is Tz and C.Te is Te and C.noise == "laplace"
    assert C.tol == G.noise_l1_mean(m, ("laplace", 0.01))
    with pytest.raises(ValueError):
        D.make_constants(n, m, d, k, 0.01, signal="cauchy")
    with pytest.raises(ValueError):
        D.make_constants(n, m, d, k, 0.01, noise="laplace", adaptive_k=1)
