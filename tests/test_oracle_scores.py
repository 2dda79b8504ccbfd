"""Pins for the oracle's tabulated scores and schedule (Table "scores", Sec. 4)."""
import math

import numpy as np
import pytest

from oracle import posterior as P
from oracle import scores as S

CASES = [
    (7, 25 / 256, 0.00826797),
    (7, 10485 / 104857, 0.0836632),
    (7, 10485 / 104857, 0.00836632),
    (7, 10485 / 104857, 0.000836632),
    (8, 1 / 8, 0.01),
]


@pytest.mark.parametrize("kind", ["z", "e"])
@pytest.mark.parametrize("d,rho,sig", CASES)
def test_table_nodes_are_rounded_posterior(kind, d, rho, sig):
    tab = S.build_table(kind, d, rho, sig)
    N = tab.T.size - 1
    nodes = np.arange(N + 1) * tab.R / N
    ref = P.p_breve(kind, nodes, d, rho, sig)       # log-domain evaluation, a different route
    assert tab.T[0] == np.float32(1.0)
    assert np.all(np.abs(tab.T.astype(np.float64) - ref) <= 2.0 ** -24 * np.maximum(ref, 2.0 ** -30) + 1e-15)
    assert np.all(np.diff(tab.T) <= 0)
    # the range ends where the posterior is negligible
    assert P.p_breve(kind, tab.R, d, rho, sig) < 2.0 ** -27
    assert P.p_breve(kind, tab.R - math.sqrt(P.rates(kind, d, rho, sig)[1]) / 8, d, rho, sig) >= 2.0 ** -27


@pytest.mark.parametrize("kind", ["z", "e"])
@pytest.mark.parametrize("d,rho,sig", CASES)
def test_lookup_error_bound(kind, d, rho, sig):
    tab = S.build_table(kind, d, rho, sig)
    rng = np.random.Generator(np.random.PCG64(1))
    a = (rng.random(200000) * 1.2 * tab.R).astype(np.float32)
    got = S.lookup(tab, a).astype(np.float64)
    ref = P.p_breve(kind, a.astype(np.float64), d, rho, sig)
    assert np.max(np.abs(got - ref)) < 1e-6


@pytest.mark.parametrize("kind", ["z", "e"])
def test_lookup_monotone_on_dense_float_grid(kind):
    d, rho, sig = CASES[2]
    tab = S.build_table(kind, d, rho, sig)
    lo = np.float32(0.0).view(np.uint32)
    hi = np.float32(tab.R * 1.01).view(np.uint32)
    # every float32 in [R/4, 1.01 R] and a stride through [0, R/4]
    a1 = np.arange(np.float32(tab.R / 4).view(np.uint32), hi, dtype=np.uint32).view(np.float32)
    a0 = np.arange(lo, np.float32(tab.R / 4).view(np.uint32), 97, dtype=np.uint32).view(np.float32)
    a = np.concatenate([a0, a1])
    v = S.lookup(tab, a)
    assert np.all(np.diff(v) <= 0)
    assert v[0] == np.float32(1.0)
    assert S.lookup(tab, np.float32(tab.R * 1.001)) == 0.0


def test_exact_mode_is_parallel_l0_indicator():
    tab = S.build_table("z", 7, 0.1, 0.0)
    assert tab.exact
    a = np.array([0.0, 1e-30, 1.0], dtype=np.float32)
    assert list(S.lookup(tab, a)) == [1.0, 0.0, 0.0]


def test_c_rule_and_schedule():
    # eq:finetune_c_cont
    assert S.c_rule(0.05) == 0.01 and S.c_rule(0.1) == 0.025 and S.c_rule(0.0999) == 0.025
    # eq:finetune_c_quant
    assert S.c_rule(0.1, 0.05, True) == 0.05
    assert S.c_rule(0.1, 0.15, True) == 0.075
    assert S.c_rule(0.1, 0.25, True) == 0.1
    assert S.c_rule(0.01, 0.25, True) == 0.01
    assert S.n_iters(0.025) == 40 and S.n_iters(0.01) == 100 and S.n_iters(0.03) == 34
    ts = [float(S.t_of(i, 0.025)) for i in range(40)]
    assert ts[0] == 1.0 and all(a > b for a, b in zip(ts, ts[1:])) and ts[-1] > 0
    assert float(S.t_of(40, 0.025)) <= 1e-9
