"""The phase-transition harness (Sec. 4): the success condition eq:success_condition_clip
worked by hand, the logistic fit against curves with a known 50% point, and the ladder's
stopping rule with a stand-in decoder (all on the CPU); on the GPU a ladder of real
decodes."""
import math

import numpy as np
import pytest

from paper_1704_09012_amd import phase as PH


def test_success_condition_by_hand():
    # m = 100, sigma = 0.01: E||eta||_1 = 100 * 0.01 * sqrt(2/pi) = 0.797885,
    # sqrt(Var) = sqrt(100 * 1e-4 * (1 - 2/pi)) = 0.060281; sum 0.858166
    x = np.zeros(50)
    x[:10] = 1.0                       # ||x||_1 = 10: bound 0.0858166 (below the clip 0.1)
    xh = x.copy()
    xh[0] = 1.0 - 0.858                # error 0.858 -> ratio 0.0858 <= 0.0858166
    assert PH.success(x, xh, 100, 0.01)
    xh[0] = 1.0 - 0.8582               # ratio 0.08582 > bound
    assert not PH.success(x, xh, 100, 0.01)
    # ||x||_1 = 5: the bound 0.17163 is clipped at 1/10
    y = np.zeros(50)
    y[:5] = 1.0
    yh = y.copy()
    yh[0] = 1.0 - 0.499
    assert PH.success(y, yh, 100, 0.01)
    yh[0] = 1.0 - 0.501
    assert not PH.success(y, yh, 100, 0.01)
    assert PH.success(np.zeros(4), np.zeros(4), 100, 0.01)


@pytest.mark.parametrize("rho50,b", [(0.2, 60.0), (0.31, 25.0), (0.08, 150.0)])
def test_logistic_fit_recovers_a_known_curve(rho50, b):
    rhos = np.round(np.arange(0.01, 0.6, 0.01), 2)
    trials = np.full(rhos.size, 4000)
    p = 1.0 / (1.0 + np.exp(b * (rhos - rho50)))
    rng = np.random.default_rng(3)
    succ = rng.binomial(trials, p)
    r, bb = PH.logistic_fit(rhos, succ, trials)
    assert abs(r - rho50) < 2e-3 and abs(bb - b) / b < 0.1


def test_logistic_fit_on_a_step_and_on_no_transition():
    rhos = [0.01, 0.02, 0.03, 0.04]
    r, b = PH.logistic_fit(rhos, [10, 10, 0, 0], [10, 10, 10, 10])
    assert 0.02 < r < 0.03 and b > 100
    assert PH.logistic_fit(rhos, [10] * 4, [10] * 4) == (0.04, math.inf)
    assert PH.logistic_fit(rhos, [0] * 4, [10] * 4) == (0.01, math.inf)


def test_ladder_stops_after_the_first_level_with_no_recovery():
    calls = []

    def fake(n, m, k, sigma, variant, trials, seed):
        rho = k / m
        calls.append(rho)
        ok = int(round(trials * max(0.0, min(1.0, (0.25 - rho) / 0.1 + 0.5))))
        return [(i < ok, 1.0) for i in range(trials)]

    res = PH.ladder(fake, n=100000, delta=0.01, sigma=0.001, trials=10)
    assert res.succ[-1] == 0 and all(s > 0 for s in res.succ[:-1])
    assert res.rhos[0] == 0.01 and np.allclose(np.diff(res.rhos), 0.01)
    assert abs(res.rho50 - 0.25) < 0.01
    assert res.rho_half == pytest.approx(0.25, abs=0.011)
    assert len(calls) == len(res.rhos)


@pytest.mark.gpu
def test_ladder_of_gpu_decodes():
    """n = 2^14, delta = 0.2, sigma = 1e-3, Robust-l0 and the quantised variant: the ladder
    ends, recovery is certain at rho = 0.01 and the fitted rho* lies where the paper finds
    the Robust-l0 transitions, below about 0.3 (Sec. 4)."""
    pytest.importorskip("torch")
    for variant in (0, 1):
        res = PH.ladder(PH.gpu_trials, n=2 ** 14, delta=0.2, sigma=1e-3, variant=variant, trials=10, seed=5)
        print(variant, res.as_dict(), flush=True)
        assert res.succ[0] == 10 and res.succ[-1] == 0
        assert 0.08 < res.rho50 < 0.4
