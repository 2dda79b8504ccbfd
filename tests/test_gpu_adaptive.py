"""Alg. 1's adaptive_k branch on the GPU (params.adaptive_k = 1) against the oracle, through
the C-ABI.

After every accepted iteration the posteriors' sparsity becomes k_0 = max(k - sum_j
(1 - p_breve_z(|x_hat_j|)), floor(m/100), 1) and the score tables, the outer-test
thresholds and (quantised) the indicator thresholds are rebuilt with rho = k_0/m.  Bar:
bitwise, as for the fixed-k decoder: x_hat, the loop statistics, the fixed-point counts
and the last k_0.  Whole decodes at 1024 x 256 (both score variants, 10 seeds each), at
ragged mid sizes (the bitmask in LDS; for m above 393216 its summary, the dense
sweep and H_k's classification kernel), and n = 2^20 decodes against stored oracle
decodes (tests/golden/decodea_*)."""
import os

import numpy as np
import pytest

from oracle import decoder as D
from paper_1704_09012_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_1704_09012_amd.rl0")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def problem(n, m, k, d, snr, seed):
    sig = float(np.float32(I.sigma_for_snr(snr, n, m, k, d)))
    inst = I.draw_instance(n, m, k, d, sig, seed)
    y = D.measure(inst.A_cols[inst.support], inst.values, inst.eta, m)
    return inst, y, sig


def assert_same_decode(xg, stg, res):
    assert np.array_equal(xg, res.x_hat)
    assert stg["iterations"] == res.iterations
    assert stg["accepted"] == res.accepted
    assert stg["l1_final_fx"] == res.L_hat
    assert stg["converged"] == int(res.converged)
    assert stg["updates_total"] == res.updates_total
    assert stg["fx_inexact_y"] == res.fx_inexact_y
    assert stg["fx_inexact_x"] == res.fx_inexact_x
    assert stg["k_post"] == res.k_post


def run_both(n, m, k, d, snr, seed, variant):
    inst, y, sig = problem(n, m, k, d, snr, seed)
    xg, stg = R.decode(dev(inst.A_cols), dev(y), sigma=sig, k=k, variant=variant, adaptive_k=1)
    res = D.decode(inst.A_cols, y, D.make_constants(n, m, d, k, sig, variant=variant, adaptive_k=1))
    return inst, y, sig, host(xg), stg, res


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("seed", range(10))
def test_adaptive_decode_small_bitwise(seed, variant):
    n, m, d, k = 1024, 256, 7, 25
    print(f"adaptive decode n={n} seed={seed} variant={variant}", flush=True)
    _, _, _, xg, stg, res = run_both(n, m, k, d, 40, I.seed_for(1, 0, seed), variant)
    assert_same_decode(xg, stg, res)
    assert res.k_post < k          # the branch ran: k_0 moved off k


@pytest.mark.parametrize("n,m,k,d,snr,seed,variant", [
    (65536, 6553, 655, 7, 20, 1, 0), (65536, 6553, 655, 7, 40, 2, 0), (65536, 6553, 655, 7, 60, 3, 0),
    (65536, 6553, 655, 7, 40, 2, 1),
    (50003, 2999, 400, 8, 30, 4, 0),       # delta <= 0.05: c = 0.01 (100 iterations)
    (20000, 5000, 1200, 16, 40, 5, 0),     # d = 16
    (10000, 2000, 300, 3, 40, 6, 1),       # d = 3, quantised
    # m > 393216: the bitmask's 8-row summary in LDS, the dense sweep (its flagged-row
    # counts) and H_k's classification kernel
    (200000, 400003, 40000, 6, 40, 8, 0),
    (200000, 400003, 40000, 6, 40, 8, 1),
])
def test_adaptive_decode_mid_size_bitwise(n, m, k, d, snr, seed, variant):
    print(f"adaptive decode n={n} m={m} k={k} d={d} snr={snr} variant={variant}", flush=True)
    _, _, _, xg, stg, res = run_both(n, m, k, d, snr, seed, variant)
    assert_same_decode(xg, stg, res)


def test_adaptive_noiseless_is_the_fixed_k_decode():
    """sigma = 0: the indicator scores of Parallel-l0 have no sparsity in them, and the
    branch leaves the decode unchanged."""
    n, m, d, k = 4096, 1024, 7, 100
    inst = I.draw_instance(n, m, k, d, 0.0, 77, kind="dyadic")
    y = D.measure(inst.A_cols[inst.support], inst.values, inst.eta, m)
    A_t, y_t = dev(inst.A_cols), dev(y)
    xa, sta = R.decode(A_t, y_t, sigma=0.0, k=k, adaptive_k=1)
    xf, stf = R.decode(A_t, y_t, sigma=0.0, k=k)
    assert np.array_equal(host(xa), host(xf))
    assert R.stats_subset(sta) == R.stats_subset(stf)
    assert sta["k_post"] == k


def test_adaptive_and_fixed_decodes_interleave():
    """An adaptive decode rewrites the workspace's own constants, never the cached ones:
    fixed-k decodes of the same problem before and after it (replayed graphs) agree, and
    a second adaptive decode repeats the first."""
    n, m, d, k = 65536, 6553, 7, 655
    inst, y, sig = problem(n, m, k, d, 40, 12)
    A_t, y_t = dev(inst.A_cols), dev(y)
    x1, st1 = R.decode(A_t, y_t, sigma=sig, k=k)
    xa, sta = R.decode(A_t, y_t, sigma=sig, k=k, adaptive_k=1)
    x2, st2 = R.decode(A_t, y_t, sigma=sig, k=k)
    xb, stb = R.decode(A_t, y_t, sigma=sig, k=k, adaptive_k=1)
    assert np.array_equal(host(x1), host(x2)) and R.stats_subset(st1) == R.stats_subset(st2)
    assert np.array_equal(host(xa), host(xb)) and R.stats_subset(sta) == R.stats_subset(stb)
    res = D.decode(inst.A_cols, y, D.make_constants(n, m, d, k, sig, adaptive_k=1))
    assert_same_decode(host(xa), sta, res)
    assert st1["k_post"] == k and sta["k_post"] < k


def test_adaptive_decode_with_iteration_cap():
    """max_iters cuts the t-sweep; the decode stops at the cap with the same state."""
    n, m, d, k = 8192, 2048, 7, 200
    inst, y, sig = problem(n, m, k, d, 30, 21)
    for cap in (1, 2, 5):
        xg, stg = R.decode(dev(inst.A_cols), dev(y), sigma=sig, k=k, adaptive_k=1, max_iters=cap)
        res = D.decode(inst.A_cols, y, D.make_constants(n, m, d, k, sig, adaptive_k=1, max_iters=cap))
        assert_same_decode(host(xg), stg, res)


def _golden_a():
    if not os.path.isdir(GOLDEN):
        return []
    return sorted(f for f in os.listdir(GOLDEN) if f.startswith("decodea") and f.endswith(".npz"))


@pytest.mark.parametrize("fname", _golden_a())
def test_adaptive_full_size_against_stored_oracle(fname):
    """n = 2^20, m = n/10, k = m/10, d = 7 at 20/40/60 dB, quantised at 40 dB, and the
    large-m case n = 2^20, m = n/2, k = m/8, d = 8: the oracle's adaptive decodes stored by
    tests/golden/make_golden.py, matched bitwise."""
    g = np.load(os.path.join(GOLDEN, fname))
    n, m, k, d = int(g["n"]), int(g["m"]), int(g["k"]), int(g["d"])
    sig = float(g["sigma"])
    variant = int(g["variant"])
    print(f"golden {fname}", flush=True)
    inst = I.draw_instance(n, m, k, d, sig, int(g["seed"]))
    y = D.measure(inst.A_cols[inst.support], inst.values, inst.eta, m)
    x_hat, stg = R.decode(dev(inst.A_cols), dev(y), sigma=sig, k=int(g["k_decode"]), variant=variant,
                          adaptive_k=1)
    xg = host(x_hat)
    ref = np.zeros(n, np.float32)
    ref[g["support"]] = g["values"]
    assert np.array_equal(np.nonzero(xg)[0], g["support"])
    assert np.array_equal(xg, ref)
    assert stg["iterations"] == int(g["iterations"]) and stg["accepted"] == int(g["accepted"])
    assert stg["l1_final_fx"] == int(g["L_hat"]) and stg["updates_total"] == int(g["updates_total"])
    assert stg["fx_inexact_x"] == int(g["fx_inexact_x"])
    assert stg["k_post"] == float(g["k_post"])
