"""The quantised variant (Table "scores", middle column; eq:finetune_c_quant) on the GPU
against the oracle, through the C-ABI (params.variant = 1).

Bar: bitwise, as for the continuous scores.  Every iteration of the 1024 x 256 workload
teacher-forced from the oracle's state (per-column decisions, omegas, trial iterate and
residual); whole decodes at that size (20 seeds), at ragged mid sizes, on the large-m
path and in batches; the first iterations at n = 2^20, and whole n = 2^20 decodes against
stored oracle decodes (tests/golden/decodeq_*)."""
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
    x = inst.x_dense()
    y = D.measure(inst.A_cols[inst.support], inst.values, inst.eta, m)
    return inst, x, y, sig


def assert_same_decode(xg, stg, res):
    assert np.array_equal(xg, res.x_hat)
    assert stg["iterations"] == res.iterations
    assert stg["accepted"] == res.accepted
    assert stg["l1_final_fx"] == res.L_hat
    assert stg["converged"] == int(res.converged)
    assert stg["updates_total"] == res.updates_total
    assert stg["fx_inexact_y"] == res.fx_inexact_y and stg["fx_inexact_x"] == res.fx_inexact_x


@pytest.mark.parametrize("seed", range(5))
def test_quantised_step_teacher_forced_small(seed):
    print(f"quantised step small seed={seed}", flush=True)
    n, m, d, k = 1024, 256, 7, 25
    inst, x, y, sig = problem(n, m, k, d, 40, I.seed_for(1, 0, seed))
    C = D.make_constants(n, m, d, k, sig, variant=1)
    assert C.n_iters == 20
    p = R.params_default(n, m, d, k, sig, variant=1)
    A_d, y_d = dev(inst.A_cols), dev(y)
    st = D.init_state(y, n)
    for it in range(C.n_iters):
        out = D.step(inst.A_cols, y, st, C)
        xh, rh = dev(st.x_hat), dev(st.r_hat)
        g = R.step(A_d, y_d, p, it, xh, rh, st.L_hat)
        assert np.array_equal(host(g["updated"]).astype(bool), out.sweep.updated), it
        assert np.array_equal(host(g["omega"]), out.sweep.omega), it
        assert np.array_equal(host(g["x_trial"]), out.x_trial), it
        assert np.array_equal(host(g["r_trial"]), out.r_trial), it
        assert g["accepted"] == out.accepted and g["L_hat"] == out.state.L_hat
        st = out.state


@pytest.mark.parametrize("seed", range(20))
def test_quantised_decode_small_bitwise(seed):
    n, m, d, k = 1024, 256, 7, 25
    inst, x, y, sig = problem(n, m, k, d, 40, I.seed_for(1, 0, seed))
    xg, stg = R.decode(dev(inst.A_cols), dev(y), sigma=sig, k=k, variant=1)
    res = D.decode(inst.A_cols, y, D.make_constants(n, m, d, k, sig, variant=1))
    assert_same_decode(host(xg), stg, res)


@pytest.mark.parametrize("n,m,k,d,snr,seed", [
    (65536, 6553, 655, 7, 20, 1), (65536, 6553, 655, 7, 40, 2), (65536, 6553, 655, 7, 60, 3),
    (50003, 2999, 400, 8, 30, 4),       # delta <= 0.05: c = 0.01 (100 iterations)
    (20000, 5000, 1200, 16, 40, 5),     # rho = 0.24: c = 0.1; d = 16
    (10000, 2000, 300, 3, 40, 6),       # rho = 0.15: c = 0.075; d = 3
    (200000, 400003, 40000, 6, 40, 8),  # m > 393216: the dense sweep and H_k's classification kernel
])
def test_quantised_decode_mid_size_bitwise(n, m, k, d, snr, seed):
    print(f"quantised decode n={n} m={m} k={k} d={d} snr={snr}", flush=True)
    inst, x, y, sig = problem(n, m, k, d, snr, seed)
    xg, stg = R.decode(dev(inst.A_cols), dev(y), sigma=sig, k=k, variant=1)
    res = D.decode(inst.A_cols, y, D.make_constants(n, m, d, k, sig, variant=1))
    assert_same_decode(host(xg), stg, res)


def test_quantised_step_teacher_forced_full_size():
    """n = 2^20, m = n/10, k = m/10, d = 7, 40 dB: iterations 1-3 from the oracle's state."""
    n = 2 ** 20
    m = n // 10
    k, d = m // 10, 7
    inst, x, y, sig = problem(n, m, k, d, 40, I.seed_for(6, 1, 1))
    C = D.make_constants(n, m, d, k, sig, variant=1)
    p = R.params_default(n, m, d, k, sig, variant=1)
    A_d, y_d = dev(inst.A_cols), dev(y)
    st = D.init_state(y, n)
    for it in range(4):
        print(f"quantised step full it={it}", flush=True)
        out = D.step(inst.A_cols, y, st, C)
        xh, rh = dev(st.x_hat), dev(st.r_hat)
        g = R.step(A_d, y_d, p, it, xh, rh, st.L_hat)
        assert np.array_equal(host(g["updated"]).astype(bool), out.sweep.updated)
        assert np.array_equal(host(g["omega"]), out.sweep.omega)
        assert np.array_equal(host(g["x_trial"]), out.x_trial)
        assert np.array_equal(host(g["r_trial"]), out.r_trial)
        assert g["accepted"] == out.accepted and g["L_hat"] == out.state.L_hat
        st = out.state


def test_quantised_batched_matches_single_decodes_and_oracle():
    insts = I.draw_batch(12, 7)
    probs, refs = [], []
    for i, inst in enumerate(insts):
        y = D.measure(inst.A_cols[inst.support], inst.values, inst.eta, inst.m)
        probs.append({"A": dev(inst.A_cols), "y": dev(y), "sigma": inst.sigma, "k": inst.k, "variant": 1})
        if i < 4:
            refs.append(D.decode(inst.A_cols, y, D.make_constants(inst.n, inst.m, 7, inst.k, inst.sigma, variant=1)))
    stats = R.decode_batched(probs)
    for i, (pr, st) in enumerate(zip(probs, stats)):
        x1, st1 = R.decode(pr["A"], pr["y"], sigma=pr["sigma"], k=pr["k"], variant=1)
        assert np.array_equal(host(pr["out"]), host(x1))
        assert R.stats_subset(st) == R.stats_subset(st1)
        if i < len(refs):
            assert np.array_equal(host(pr["out"]), refs[i].x_hat)
            assert st["iterations"] == refs[i].iterations and st["l1_final_fx"] == refs[i].L_hat


def test_quantised_noiseless_is_parallel_l0():
    """sigma = 0: both variants run Parallel-l0's indicators; the decodes are identical."""
    n, m, k, d = 8192, 1024, 150, 7
    inst = I.draw_instance(n, m, k, d, 0.0, 5, kind="dyadic")
    x = inst.x_dense()
    y = D.measure(inst.A_cols, x, inst.eta, m)
    xa, sa = R.decode(dev(inst.A_cols), dev(y), sigma=0.0, k=k, variant=0)
    xq, sq = R.decode(dev(inst.A_cols), dev(y), sigma=0.0, k=k, variant=1, c=0.025)
    assert np.array_equal(host(xa), x) and np.array_equal(host(xq), x)
    assert R.stats_subset(sa) == R.stats_subset(sq)


def _golden_q():
    if not os.path.isdir(GOLDEN):
        return []
    return sorted(f for f in os.listdir(GOLDEN) if f.startswith("decodeq_n") and f.endswith(".npz"))


@pytest.mark.parametrize("fname", _golden_q())
def test_quantised_full_size_against_stored_oracle(fname):
    g = np.load(os.path.join(GOLDEN, fname))
    n, m, k, d = int(g["n"]), int(g["m"]), int(g["k"]), int(g["d"])
    assert int(g["variant"]) == 1
    sig = float(g["sigma"])
    print(f"golden {fname}", flush=True)
    inst = I.draw_instance(n, m, k, d, sig, int(g["seed"]))
    y = D.measure(inst.A_cols[inst.support], inst.values, inst.eta, m)
    x_hat, stg = R.decode(dev(inst.A_cols), dev(y), sigma=sig, k=int(g["k_decode"]), variant=1)
    xg = host(x_hat)
    ref = np.zeros(n, np.float32)
    ref[g["support"]] = g["values"]
    assert np.array_equal(np.nonzero(xg)[0], g["support"])
    assert np.array_equal(xg, ref)
    assert stg["iterations"] == int(g["iterations"]) and stg["accepted"] == int(g["accepted"])
    assert stg["l1_final_fx"] == int(g["L_hat"])
    assert stg["fx_inexact_y"] == int(g["fx_inexact_y"]) and stg["fx_inexact_x"] == int(g["fx_inexact_x"])
