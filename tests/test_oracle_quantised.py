"""Pins for the quantised variant of the oracle (Table "scores", middle column; Alg. 1's
quantised flag; eq:finetune_c_quant), all on the CPU:

  * the indicator scores are thresholds of the fp64 posteriors: q_e(a | t) = 1 exactly
    where p_breve_e(a) >= t and q_z(v | t) = 1 where p_breve_z(v) >= 1 - t, away from the
    tables' error band;
  * a column worked out by hand (counts, mean, winner);
  * iteration 0 (t = 1) counts every row as a zero and updates nothing;
  * the vectorised float32 sweep against the fp64 shadow with indicator scores;
  * the c rule and the recovery error of whole decodes.
"""
import numpy as np
import pytest

from oracle import decoder as D
from oracle import posterior as P
from oracle import scores as S
from oracle import shadow as SH
from paper_1704_09012_amd import instances as I


@pytest.mark.parametrize("d,rho,sig", [(7, 25 / 256, 0.00826797), (7, 0.1, 0.0836632), (8, 1 / 8, 0.01)])
@pytest.mark.parametrize("t", [0.95, 0.7, 0.5, 0.25, 0.05])
def test_indicator_scores_are_posterior_thresholds(d, rho, sig, t):
    t32 = np.float32(t)
    Te = S.build_table("e", d, rho, sig)
    Tz = S.build_table("z", d, rho, sig)
    rng = np.random.Generator(np.random.PCG64(int(t * 100)))
    for kind, tab, level in (("e", Te, t32), ("z", Tz, (np.float32(1.0) - t32).astype(np.float32))):
        a = (rng.random(20000) * 1.2 * tab.R).astype(np.float32)
        q = S.lookup(tab, a) >= level
        ref = P.p_breve(kind, a.astype(np.float64), d, rho, sig)
        clear = np.abs(ref - float(level)) > 2e-6      # the table is within 1e-6 of p_breve
        assert clear.sum() > 19000
        assert np.array_equal(q[clear], (ref >= float(level))[clear])
        # a threshold in |a|: once 0, it stays 0 on the sorted grid
        o = np.argsort(a)
        assert np.all(np.diff(q[o].astype(np.int8)) <= 0)


def test_quantised_column_by_hand():
    """sigma = 0.01, t = 0.5 (iteration 20 at c = 0.025).  Rows 0.5, 0.5 + 2^-10, 0.5 - 2^-10
    agree with each other (differences far below the e-threshold, about 0.03) and with no
    other row; only the row 0 counts as a zero.  For p = 0: n_e = 3, n_z = 1, omega =
    (0.5 + (0.5 + 2^-10) + (0.5 - 2^-10)) / 3 = 1.5 / 3 = 0.5 exactly, sum |v - omega| =
    6.25 + 2^-9 <= 7.75 = sum |v|, so row 0 passes (n_e - n_z = 2 >= alpha = 2); rows 1
    and 2 tie with it on n_e and the first wins.  The continuous scores weigh the two
    near rows below 1, so their omega differs."""
    C = D.make_constants(1024, 256, 7, 25, 0.01, variant=1, c=0.025)
    v = np.float32([0.5, 0.5 + 2 ** -10, 0.5 - 2 ** -10, 0.0, 3.0, -2.0, 1.25])
    A = np.arange(7, dtype=np.int32)[None, :]
    sw = D.sweep(A, v, np.zeros(1, np.float32), S.t_of(20, C.c), C)
    assert float(S.t_of(20, C.c)) == 0.5
    assert sw.updated[0] and sw.p_star[0] == 0
    assert sw.omega[0] == np.float32(0.5) and sw.n_e[0] == 3 and sw.n_z[0] == 1
    Cc = D.make_constants(1024, 256, 7, 25, 0.01, variant=0, c=0.025)
    swc = D.sweep(A, v, np.zeros(1, np.float32), S.t_of(20, Cc.c), Cc)
    assert swc.omega[0] != np.float32(0.5) and swc.n_e[0] < 3


def test_quantised_iteration_zero_updates_nothing():
    n, m, k, d = 4096, 1024, 100, 7
    sig = I.sigma_for_snr(30, n, m, k, d)
    inst = I.draw_instance(n, m, k, d, sig, 3)
    y = D.measure(inst.A_cols, inst.x_dense(), inst.eta, m)
    C = D.make_constants(n, m, d, k, sig, variant=1)
    sw = D.sweep(inst.A_cols, y, np.zeros(n, np.float32), S.t_of(0, C.c), C)
    assert not sw.updated.any() and np.all(sw.n_z == np.float32(d))
    sw1 = D.sweep(inst.A_cols, y, np.zeros(n, np.float32), S.t_of(1, C.c), C)
    assert sw1.updated.any()


def test_quantised_c_rule_and_iterations():
    # eq:finetune_c_quant: delta = 0.25, rho = 25/256 < 0.1 -> 0.05 (20 iterations)
    assert D.make_constants(1024, 256, 7, 25, 0.01, variant=1).c == 0.05
    assert D.make_constants(1024, 256, 7, 25, 0.01, variant=1).n_iters == 20
    assert D.make_constants(1024, 256, 7, 40, 0.01, variant=1).c == 0.075    # rho = 0.156
    assert D.make_constants(1024, 256, 7, 60, 0.01, variant=1).c == 0.1      # rho = 0.234
    assert D.make_constants(10000, 400, 7, 60, 0.01, variant=1).c == 0.01    # delta = 0.04
    assert D.make_constants(1024, 256, 7, 25, 0.01, variant=0).c == 0.025


@pytest.mark.parametrize("it", [1, 3, 8, 15])
def test_quantised_sweep_matches_fp64_shadow(it):
    n, m, k, d = 4096, 1024, 100, 7
    sig = I.sigma_for_snr(30, n, m, k, d)
    inst = I.draw_instance(n, m, k, d, sig, 7)
    y = D.measure(inst.A_cols, inst.x_dense(), inst.eta, m)
    C = D.make_constants(n, m, d, k, sig, variant=1)
    st = D.init_state(y, n)
    for _ in range(2):
        st = D.step(inst.A_cols, y, st, C).state
    t = S.t_of(it, C.c)
    sw = D.sweep(inst.A_cols, st.r_hat, st.x_hat, t, C)
    rng = np.random.Generator(np.random.PCG64(it))
    cols = np.concatenate([np.nonzero(sw.updated)[0], rng.choice(n, 600, replace=False)])
    checked = 0
    for j in cols:
        v = [float(st.r_hat[r]) for r in inst.A_cols[j]]
        upd, row, omega, m_outer, m_other = SH.decision(v, float(t), 2.0, d, k / m, sig, split=True, quantised=True)
        if m_outer < 1e-5 or m_other < 2e-6:
            continue
        checked += 1
        assert bool(sw.updated[j]) == upd, j
        if upd:
            assert sw.p_star[j] == row
            assert abs(float(sw.omega[j]) - omega) <= 1e-6 * max(1.0, abs(omega))
    assert checked >= 300 and sw.updated.sum() > 0


@pytest.mark.parametrize("snr,bound", [(40, 1e-2), (60, 2e-3)])
def test_quantised_recovery_at_noise_floor(snr, bound):
    n = 2 ** 14
    m = n // 10
    k = m // 10
    errs = []
    for seed in range(3):
        sig = I.sigma_for_snr(snr, n, m, k, 7)
        inst = I.draw_instance(n, m, k, 7, sig, seed)
        x = inst.x_dense()
        y = D.measure(inst.A_cols, x, inst.eta, m)
        res = D.decode(inst.A_cols, y, D.make_constants(n, m, 7, k, sig, variant=1))
        errs.append(np.linalg.norm(res.x_hat - x) / np.linalg.norm(x))
    print(snr, errs)
    assert np.median(errs) < bound, errs
