"""Pins for the oracle decoder (Alg. 1 / Alg. 2), all on the CPU.

  * sketch and residual against exact rational arithmetic (fractions.Fraction);
  * the vectorised float32 sweep against a scalar fp64 transcription of the column loop
    of Alg. 1 that evaluates p_breve directly (decisions must agree wherever the fp64
    margin exceeds the float32/table resolution);
  * H_k against Python's sorted();
  * noiseless exact recovery (the sigma = 0 reduction is Parallel-l0, whose convergence
    theorem guarantees recovery of dissociated signals), bitwise x_hat == x;
  * brute-force l0 minimisation for n <= 16;
  * invariants of the loop: r_hat equals the exact residual of x_hat after every
    iteration, ||r_hat||_1 strictly decreases on accepted iterations, |supp x_hat| <= k,
    a rejected iteration leaves the state untouched;
  * recovery error at the noise floor for 40 and 60 dB.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import bruteforce as B
from oracle import decoder as D
from oracle import posterior as P
from oracle import scores as S
from oracle import shadow as SH
from paper_1704_09012_amd import instances as I


def _instance(n, m, k, d, snr, seed, kind="gaussian"):
    sig = 0.0 if snr is None else I.sigma_for_snr(snr, n, m, k, d)
    inst = I.draw_instance(n, m, k, d, sig, seed, kind=kind)
    x = inst.x_dense()
    y = D.measure(inst.A_cols, x, inst.eta, m)
    return inst, x, y, sig


def _exact_fl32(fr: Fraction) -> np.float32:
    # Fraction -> nearest float64 (correctly rounded by Python) -> float32 is a double
    # rounding; both contract paths use fl64 then fl32, which this reproduces.
    return np.float32(float(fr))


def test_sketch_matches_exact_rational_sum():
    rng = np.random.Generator(np.random.PCG64(3))
    n, m, d = 300, 40, 5
    A = I.draw_columns(rng, n, m, d)
    x = (rng.standard_normal(n) * 3).astype(np.float32)
    x[np.abs(x) < 2.0 ** -15] = 1.0          # keep every value a multiple of 2^-40
    y = D.sketch(A, x, m)
    for i in range(m):
        cols = np.nonzero((A == i).any(axis=1))[0]
        exact = sum((Fraction(float(x[j])) for j in cols), Fraction(0))
        assert y[i] == _exact_fl32(exact)


def test_residual_is_exact_after_every_iteration():
    inst, x, y, sig = _instance(512, 128, 12, 7, 40, seed=2)
    C = D.make_constants(512, 128, 7, 12, sig)
    st = D.init_state(y, 512)
    for _ in range(6):
        out = D.step(inst.A_cols, y, st, C)
        st = out.state
        xs = st.x_hat
        for i in range(128):
            cols = np.nonzero((inst.A_cols == i).any(axis=1))[0]
            exact = Fraction(float(y[i])) - sum((Fraction(float(xs[j])) for j in cols), Fraction(0))
            assert st.r_hat[i] == _exact_fl32(exact)
        assert st.L_hat == sum(int(round(abs(float(v)) * 2 ** 30)) for v in st.r_hat) or \
            st.L_hat == D.l1_fixed(st.r_hat)


@pytest.mark.parametrize("it", [0, 1, 5, 20, 38])
def test_sweep_matches_scalar_fp64_transcription(it):
    n, m, k, d = 4096, 1024, 100, 7
    inst, x, y, sig = _instance(n, m, k, d, 30, seed=7)
    C = D.make_constants(n, m, d, k, sig)
    # a realistic residual: after the first accepted iterations of a decode
    st = D.init_state(y, n)
    st = D.step(inst.A_cols, y, st, C).state
    t = S.t_of(it, C.c)
    sw = D.sweep(inst.A_cols, st.r_hat, st.x_hat, t, C)
    # at t = 1 the float32 outer test fl32(1 - z) >= 1 holds exactly for z <= 2^-25 (see
    # test_first_pass_outer_test_is_float32_rounding); the fp64 shadow takes that threshold
    t_shadow = float(t) if it > 0 else 1.0 - 2.0 ** -25
    checked = agree = 0
    rng = np.random.Generator(np.random.PCG64(it))
    cols = np.concatenate([np.nonzero(sw.updated)[0], rng.choice(n, 600, replace=False)])
    for j in cols:
        v = [float(st.r_hat[r]) for r in inst.A_cols[j]]
        upd, row, omega, m_outer, m_other = SH.decision(v, t_shadow, 2.0, d, k / m, sig, split=True)
        # the outer test's margin relative to its threshold 1 - t (the table's error in
        # the tail is about 1e-5 of the score), the others' absolute
        if m_outer < (1e-3 * (1.0 - t_shadow) if it == 0 else 1e-5) or m_other < 1e-5:
            continue
        checked += 1
        if not upd:
            assert not sw.updated[j]
            agree += 1
            continue
        assert sw.updated[j]
        assert sw.p_star[j] == row
        assert abs(float(sw.omega[j]) - omega) <= 1e-5 * max(1.0, abs(omega))
        agree += 1
    assert checked >= 300 and agree == checked
    if it == 0:
        assert sw.updated.sum() > 0       # iteration 0 does update columns


def test_hard_threshold_against_sorted():
    rng = np.random.Generator(np.random.PCG64(9))
    x = rng.standard_normal(1000).astype(np.float32)
    x[rng.choice(1000, 400, replace=False)] = 0.0
    x[10] = x[20] = np.float32(9.5)           # a tie: the smaller index wins
    x[30] = np.float32(-9.5)
    for k in (1, 2, 3, 50, 599, 600, 700):
        got = D.hard_threshold(x, k)
        order = sorted(np.nonzero(x)[0], key=lambda j: (-abs(float(x[j])), j))[:k]
        want = np.zeros_like(x)
        want[order] = x[order]
        assert np.array_equal(got, want)
    assert np.array_equal(np.nonzero(D.hard_threshold(x, 1))[0], [10])


@pytest.mark.parametrize("n,m,k,seed", [(1024, 256, 20, 1), (4096, 512, 50, 2), (8192, 1024, 150, 3)])
def test_noiseless_exact_recovery_parallel_l0(n, m, k, seed):
    """sigma = 0: the scores are Parallel-l0's indicators; rho well below 0.3 recovers x exactly."""
    inst, x, y, sig = _instance(n, m, k, 7, None, seed, kind="dyadic")
    C = D.make_constants(n, m, 7, k, 0.0, alpha=2.0)
    res = D.decode(inst.A_cols, y, C)
    assert res.converged and res.L_hat == 0
    assert np.array_equal(res.x_hat, x)
    assert res.iterations <= 3 * math.ceil(math.log2(k)) + 2


def test_bruteforce_l0_tiny():
    """A converged noiseless decode is the unique sparsest solution of A x = y."""
    n, m, k, d = 16, 14, 2, 3
    n_conv = 0
    for seed in range(100, 140):
        inst = I.draw_instance(n, m, k, d, 0.0, seed, kind="dyadic")
        x = inst.x_dense()
        y = D.measure(inst.A_cols, x, inst.eta, m)
        A = B.dense_matrix(inst.A_cols, m)
        s, sols = B.l0_minimisers(A, y.astype(np.float64), max_support=3)
        assert s is not None and s <= k
        C = D.make_constants(n, m, d, k, 0.0, alpha=3.0)
        res = D.decode(inst.A_cols, y, C)
        if res.converged:
            n_conv += 1
            assert np.count_nonzero(res.x_hat) == s
            assert any(np.allclose(res.x_hat.astype(np.float64), sol, rtol=0, atol=1e-9) for sol in sols)
            if len(sols) == 1:
                assert np.array_equal(res.x_hat, x)
    assert n_conv >= 10


def test_loop_invariants_and_rollback():
    n, m, k, d = 2048, 512, 40, 7
    inst, x, y, sig = _instance(n, m, k, d, 30, seed=4)
    C = D.make_constants(n, m, d, k, sig)
    st = D.init_state(y, n)
    prev_t = 2.0
    seen_reject = False
    while st.it < C.n_iters:
        t = float(S.t_of(st.it, C.c))
        assert t < prev_t
        prev_t = t
        out = D.step(inst.A_cols, y, st, C)
        assert np.count_nonzero(out.x_trial) <= k
        if out.accepted:
            assert out.state.L_hat < st.L_hat
            assert np.array_equal(out.state.x_hat, out.x_trial)
        else:
            seen_reject = True
            assert out.state.L_hat == st.L_hat
            assert out.state.x_hat is st.x_hat and out.state.r_hat is st.r_hat
        assert D.l1_fixed(out.state.r_hat) == out.state.L_hat
        st = out.state
    assert seen_reject


@pytest.mark.parametrize("snr,bound", [(40, 1e-2), (60, 2e-3)])
def test_recovery_at_noise_floor(snr, bound):
    n = 2 ** 14
    m = n // 10
    k = m // 10
    errs = []
    for seed in range(3):
        inst, x, y, sig = _instance(n, m, k, 7, snr, seed)
        res = D.decode(inst.A_cols, y, D.make_constants(n, m, 7, k, sig))
        errs.append(np.linalg.norm(res.x_hat - x) / np.linalg.norm(x))
    assert np.median(errs) < bound, errs


def test_fixed_point_round_trip_and_l1():
    v = np.array([0.0, 1.0, -2.5, 3e-5, -7.25e-3], dtype=np.float32)
    assert np.array_equal(D.from_fixed(D.to_fixed(v)), v)
    assert D.l1_fixed(v) == sum(int(round(abs(float(a)) * 2 ** 30)) for a in v)
    with pytest.raises(OverflowError):
        D.to_fixed(np.array([2.0 ** 23], dtype=np.float32))


def _rint_half_even(q: Fraction) -> int:
    fl = q.numerator // q.denominator
    rem = q - fl
    return fl + (1 if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1) else 0)


def test_fixed_point_small_values_against_fractions():
    """rint(2^40 v) is exact for every float32 |v| >= 2^-17 and rounds (half to even)
    below; the round trip gives fl32(2^-40 rint(2^40 v)) and fx_inexact counts exactly the
    entries that round.  This is the one place where the residual departs from the exactly
    rounded y - A x: r_hat <- y is inexact on rows with |y_i| < 2^-17."""
    rng = np.random.Generator(np.random.PCG64(12))
    v = np.concatenate([
        (rng.standard_normal(3000) * 2.0 ** rng.integers(-30, 3, 3000)).astype(np.float32),
        np.float32([2.0 ** -17, -2.0 ** -17, 2.0 ** -40, 3 * 2.0 ** -41, 2.0 ** -41, -(2.0 ** -41), 0.0])])
    got = D.from_fixed(D.to_fixed(v))
    n_round = 0
    for a, g in zip(v, got):
        q = Fraction(float(a)) * 2 ** 40
        assert g == np.float32(float(Fraction(_rint_half_even(q), 2 ** 40)))
        if q.denominator != 1:
            n_round += 1
            assert abs(float(a)) < 2.0 ** -17
        else:
            assert g == a
    assert D.fx_inexact(v) == n_round and n_round > 100
    # the half-way cases go to the even neighbour: 1.5 -> 2, 0.5 -> 0, -0.5 -> 0
    assert list(D.to_fixed(np.float32([3 * 2.0 ** -41, 2.0 ** -41, -(2.0 ** -41)]))) == [2, 0, 0]


def test_decode_counts_inexact_conversions():
    """The decode's counters: rows of y_hat below 2^-17 (here forced by zeroing most of
    a small instance's noise and signal rows) and updated entries x'_j below it."""
    inst, x, y, sig = _instance(1024, 256, 25, 7, 40, seed=21)
    y = y.copy()
    y[:40] = (np.random.default_rng(21).uniform(-1.0, 1.0, 40) * 2.0 ** -18).astype(np.float32)
    C = D.make_constants(1024, 256, 7, 25, sig)
    res = D.decode(inst.A_cols, y, C)
    want_y = sum(1 for v in y if (Fraction(float(v)) * 2 ** 40).denominator != 1)
    assert res.fx_inexact_y == want_y >= 25
    assert res.fx_inexact_x >= 0


def test_first_pass_outer_test_is_float32_rounding():
    """At t = 1 (iteration 0) the outer test 1 - p_breve_z(r_i) >= t holds, in float32,
    exactly where the score has dropped to 2^-25 or below: fl32(1 - z) rounds to 1 for
    z <= 2^-25 (the half-way value ties to the even neighbour, 1) and stays below 1 above.
    With the headline workload's ratios at 40 dB that starts near 6.67 sigma, before the
    table's end R_z beyond which the score is exactly 0; so iteration 0 can update columns
    whose rows carry large residuals."""
    lo, hi = np.float32(2.0 ** -27).view(np.uint32), np.float32(2.0 ** -23).view(np.uint32)
    z = np.arange(lo, hi + 1, dtype=np.uint32).view(np.float32)      # every float32 in between
    one = (np.float32(1.0) - z).astype(np.float32) >= np.float32(1.0)
    assert np.array_equal(one, z <= np.float32(2.0 ** -25))
    d, m, k, sig = 7, 104857, 10485, 0.00836632
    C = D.make_constants(2 ** 20, m, d, k, sig)
    a = (np.linspace(5.0, 8.0, 300001) * sig).astype(np.float32)
    zt = S.lookup(C.Tz, a)
    passes = (np.float32(1.0) - zt).astype(np.float32) >= np.float32(1.0)
    i0 = int(np.argmax(passes))
    first = a[i0]
    assert passes[i0:].all()
    assert 6.5 < first / sig < 6.8 < C.Tz.R / sig
    assert S.lookup(C.Tz, np.float32(first)) > 0.0          # the score itself is not 0 there
    # the fp64 posterior puts that onset where p_breve_z is about 2^-25
    assert 0.5 * 2.0 ** -25 < P.p_breve("z", float(first), d, k / m, sig) < 2.0 * 2.0 ** -25
    # the sweep at t = 1: a column whose rows all carry the same large residual updates by
    # about that residual; one whose rows stay below the onset does not
    A = np.array([[0, 1, 2, 3, 4, 5, 6], [7, 8, 9, 10, 11, 12, 13]], dtype=np.int32)
    r = np.zeros(14, np.float32)
    r[:7] = np.float32(10 * sig)
    r[7:] = np.float32(6.4 * sig)
    sw = D.sweep(A, r, np.zeros(2, np.float32), S.t_of(0, C.c), C)
    assert list(sw.updated) == [True, False]
    assert abs(float(sw.omega[0]) - 10 * sig) <= 1e-6 * 10 * sig
    assert sw.n_e[0] == np.float32(7.0) and sw.n_z[0] == np.float32(0.0)


def test_alpha_outside_its_range_is_refused():
    # Alg. 1's input: alpha in (1, d]; d = 1 leaves no admissible alpha
    for d, alpha in [(7, 1.0), (7, 7.5), (1, 2.0), (1, 1.0)]:
        with pytest.raises(ValueError):
            D.make_constants(1000, 300, d, 20, 0.01, alpha=alpha)
    assert D.make_constants(1000, 300, 7, 20, 0.01, alpha=7.0).alpha == np.float32(7.0)
