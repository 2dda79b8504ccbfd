"""Pins for the adaptive_k branch of the oracle (Alg. 1, reading R17): the sparsity k_0
worked out by hand, the rebuilt posteriors against the ordinary constants builder, and
whole decodes (recovery at the noise floor, k_0 shrinking as the support is found)."""
import numpy as np
import pytest

from oracle import decoder as D
from oracle import scores as S
from paper_1704_09012_amd import instances as I


def test_adapted_sparsity_by_hand():
    # sigma = 0.01: the z-table ends near 7 sigma = 0.07, so entries of magnitude >= 5 have
    # p_breve_z = 0 and each adds exactly 1; zeros add nothing
    C = D.make_constants(4096, 1000, 7, 30, 0.01, adaptive_k=1)
    x = np.zeros(4096, np.float32)
    x[[3, 70, 900]] = [5.0, -5.0, 7.5]
    assert D.adapted_sparsity(C, x) == 27.0
    # an entry inside the table adds fl32(1 - Tz(|v|)), a fraction with 30 bits kept
    x[5] = np.float32(0.02)
    z = S.lookup(C.Tz, np.float32(0.02))
    term = float(np.rint(float(np.float32(1.0) - z) * 2 ** 30)) * 2.0 ** -30
    assert D.adapted_sparsity(C, x) == 27.0 - term and 0.0 < term < 1.0
    # the floor: m // 100 = 10 once 25 entries are found
    y = np.zeros(4096, np.float32)
    y[:25] = 4.0
    assert D.adapted_sparsity(C, y) == 10.0
    # and never below 1 when m < 100
    C2 = D.make_constants(500, 60, 7, 5, 0.01, adaptive_k=1)
    z5 = np.zeros(500, np.float32)
    z5[:7] = 3.0
    assert D.adapted_sparsity(C2, z5) == 1.0


def test_rebuilt_posteriors_are_the_constants_of_k0():
    C = D.make_constants(4096, 1000, 7, 30, 0.01, adaptive_k=1)
    x = np.zeros(4096, np.float32)
    x[:12] = 2.0
    A = D.adapt(C, x)
    ref = D.make_constants(4096, 1000, 7, 18, 0.01)
    assert A.k_post == 18.0 and A.k == 30
    assert np.array_equal(A.Tz.T, ref.Tz.T) and np.array_equal(A.Te.T, ref.Te.T)
    assert A.Tz.inv_h == ref.Tz.inv_h and A.c == C.c and A.n_iters == C.n_iters and A.tol == C.tol


def test_adaptive_decode_shrinks_k0_and_recovers():
    n, m, k, d = 8192, 1024, 100, 7
    sig = I.sigma_for_snr(40, n, m, k, d)
    inst = I.draw_instance(n, m, k, d, sig, 17)
    x = inst.x_dense()
    y = D.measure(inst.A_cols, x, inst.eta, m)
    C = D.make_constants(n, m, d, k, sig, adaptive_k=1)
    st = D.init_state(y, n)
    ks = [C.k_post]
    while st.it < C.n_iters and not D.converged(st, C):
        out = D.step(inst.A_cols, y, st, C)
        if out.accepted:
            C = D.adapt(C, out.state.x_hat)
            ks.append(C.k_post)
        st = out.state
    assert len(ks) > 2 and all(a >= b for a, b in zip(ks, ks[1:]))
    assert ks[-1] < 0.5 * k
    res = D.decode(inst.A_cols, y, D.make_constants(n, m, d, k, sig, adaptive_k=1))
    assert np.array_equal(res.x_hat, st.x_hat)
    assert np.linalg.norm(res.x_hat - x) / np.linalg.norm(x) < 1e-2


@pytest.mark.parametrize("variant", [0, 1])
def test_adaptive_recovery_at_noise_floor(variant):
    n = 2 ** 14
    m = n // 10
    k = m // 10
    errs = []
    for seed in range(3):
        sig = I.sigma_for_snr(40, n, m, k, 7)
        inst = I.draw_instance(n, m, k, 7, sig, seed)
        x = inst.x_dense()
        y = D.measure(inst.A_cols, x, inst.eta, m)
        res = D.decode(inst.A_cols, y, D.make_constants(n, m, 7, k, sig, variant=variant, adaptive_k=1))
        errs.append(np.linalg.norm(res.x_hat - x) / np.linalg.norm(x))
    assert np.median(errs) < 1e-2, errs
