"""Pins of the learned-decision oracle (oracle/mlp.py) against facts that do not come
from the oracle itself: central finite differences of the loss, identities of GELU and
of the logistic loss, torch's own bfloat16 rounding, Adam's first step, and the
definition of the features and labels worked out by hand."""
import math

import numpy as np
import pytest

from oracle import decoder as D
from oracle import mlp as M
from paper_1704_09012_amd import instances as I


def small_net(d, seed):
    rng = np.random.default_rng(seed)
    w = M.init_params(d, seed).astype(np.float64)
    # non-zero biases so that every block of the gradient is exercised
    W1, b1, W2, b2, W3, b3 = M.unpack(w, d)
    b1[:] = rng.normal(0, 0.3, b1.shape)
    b2[:] = rng.normal(0, 0.3, b2.shape)
    b3[:] = rng.normal(0, 0.3, b3.shape)
    return w


def test_param_count_and_layout():
    assert M.n_params(7) == 4866
    w = np.arange(M.n_params(3), dtype=np.float64)
    W1, b1, W2, b2, W3, b3 = M.unpack(w, 3)
    assert W1.shape == (64, 4) and W1[0, 0] == 0 and W1[1, 0] == 4
    assert b1[0] == 256 and W2[0, 0] == 320 and b2[0] == 320 + 4096
    assert W3[1, 0] == 320 + 4096 + 64 + 64 and b3[1] == w[-1]


def test_gelu_identities():
    u = np.linspace(-6, 6, 121)
    g = M.gelu(u)
    assert abs(M.gelu(0.0)) == 0.0
    # Phi(u) + Phi(-u) = 1  =>  gelu(u) - gelu(-u) = u
    assert np.allclose(g - M.gelu(-u), u, atol=1e-15)
    # gelu -> u for large u, -> 0 for very negative u
    assert abs(M.gelu(8.0) - 8.0) < 1e-12 and abs(M.gelu(-8.0)) < 1e-12
    # derivative against central differences
    h = 1e-6
    fd = (M.gelu(u + h) - M.gelu(u - h)) / (2 * h)
    assert np.max(np.abs(fd - M.gelu_grad(u))) < 1e-8


@pytest.mark.parametrize("d,seed", [(3, 1), (7, 2)])
def test_gradient_against_finite_differences(d, seed):
    rng = np.random.default_rng(seed)
    w = small_net(d, seed)
    N = 9
    F = rng.normal(0, 0.5, (N, d + 1))
    Y = np.stack([(rng.random(N) < 0.4).astype(np.float64), rng.normal(0, 1, N)], axis=1)
    loss, g = M.loss_and_grad(w, F, Y, d, lam=0.7)
    idx = np.concatenate([rng.choice(w.size, 300, replace=False), np.arange(w.size - 130, w.size)])
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (M.loss_and_grad(wp, F, Y, d, 0.7)[0] - M.loss_and_grad(wm, F, Y, d, 0.7)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), i


def test_loss_special_values():
    d = 3
    w = np.zeros(M.n_params(d))   # every output is 0: logit 0, value 0
    F = np.ones((4, d + 1))
    Y = np.array([[1, 2.0], [0, 5.0], [1, -1.0], [0, 0.0]])
    loss, g = M.loss_and_grad(w, F, Y, d, lam=1.0)
    # BCE(0, y) = log 2 for either label; squared error of every value: (4 + 25 + 1 + 0) / 4
    assert math.isclose(loss, math.log(2) + 30.0 / 4, rel_tol=1e-12)
    # d loss / d b3 = mean of (sigmoid(0) - y) and of 2 (0 - y_val)
    assert np.allclose(g[-2:], [np.mean(0.5 - Y[:, 0]), np.mean(2 * (0 - Y[:, 1]))])


def test_adam_first_step_is_lr_times_sign():
    rng = np.random.default_rng(3)
    w = rng.normal(size=50)
    g = rng.normal(size=50)
    w1, m, v = M.adam_step(w, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    # bias-corrected m / sqrt(v) is g / |g| at t = 1
    assert np.allclose(w - w1, 1e-3 * np.sign(g), rtol=1e-4)
    # a constant gradient keeps the step at lr
    w2, m, v = M.adam_step(w1, g, m, v, 2, lr=1e-3)
    assert np.allclose(w1 - w2, 1e-3 * np.sign(g), rtol=1e-4)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.normal(0, 3, 5000).astype(np.float32),
                        np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8, 0.0, 65504.0], np.float32)])
    ours = M.to_bf16(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(ours, ref)
    assert M.to_bf16(np.float32(1 + 2 ** -8)) == 1.0            # tie to even
    assert M.to_bf16(np.float32(1 + 3 * 2 ** -8)) == 1 + 2 ** -6   # tie, rounds to the even neighbour above


def test_bf16_forward_close_to_exact():
    d = 7
    rng = np.random.default_rng(5)
    w = small_net(d, 5).astype(np.float32)
    F = rng.normal(0, 0.1, (500, d + 1)).astype(np.float32)
    exact, _ = M.forward(w, F, d)
    approx = M.forward_bf16(w, F, d)
    # bf16 keeps 8 significant bits: relative error of each product operand <= 2^-9
    assert np.max(np.abs(approx - exact)) < 0.05 * (1 + np.max(np.abs(exact)))
    assert not np.array_equal(approx, exact.astype(np.float32))


def test_bf16_forward_rounds_every_product_input():
    """A hand-set chain through one hidden unit per layer, with values worked out by hand.
    GELU is the identity on these inputs (all above 20, where erf is 1 in float64).
      input 20.0703125 = 16 x 1.25439453125; 7 fraction bits: 32.5625 / 128 -> 33: 20.125
      layer 1: 1.75 x 20.125 = 35.21875
      bf16(35.21875) = 32 x (1 + 12.875 / 128) -> 32 x (1 + 13 / 128) = 35.25
      layer 2: 1.5 x 35.25 = 52.875
      bf16(52.875) = 32 x (1 + 83.5 / 128), a tie -> the even 84: 53.0
      layer 3: logit = 1 x 53.0, value = 0.5 x 53.0 = 26.5
    Leaving out the rounding of the input of layer 1, 2 or 3 gives a logit of 52.5, 52.75
    or 52.875 instead, so each of the three roundings is pinned."""
    d = 3
    w = np.zeros(M.n_params(d), np.float32)
    W1, b1, W2, b2, W3, b3 = M.unpack(w, d)
    W1[0, 0] = 1.75
    W2[0, 0] = 1.5
    W3[0, 0] = 1.0
    W3[1, 0] = 0.5
    F = np.zeros((1, d + 1), np.float32)
    F[0, 0] = 20.0703125
    out = M.forward_bf16(w, F, d)
    assert out[0, 0] == np.float32(53.0) and out[0, 1] == np.float32(26.5)
    # planted mistakes: skip the rounding of one product's input (the first of the two
    # to_bf16 calls of each layer) and the output moves as worked out above
    real = M.to_bf16
    for layer, want in ((0, 52.5), (1, 52.75), (2, 52.875)):
        calls = []

        def skipping(a, _layer=layer, _calls=calls):
            _calls.append(1)
            if len(_calls) - 1 == 2 * _layer:
                return np.asarray(a, dtype=np.float32)
            return real(a)
        M.to_bf16 = skipping
        try:
            got = M.forward_bf16(w, F, d)[0, 0]
        finally:
            M.to_bf16 = real
        assert got == np.float32(want), (layer, got)


def test_logit_threshold_inverts_the_sigmoid():
    for t in (0.975, 0.5, 0.1, 0.025):
        lt = M.logit_threshold(t)
        assert abs(1 / (1 + math.exp(-lt)) - t) < 1e-6
    assert M.logit_threshold(1.0) == math.inf


def test_features_and_labels_by_hand():
    A = np.array([[0, 2, 3], [1, 2, 4]], dtype=np.int32)
    r = np.array([0.5, -1.0, 0.25, -0.125, 2.0], np.float32)
    F = M.features(A, r, 0.01)
    assert np.array_equal(F[0], np.float32([-0.125, 0.25, 0.5, 0.01]))
    assert np.array_equal(F[1], np.float32([-1.0, 0.25, 2.0, 0.01]))
    x = np.array([0, 1.0, -0.5, 0.2], np.float32)
    xh = np.array([0.3, 1.0, 0.0, 0.199], np.float32)
    L = M.labels(x, xh, sigma=0.01, d=9)      # threshold 0.01
    assert np.array_equal(L[:, 0], [0, 0, 1, 0])   # j=0 not in supp(x); j=1 exact; j=3 within 0.001
    assert np.allclose(L[:, 1], [-0.3, 0.0, -0.5, 0.001], atol=1e-7)


def test_learned_loop_with_a_silent_network_is_the_analytic_loop():
    """A network whose logit is always below threshold never updates: every learned
    iteration is rejected (x' = x_hat) and the retry is the analytic iteration."""
    n, m, k, d = 512, 128, 10, 7
    sig = float(np.float32(I.sigma_for_snr(40, n, m, k, d)))
    inst = I.draw_instance(n, m, k, d, sig, 11)
    y = D.measure(inst.A_cols, inst.x_dense(), inst.eta, m)
    C = D.make_constants(n, m, d, k, sig)
    w = np.zeros(M.n_params(d), np.float32)
    w[-2] = -1e4                     # b3[0]: logit = -1e4
    x, iters, acc, L = M.learned_decode(inst.A_cols, y, C, w)
    ref = D.decode(inst.A_cols, y, C)
    assert np.array_equal(x, ref.x_hat) and L == ref.L_hat and acc == ref.accepted



def test_learned_loop_counts_rounded_updates_as_the_analytic_loop():
    """With the silent network the learned loop's count of updated x'_j != 0 whose 2^-40
    fixed-point conversion rounds is the analytic decode's fx_inexact_x (only the retries
    update).  The instance is scaled by 2^-20 (y and sigma; exact in float), so that
    its x'_j fall below 2^-17 and the count is not 0."""
    n, m, k, d = 512, 128, 10, 7
    sig = float(np.float32(I.sigma_for_snr(40, n, m, k, d)))
    inst = I.draw_instance(n, m, k, d, sig, 12)
    scale = np.float32(2.0 ** -20)
    y = D.measure(inst.A_cols, inst.x_dense(), inst.eta, m) * scale
    C = D.make_constants(n, m, d, k, sig * float(scale))
    w = np.zeros(M.n_params(d), np.float32)
    w[-2] = -1e4
    x, iters, acc, L, inexact = M.learned_decode(inst.A_cols, y, C, w, count_inexact=True)
    ref = D.decode(inst.A_cols, y, C)
    assert np.array_equal(x, ref.x_hat) and L == ref.L_hat
    assert inexact == ref.fx_inexact_x > 0