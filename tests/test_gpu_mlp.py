"""The learned column decision on the GPU against the oracle (oracle/mlp.py).

Bars: features and labels bitwise; fp32 gradients within 1e-4 of the fp64 oracle's
(relative to the largest component); fp32 inference within 1e-4; matrix-core bf16
inference within 1e-2 of the oracle's bf16 emulation (the accumulation order of the
matrix cores is not specified); the learned iteration's decisions equal the oracle's
wherever the logit is more than 1e-2 from the threshold; training lowers the loss; and
a silent network reproduces the analytic decoder bit for bit; training resumed from a
checkpoint equals uninterrupted training bit for bit.
"""
import math

import numpy as np
import pytest

from oracle import decoder as D
from oracle import mlp as M
from paper_1704_09012_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_1704_09012_amd.rl0")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def net(d, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    w = M.init_params(d, seed)
    W1, b1, W2, b2, W3, b3 = M.unpack(w, d)
    W1 *= scale
    b1[:] = rng.normal(0, 0.2, 64)
    b2[:] = rng.normal(0, 0.2, 64)
    b3[:] = rng.normal(0, 0.2, 2)
    return w.astype(np.float32)


def state_after(inst, y, its):
    C = D.make_constants(inst.n, inst.m, inst.d, inst.k, inst.sigma)
    st = D.init_state(y, inst.n)
    for _ in range(its):
        st = D.step(inst.A_cols, y, st, C).state
    return st, C


@pytest.mark.parametrize("d", [7, 3, 12])
def test_features_and_labels_bitwise(d):
    inst = I.draw_instance(5000, 700, 60, d, 0.01, 21)
    y = D.measure(inst.A_cols, inst.x_dense(), inst.eta, inst.m)
    st, _ = state_after(inst, y, 6)
    f = R.mlp_features(dev(inst.A_cols), dev(st.r_hat), 0.01)
    assert np.array_equal(host(f), M.features(inst.A_cols, st.r_hat, 0.01))
    lab = R.mlp_labels(dev(inst.x_dense()), dev(st.x_hat), d, 0.01)
    assert np.array_equal(host(lab), M.labels(inst.x_dense(), st.x_hat, 0.01, d))


@pytest.mark.parametrize("d,N", [(7, 4096), (7, 1000), (3, 130)])
def test_gradient_matches_fp64_oracle(d, N):
    rng = np.random.default_rng(N)
    w = net(d, 7)
    F = rng.normal(0, 0.3, (N, d + 1)).astype(np.float32)
    Y = np.stack([(rng.random(N) < 0.3).astype(np.float32), rng.normal(0, 1, N).astype(np.float32)], 1)
    g, loss = R.mlp_grad(dev(F), dev(Y), dev(w), lam=1.0)
    lo, go = M.loss_and_grad(w, F, Y, d, lam=1.0)
    g = host(g)
    err = np.max(np.abs(g - go)) / np.max(np.abs(go))
    print(f"d={d} N={N} grad rel err {err:.2e} loss {loss} vs {lo}", flush=True)
    assert err <= 1e-4
    assert abs(loss - lo) <= 1e-4 * max(1.0, abs(lo))


@pytest.mark.parametrize("d", [7, 3, 15])
def test_inference_fp32_and_bf16(d):
    rng = np.random.default_rng(8)
    w = net(d, 9)
    F = rng.normal(0, 0.2, (3000, d + 1)).astype(np.float32)
    exact, _ = M.forward(w, F, d)
    o32 = host(R.mlp_forward(dev(F), dev(w), bf16=False))
    assert np.max(np.abs(o32 - exact)) <= 1e-4 * (1 + np.max(np.abs(exact)))
    o16 = host(R.mlp_forward(dev(F), dev(w), bf16=True))
    emu = M.forward_bf16(w, F, d)
    print("bf16 max diff", np.max(np.abs(o16 - emu)), flush=True)
    assert np.max(np.abs(o16 - emu)) <= 1e-2


@pytest.mark.parametrize("d", [7, 12])
def test_learned_step_decisions_match_the_oracle(d):
    n, m, k = 4096, 1024, 100
    sig = float(np.float32(I.sigma_for_snr(40, n, m, k, d)))
    inst = I.draw_instance(n, m, k, d, sig, 31)
    y = D.measure(inst.A_cols, inst.x_dense(), inst.eta, m)
    for its in (3, 12):
        st, C = state_after(inst, y, its)
        t = D._scores.t_of(its, C.c)
        # a network whose logit passes the threshold for about a tenth of the columns
        w = net(d, 12 + its, scale=4.0)
        w[-2] = 0.0
        logit0 = M.forward_bf16(w, M.features(inst.A_cols, st.r_hat, sig), d)[:, 0]
        w[-2] = np.float32(M.logit_threshold(t) - np.quantile(logit0, 0.9))
        x_prime, upd, value, logit = M.learned_sweep(inst.A_cols, st.r_hat, st.x_hat, t, sig, w)
        assert 0 < upd.sum() < n
        params = R.params_default(n, m, d, k, sig, mlp=dev(w))
        x_t, r_t = dev(st.x_hat), dev(st.r_hat)
        wt = dev(w)
        params.mlp = wt.data_ptr()
        out = R.step(dev(inst.A_cols), dev(y), params, its, x_t, r_t, st.L_hat)
        gu = host(out["updated"]).astype(bool)
        go = host(out["omega"])
        lt = M.logit_threshold(D._scores.t_of(its, C.c))
        clear = np.abs(logit - lt) > 1e-2
        print(f"its={its}: oracle updates {upd.sum()}, gpu {gu.sum()}, clear {clear.sum()}", flush=True)
        assert np.array_equal(gu[clear], upd[clear])
        both = gu & upd
        assert np.max(np.abs(go[both] - value[both]), initial=0.0) <= 1e-2


@pytest.mark.parametrize("shift", [0, 20])
def test_silent_network_reproduces_the_analytic_decoder(shift):
    """A network whose logit stays below threshold: the learned decode is the analytic
    one.  With the instance scaled by 2^-20 (y and sigma; exact in float) its x'_j fall
    below 2^-17, so the count of rounded updates (fx_inexact_x, over the learned and the
    analytic sub-iterations) is not 0 and is the oracle's, by both of its routes."""
    n, m, k, d = 4096, 800, 70, 7
    sig = float(np.float32(I.sigma_for_snr(40, n, m, k, d)))
    inst = I.draw_instance(n, m, k, d, sig, 41)
    y = D.measure(inst.A_cols, inst.x_dense(), inst.eta, m)
    if shift:
        scale = np.float32(2.0 ** -shift)
        y = y * scale
        sig *= float(scale)
    w = np.zeros(M.n_params(d), np.float32)
    w[-2] = -1e4
    wt = dev(w)
    xg, stg = R.decode(dev(inst.A_cols), dev(y), sigma=sig, k=k, mlp=wt)
    C = D.make_constants(n, m, d, k, sig)
    ref = D.decode(inst.A_cols, y, C)
    assert np.array_equal(host(xg), ref.x_hat)
    assert stg["l1_final_fx"] == ref.L_hat and stg["accepted"] == ref.accepted
    *_, inexact = M.learned_decode(inst.A_cols, y, C, w, count_inexact=True)
    assert stg["fx_inexact_x"] == inexact == ref.fx_inexact_x
    assert inexact > 0 or not shift


def test_training_lowers_the_loss():
    from paper_1704_09012_amd import learned as Lrn
    F, Y = Lrn.trajectories(6, 3)
    print("samples", F.shape[0], "positives", int(Y[:, 0].sum()), flush=True)
    w0 = R.mlp_init(7, 5)
    _, l0 = R.mlp_grad(F, Y, w0)
    w, l1 = Lrn.train(F, Y, epochs=30, batch=256, w=w0.clone())
    _, l2 = R.mlp_grad(F, Y, w)
    print("loss before", l0, "after", l2, flush=True)
    assert l2 < 0.7 * l0


def test_trained_network_gain_over_the_analytic_rule():
    """Train on trajectories of the n = 1024 workload (2000 decodes, SNR in [20, 60] dB;
    the training is deterministic) and decode 12 unseen n = 2^17 instances at each of 20,
    40 and 60 dB with and without the network.

    What it gains: at 20 and 40 dB it reaches the paper's stopping condition
    (||r||_1 <= m sigma sqrt(2/pi)) on 24 of 24 instances against 5 of 24 for the analytic
    rule; the test requires a lead of at least 12.  What it loses: at 60 dB the analytic
    rule stops on 12 of 12 and the learned one on 2, and the learned relative error is a
    little larger at every SNR (0.095 against 0.088 at worst at 20 dB, 0.0062 against
    0.0055 at 40 dB, 5.7e-4 against 4.7e-4 at 60 dB); the test holds both to the error
    bars 0.15, 1e-2 and 1e-3."""
    from paper_1704_09012_amd import learned as Lrn
    F, Y = Lrn.trajectories(2000, 1)
    w, loss = Lrn.train(F, Y, epochs=30)
    n = 2 ** 17
    m, k = n // 10, n // 100
    conv = {snr: {"analytic": 0, "learned": 0} for snr in (20, 40, 60)}
    bar = {20: 0.15, 40: 1e-2, 60: 1e-3}
    for snr in (20, 40, 60):
        rows = Lrn.compare(w, n, m, k, snr, range(70000, 70012))
        for r in rows:
            print(snr, r["seed"], {t: (round(r[t]["rel_err"], 5), r[t]["iterations"], r[t]["converged"])
                                  for t in ("analytic", "learned")}, flush=True)
            for t in ("analytic", "learned"):
                conv[snr][t] += r[t]["converged"]
                assert r[t]["rel_err"] < bar[snr], (snr, r["seed"], t)
    print("converged (of 12 per SNR):", conv, "train loss", loss, flush=True)
    lead = sum(conv[s]["learned"] - conv[s]["analytic"] for s in (20, 40))
    assert lead >= 12, conv


def median_net(d, sigma, bias):
    """A hand-set network: value = the median residual of the column, logit =
    s|r_med| (2 Phi(s r_med) - 1) - bias with s = 1/sigma.  Hidden units come in pairs
    gelu(u), gelu(-u), whose difference is u, so the value survives both layers."""
    w = np.zeros(M.n_params(d), np.float32)
    W1, b1, W2, b2, W3, b3 = M.unpack(w, d)
    s = 1.0 / sigma
    mid = d // 2
    W1[0, mid], W1[1, mid] = s, -s
    W2[0, 0], W2[0, 1] = 1.0, -1.0
    W2[1, 0], W2[1, 1] = -1.0, 1.0
    W3[0, 0], W3[0, 1] = 1.0, 1.0
    b3[0] = -bias
    W3[1, 0], W3[1, 1] = 1.0 / s, -1.0 / s
    return w


def stepwise_learned(A, y, n, m, d, k, sig, wt):
    """The learned loop through rl0_step: at each t a learned iteration, then the
    analytic one at the same t when it is not accepted."""
    pa = R.params_default(n, m, d, k, sig)
    pl = R.params_default(n, m, d, k, sig, mlp=wt)
    C = R.compute_constants(pa, n, m, d)
    tol = C.tol * 2.0 ** 30
    x = torch.zeros(n, dtype=torch.float32, device="cuda")
    r = torch.empty(m, dtype=torch.float32, device="cuda")
    L = None
    iters = acc = learned_acc = retries = 0
    for it in range(C.n_iters):
        if L is not None and L <= tol:
            break
        out = R.step(A, y, pl, it, x, r, 0, debug=False)
        iters += 1
        L = out["L_hat"]
        if out["accepted"]:
            acc += 1
            learned_acc += 1
            continue
        out = R.step(A, y, pa, it, x, r, 0, debug=False)
        iters += 1
        retries += 1
        L = out["L_hat"]
        acc += int(out["accepted"])
    return host(x), L, iters, acc, learned_acc, retries


@pytest.mark.parametrize("n,m,k,snr,seed", [
    (8192, 2048, 160, 40, 51), (20000, 3000, 250, 25, 52),
    # m above 393216: the 8-row bitmask summary, H_k's classification kernel and the
    # dense-capable sweep instance (whose dense mode the learned branch never takes)
    (200000, 400003, 20000, 30, 53),
])
def test_device_learned_decode_matches_the_stepwise_loop(n, m, k, snr, seed):
    d = 7
    sig = float(np.float32(I.sigma_for_snr(snr, n, m, k, d)))
    inst = I.draw_instance(n, m, k, d, sig, seed)
    y = D.measure(inst.A_cols, inst.x_dense(), inst.eta, m)
    A, yt = dev(inst.A_cols), dev(y)
    wt = dev(median_net(d, sig, 1.5))
    xe, Le, ie, ae, la, rt = stepwise_learned(A, yt, n, m, d, k, sig, wt)
    print(f"n={n}: iterations {ie}, accepted {ae} (learned {la}), retries {rt}", flush=True)
    assert la > 0 and rt > 0          # both branches of the schedule ran
    for _ in range(2):                # captured, then replayed
        xg, st = R.decode(A, yt, sigma=sig, k=k, mlp=wt)
        assert np.array_equal(host(xg), xe)
        assert st["l1_final_fx"] == Le and st["iterations"] == ie and st["accepted"] == ae


def test_adam_update_matches_the_oracle():
    """rl0_mlp_adam (the update rl0_mlp_train applies) against oracle.mlp.adam_step over
    three steps with given gradients.  The device computes in float32, the oracle in fp64;
    the bar on m and v is a few float32 roundings of the terms of each update (b1 m and
    (1 - b1) g can cancel), carried over the steps, and on w its float32 rounding plus
    the step's share of the error in m."""
    d = 7
    P = M.n_params(d)
    rng = np.random.default_rng(61)
    w = net(d, 61)
    m = np.zeros(P, np.float32)
    v = np.zeros(P, np.float32)
    wt, mt, vt = dev(w), dev(m), dev(v)
    wo, mo, vo = w.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    # the settings cross the C-ABI as float32: the oracle takes the same values
    hp = {k: float(np.float32(x)) for k, x in dict(lr=1e-3, b1=0.9, b2=0.999, eps=1e-8).items()}
    b1, b2, lr = hp["b1"], hp["b2"], hp["lr"]
    u = 2.0 ** -24
    em = np.zeros(P)
    ev = np.zeros(P)
    ew = np.zeros(P)
    for t in (1, 2, 3):
        g = (rng.normal(0, 1, P) * 10.0 ** rng.uniform(-4, 0, P)).astype(np.float32).astype(np.float64)
        em = b1 * em + 4 * u * (b1 * np.abs(mo) + (1 - b1) * np.abs(g))
        ev = b2 * ev + 4 * u * (b2 * vo + (1 - b2) * g * g)
        R.mlp_adam(wt, dev(g.astype(np.float32)), mt, vt, d, t, lr=1e-3)
        wo, mo, vo = M.adam_step(wo, g, mo, vo, t, **hp)
        c1, c2 = 1 - b1 ** t, 1 - b2 ** t
        den = np.sqrt(vo / c2) + hp["eps"]
        step = lr * np.abs(mo) / c1 / den
        ew = ew + 2 * u * np.abs(wo) + lr * (em / c1) / den + step * (8 * u + 0.5 * ev / np.maximum(vo, 1e-300))
        gw, gm, gv = host(wt), host(mt), host(vt)
        assert np.all(np.abs(gm - mo) <= em), t
        assert np.all(np.abs(gv - vo) <= ev), t
        assert np.all(np.abs(gw - wo) <= ew), t


def test_training_steps_match_the_oracle():
    """Three rl0_mlp_train steps (fp32 gradient, then Adam) against the fp64 oracle's
    gradient and adam_step.  Where the oracle's gradient component is not small against
    the largest one (the fp32 gradient is within 1e-4 of that largest component), the
    steps are settled and the weights agree to 2e-2 of the learning rate; elsewhere (a
    sign that fp32 rounding can flip) within the 2 lr a step can move."""
    d, N, lr = 7, 4096, 1e-3
    rng = np.random.default_rng(62)
    w = net(d, 62)
    F = rng.normal(0, 0.3, (3 * N, d + 1)).astype(np.float32)
    Y = np.stack([(rng.random(3 * N) < 0.3).astype(np.float32), rng.normal(0, 1, 3 * N).astype(np.float32)], 1)
    P = M.n_params(d)
    wt, mt, vt = dev(w), torch.zeros(P, device="cuda"), torch.zeros(P, device="cuda")
    R.mlp_train(dev(F), dev(Y), wt, mt, vt, steps=3, lr=lr, batch=N)
    wo, mo, vo = w.astype(np.float64), np.zeros(P), np.zeros(P)
    hp = {k: float(np.float32(x)) for k, x in dict(lr=lr, b1=0.9, b2=0.999, eps=1e-8).items()}
    settled = np.ones(P, bool)
    for t in (1, 2, 3):
        _, g = M.loss_and_grad(wo, F[(t - 1) * N:t * N], Y[(t - 1) * N:t * N], d, lam=1.0)
        settled &= np.abs(g) > 0.05 * np.max(np.abs(g))
        wo, mo, vo = M.adam_step(wo, g, mo, vo, t, **hp)
    gw = host(wt)
    print("settled components", int(settled.sum()), "of", P, flush=True)
    assert settled.sum() >= 20
    assert np.max(np.abs(gw - wo)[settled]) <= 2e-2 * lr
    assert np.max(np.abs(gw - wo)) <= 2 * lr * 3


def test_checkpoint_resume_is_exact(tmp_path):
    """rl0_mlp_save after 7 Adam steps, rl0_mlp_load into new arrays and 5 more steps from
    the stored step and hyper-parameters give, bit for bit, the weights and moments of 12
    uninterrupted steps (the batch order and the bias corrections depend on the step only,
    and the gradient sum has a fixed order).  The loaded arrays equal the saved ones, the
    file's payload is their bytes and its CRC-32 is zlib's."""
    import struct
    import zlib

    d, B = 7, 512
    N = 5 * B + 100                       # five blocks and a remainder no step takes
    rng = np.random.default_rng(81)
    F = dev(rng.normal(0, 0.3, (N, d + 1)).astype(np.float32))
    Y = dev(np.stack([(rng.random(N) < 0.3).astype(np.float32), rng.normal(0, 1, N).astype(np.float32)], 1))
    hp = dict(lr=2e-3, beta1=0.9, beta2=0.99, eps=1e-7, lam=0.5, batch=B)

    def fresh():
        w = R.mlp_init(d, 4)
        return w, torch.zeros_like(w), torch.zeros_like(w)

    w1, m1, v1 = fresh()
    R.mlp_train(F, Y, w1, m1, v1, steps=12, t0=0, **hp)
    w2, m2, v2 = fresh()
    R.mlp_train(F, Y, w2, m2, v2, steps=7, t0=0, **hp)
    path = str(tmp_path / "mlp.ckpt")
    R.mlp_save(path, w2, m2, v2, d, step=7, seed=4, **hp)
    info, w3, m3, v3 = R.mlp_load(path)
    assert torch.equal(w3, w2) and torch.equal(m3, m2) and torch.equal(v3, v2)
    blob = open(path, "rb").read()
    assert blob[80:] == host(w2).tobytes() + host(m2).tobytes() + host(v2).tobytes()
    assert struct.unpack_from("<I", blob, 68)[0] == zlib.crc32(blob[80:])
    cfg = info["cfg"]
    assert info["step"] == 7 and cfg["t0"] == 7 and info["seed"] == 4 and info["d"] == d
    R.mlp_train(F, Y, w3, m3, v3, steps=5, t0=cfg["t0"], lr=cfg["lr"], beta1=cfg["beta1"], beta2=cfg["beta2"],
                eps=cfg["eps"], lam=cfg["lam"], batch=cfg["batch"])
    assert torch.equal(w3, w1) and torch.equal(m3, m1) and torch.equal(v3, v1)
    # a later save replaces the file whole; the weights alone can be read back
    R.mlp_save(path, w3, m3, v3, d, step=12, seed=4, **hp)
    info, w4, m4, v4 = R.mlp_load(path, moments=False)
    assert info["step"] == 12 and m4 is None and v4 is None and torch.equal(w4, w1)
    assert not (tmp_path / "mlp.ckpt.tmp").exists()


def exact_net(d, sigma):
    """A hand-set network whose every output that a decision lets through is the same,
    bit for bit, in the oracle's bf16 emulation and on the matrix cores, whatever their
    accumulation order.  s = 1/sigma is a power of two and f = bf16 of the column's median
    residual (feature d // 2):
      layer 1: u0 = s f - 8, u1 = -s f - 8, u2 = s f, u3 = -s f
      layer 2: v_i = gelu(u_i) + 16, i < 4
      layer 3: logit = v0 + v1 - 48, value = (v2 - v3) / s
    A column updates when logit >= log(t / (1 - t)) >= -3.67, which needs s|f| >= 20.3.
    Every GELU input is then >= 12 in magnitude, where both GELUs give u or 0 to float32
    precision, so the outputs are sums of bf16 numbers times dyadic weights, exact in fp32.
    Where s|f| < 16 the logit is below -7.9, far from every threshold."""
    w = np.zeros(M.n_params(d), np.float32)
    W1, b1, W2, b2, W3, b3 = M.unpack(w, d)
    s = np.float32(1.0 / sigma)
    mid = d // 2
    W1[0, mid], b1[0] = s, -8.0
    W1[1, mid], b1[1] = -s, -8.0
    W1[2, mid] = s
    W1[3, mid] = -s
    for i in range(4):
        W2[i, i], b2[i] = 1.0, 16.0
    W3[0, 0], W3[0, 1], b3[0] = 1.0, 1.0, -48.0
    W3[1, 2], W3[1, 3] = 1.0 / s, -1.0 / s
    return w


@pytest.mark.parametrize("n,m,k,seed", [(4096, 1024, 80, 71), (8192, 2048, 160, 72)])
def test_device_learned_decode_matches_the_oracle(n, m, k, seed):
    """The whole learned decode (Alg. 1 with the learned decision, the analytic retry at
    the same t when a learned iteration is not accepted) on the device against
    oracle.mlp.learned_decode, bitwise, with the exactly evaluated network above."""
    d = 7
    sig = 2.0 ** -7
    inst = I.draw_instance(n, m, k, d, sig, seed)
    y = D.measure(inst.A_cols, inst.x_dense(), inst.eta, m)
    w = exact_net(d, sig)
    C = D.make_constants(n, m, d, k, sig)
    xo, io, ao, Lo, inx = M.learned_decode(inst.A_cols, y, C, w, count_inexact=True)
    xg, st = R.decode(dev(inst.A_cols), dev(y), sigma=sig, k=k, mlp=dev(w))
    print(f"n={n}: oracle iterations {io}, accepted {ao}; gpu {st['iterations']}, {st['accepted']}", flush=True)
    assert ao > 0
    assert np.array_equal(host(xg), xo)
    assert st["iterations"] == io and st["accepted"] == ao and st["l1_final_fx"] == Lo
    assert st["fx_inexact_x"] == inx
