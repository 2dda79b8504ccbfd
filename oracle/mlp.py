"""The learned column decision: features, network, loss, gradients, Adam, in fp64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's decision for column j (Alg. 1, inner loop) is built from the approximate
posteriors p_z, p_e (Sec. 3).  The learned variant replaces that decision by a small
network of the column's residual neighbourhood; everything else in the iteration (H_k,
the residual, the acceptance test) is unchanged.  Nothing here is in the paper; it is
the contract the HIP kernels are checked against:

  features   f_j = [sort_ascending(r_{i_1}, ..., r_{i_d}), sigma_n]     (d + 1 values)
  network    z1 = W1 f + b1,  h1 = gelu(z1)          (64)
             z2 = W2 h1 + b2, h2 = gelu(z2)          (64)
             o  = W3 h2 + b3 = (logit, value)        (2)
             gelu(u) = u/2 (1 + erf(u / sqrt 2))     (the exact form)
  decision   column j updates iff logit >= logit_t = log(t / (1 - t)) (i.e. the
             predicted acceptance probability sigmoid(logit) reaches t; t = 1 gives
             +inf: nothing updates, as in the analytic loop); x'_j = x_hat_j + value
  labels     y_acc = 1 iff j in supp(x) and |x_j - x_hat_j| > 3 sigma_n / sqrt(d);
             y_val = x_j - x_hat_j
  loss       mean over the batch of  BCE(logit, y_acc) + lam * (value - y_val)^2
             (the value is fitted on every sample, so that a column the decision lets
             through by mistake moves by about its true error, usually about 0)
  optimiser  Adam (Kingma and Ba): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
             w <- w - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)

Parameter layout (one flat vector, 4866 values for d = 7): W1 [64][d+1], b1 [64],
W2 [64][64], b2 [64], W3 [2][64], b3 [2].

bf16 inference (the decoder's matrix cores): weights and the inputs of each of the
three products are rounded to bfloat16 (round to nearest, ties to even); products are
accumulated in fp32; biases, GELU and the decision stay fp32.
"""
from __future__ import annotations

import math

import numpy as np

from . import decoder as _dec
from . import scores as _scores

__all__ = [
    "HIDDEN",
    "n_params",
    "unpack",
    "features",
    "labels",
    "gelu",
    "gelu_grad",
    "forward",
    "loss_and_grad",
    "adam_step",
    "to_bf16",
    "forward_bf16",
    "logit_threshold",
    "init_params",
    "learned_sweep",
    "learned_step",
    "learned_decode",
]

HIDDEN = 64


def n_params(d: int) -> int:
    f = d + 1
    return HIDDEN * f + HIDDEN + HIDDEN * HIDDEN + HIDDEN + 2 * HIDDEN + 2


def unpack(w: np.ndarray, d: int):
    """Views (W1, b1, W2, b2, W3, b3) of the flat parameter vector."""
    f = d + 1
    o = 0
    out = []
    for shape in ((HIDDEN, f), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (2, HIDDEN), (2,)):
        size = int(np.prod(shape))
        out.append(w[o:o + size].reshape(shape))
        o += size
    assert o == w.size
    return out


def features(A_cols: np.ndarray, r: np.ndarray, sigma: float) -> np.ndarray:
    """[n][d+1] float32: the column's residual entries sorted ascending, then sigma_n."""
    v = r[A_cols.astype(np.int64)]
    out = np.empty((A_cols.shape[0], A_cols.shape[1] + 1), dtype=np.float32)
    out[:, :-1] = np.sort(v, axis=1)
    out[:, -1] = np.float32(sigma)
    return out


def labels(x_true: np.ndarray, x_hat: np.ndarray, sigma: float, d: int) -> np.ndarray:
    """[n][2] float32: (y_acc, y_val).  The threshold 3 sigma_n / sqrt(d) is evaluated in
    fp64 and compared with |x_j - x_hat_j| computed in float32."""
    diff = (x_true.astype(np.float32) - x_hat.astype(np.float32)).astype(np.float32)
    thr = 3.0 * float(sigma) / math.sqrt(d)
    acc = (x_true != 0) & (np.abs(diff).astype(np.float64) > thr)
    return np.stack([acc.astype(np.float32), diff], axis=1)


def gelu(u):
    """The exact GELU, u Phi(u), in fp64."""
    return _gelu(np.asarray(u, dtype=np.float64))


def _erf(u: np.ndarray) -> np.ndarray:
    return np.vectorize(math.erf, otypes=[np.float64])(u)


def _gelu(u: np.ndarray) -> np.ndarray:
    return 0.5 * u * (1.0 + _erf(u / math.sqrt(2.0)))


def gelu_grad(u):
    """d/du of u Phi(u): Phi(u) + u phi(u)."""
    u = np.asarray(u, dtype=np.float64)
    return 0.5 * (1.0 + _erf(u / math.sqrt(2.0))) + u * np.exp(-0.5 * u * u) / math.sqrt(2.0 * math.pi)


def forward(w: np.ndarray, F: np.ndarray, d: int):
    """fp64 forward pass on [N][d+1] features; returns (out [N][2], cache)."""
    W1, b1, W2, b2, W3, b3 = (a.astype(np.float64) for a in unpack(np.asarray(w, np.float64), d))
    F = F.astype(np.float64)
    z1 = F @ W1.T + b1
    h1 = _gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = _gelu(z2)
    out = h2 @ W3.T + b3
    return out, (F, z1, h1, z2, h2)


def _bce_with_logits(s: np.ndarray, y: np.ndarray) -> np.ndarray:
    # log(1 + e^s) - y s, written to stay finite for large |s|
    return np.maximum(s, 0.0) - y * s + np.log1p(np.exp(-np.abs(s)))


def loss_and_grad(w: np.ndarray, F: np.ndarray, Y: np.ndarray, d: int, lam: float = 1.0):
    """Mean loss over the N samples and its gradient (flat, fp64), by backpropagation
    written out layer by layer."""
    w = np.asarray(w, dtype=np.float64)
    W1, b1, W2, b2, W3, b3 = unpack(w, d)
    out, (Fd, z1, h1, z2, h2) = forward(w, F, d)
    N = F.shape[0]
    s, val = out[:, 0], out[:, 1]
    ya, yv = Y[:, 0].astype(np.float64), Y[:, 1].astype(np.float64)
    loss = float(np.mean(_bce_with_logits(s, ya) + lam * (val - yv) ** 2))
    dout = np.empty_like(out)
    dout[:, 0] = (1.0 / (1.0 + np.exp(-s)) - ya) / N
    dout[:, 1] = 2.0 * lam * (val - yv) / N
    gW3 = dout.T @ h2
    gb3 = dout.sum(axis=0)
    dz2 = (dout @ W3) * gelu_grad(z2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * gelu_grad(z1)
    gW1 = dz1.T @ Fd
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def adam_step(w, g, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t >= 1 (fp64); returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def to_bf16(a) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float32."""
    x = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).copy()
    nan = np.isnan(x)
    out[nan] = x[nan]
    return out


def forward_bf16(w: np.ndarray, F: np.ndarray, d: int) -> np.ndarray:
    """The decoder's inference: bf16 operands of every product, fp32 accumulation
    (here exact in fp64, then rounded to fp32), fp32 bias and GELU."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(w, dtype=np.float32), d)

    def layer(X, W, b):
        acc = to_bf16(X).astype(np.float64) @ to_bf16(W).astype(np.float64).T
        return (acc.astype(np.float32) + b.astype(np.float32)).astype(np.float32)

    def g32(u):
        return _gelu(u.astype(np.float64)).astype(np.float32)

    h1 = g32(layer(F.astype(np.float32), W1, b1))
    h2 = g32(layer(h1, W2, b2))
    return layer(h2, W3, b3)


def logit_threshold(t: float) -> float:
    """fl32(log(t / (1 - t))): sigmoid(logit) >= t iff logit >= this (t in (0, 1]);
    +inf at t = 1."""
    if t >= 1.0:
        return float("inf")
    return float(np.float32(math.log(t / (1.0 - t))))


def init_params(d: int, seed: int) -> np.ndarray:
    """Weights uniform in +-sqrt(3 / fan_in) (Kaiming-uniform with unit gain) and zero
    biases, float32, drawn from numpy PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f = d + 1
    parts = []
    for fan_out, fan_in in ((HIDDEN, f), (HIDDEN, HIDDEN), (2, HIDDEN)):
        bound = math.sqrt(3.0 / fan_in)
        parts.append(rng.uniform(-bound, bound, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


# ----------------------------------------------------------------------------- the loop

def learned_sweep(A_cols, r_hat, x_hat, t: float, sigma: float, w: np.ndarray):
    """The column loop with the learned decision on the snapshot r_hat: returns
    (x_prime, updated, value, logit) with the network evaluated as the decoder does
    (bf16 operands, fp32 accumulation)."""
    A_cols = np.asarray(A_cols)
    d = A_cols.shape[1]
    out = forward_bf16(w, features(A_cols, np.asarray(r_hat, np.float32), sigma), d)
    logit, value = out[:, 0], out[:, 1]
    upd = logit >= np.float32(logit_threshold(float(t)))
    x_prime = np.asarray(x_hat, dtype=np.float32).copy()
    x_prime[upd] = (x_prime[upd] + value[upd]).astype(np.float32)
    return x_prime, upd, value, logit


def learned_step(A_cols, y_hat, state, C, w: np.ndarray):
    """One iteration at t = t_of(state.it) with the learned decision; H_k, the residual
    and the acceptance test as in the analytic step.  Returns (new state, accepted,
    updated mask, value, logit, x_prime)."""
    t = _scores.t_of(state.it, C.c)
    x_prime, upd, value, logit = learned_sweep(A_cols, state.r_hat, state.x_hat, t, C.sigma, w)
    x_trial = _dec.hard_threshold(x_prime, C.k)
    r_trial = _dec.residual(A_cols, y_hat, x_trial, C.m)
    L_trial = _dec.l1_fixed(r_trial)
    if L_trial < state.L_hat:
        new = _dec.State(x_hat=x_trial, r_hat=r_trial, L_hat=L_trial, it=state.it + 1, accepted=state.accepted + 1)
        return new, True, upd, value, logit, x_prime
    new = _dec.State(x_hat=state.x_hat, r_hat=state.r_hat, L_hat=state.L_hat, it=state.it + 1,
                     accepted=state.accepted)
    return new, False, upd, value, logit, x_prime


def learned_decode(A_cols, y_hat, C, w: np.ndarray, count_inexact: bool = False):
    """At each t: a learned iteration, and if it is not accepted, the analytic one at the
    same t.  Returns (x_hat, iterations executed, accepted, L_hat); with count_inexact,
    also the number of updated x'_j != 0 whose 2^-40 fixed-point conversion rounds,
    summed over every executed sub-iteration (the decoder's fx_inexact_x)."""
    A_cols = np.asarray(A_cols)
    st = _dec.init_state(y_hat, A_cols.shape[0])
    iters = 0
    inexact_x = 0
    for it in range(C.n_iters):
        if _dec.converged(st, C):
            break
        st.it = it
        new, acc, upd, _, _, x_prime = learned_step(A_cols, y_hat, st, C, w)
        xp = x_prime[upd]
        inexact_x += _dec.fx_inexact(xp[xp != 0])
        iters += 1
        if not acc:
            st.it = it
            out = _dec.step(A_cols, y_hat, st, C)
            new = out.state
            xp = out.sweep.x_prime[out.sweep.updated]
            inexact_x += _dec.fx_inexact(xp[xp != 0])
            iters += 1
        st = new
    if count_inexact:
        return st.x_hat, iters, st.accepted, st.L_hat, inexact_x
    return st.x_hat, iters, st.accepted, st.L_hat
