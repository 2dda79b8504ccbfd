"""Phase transitions of Robust-l0 (Sec. 4, "Phase transitions and runtime", "Dependence on
noise variance" and "Phase transitions for extreme subsampling").

For a fixed delta = m/n the phase transition rho*(delta) is the largest k/m at which the
decoder typically recovers x.  The paper finds it with a ladder: start at rho = 0.01, draw
`trials` instances of GM(n, m, k, d, N(0,1), N(0, sigma^2)) (k = rho m), decode them, and
while at least one is recovered raise rho by 0.01; the recovery fractions are then fitted
with a logistic curve in rho, whose 50% point is rho*.

Recovery is the success condition eq:success_condition_clip with C_1 = 1:
    ||x - x_hat||_1 / ||x||_1 <= min((E||eta||_1 + C_1 sqrt(Var||eta||_1)) / ||x||_1, 1/10),
with E||eta||_1 = m sigma sqrt(2/pi) and Var||eta||_1 = m sigma^2 (1 - 2/pi) (Sec. 4).

The decodes run in librl0 (rl0_decode, or rl0_decode_batched for many small instances);
this module draws the instances on the device, evaluates the success condition on the
host and fits the curve.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import instances as I

__all__ = ["success", "logistic_fit", "LadderResult", "ladder", "gpu_trials"]


def success(x: np.ndarray, x_hat: np.ndarray, m: int, sigma: float, C1: float = 1.0) -> bool:
    """eq:success_condition_clip for one decode (x, x_hat as float arrays)."""
    x = np.asarray(x, dtype=np.float64)
    e = np.asarray(x_hat, dtype=np.float64) - x
    l1x = float(np.abs(x).sum())
    if l1x == 0.0:
        return float(np.abs(e).sum()) == 0.0
    mean = m * sigma * math.sqrt(2.0 / math.pi)
    var = m * sigma * sigma * (1.0 - 2.0 / math.pi)
    bound = min((mean + C1 * math.sqrt(var)) / l1x, 0.1)
    return float(np.abs(e).sum()) / l1x <= bound


def logistic_fit(rhos, succ, trials, iters: int = 200):
    """Maximum-likelihood fit of P(success | rho) = 1 / (1 + exp(b (rho - rho50))) to the
    counts succ[i] of trials[i] at rhos[i] (Newton's method on (rho50, b) with b > 0);
    returns (rho50, b).  With no transition in the data (all or none recovered) it
    returns the edge of the grid and b = inf."""
    r = np.asarray(rhos, dtype=np.float64)
    s = np.asarray(succ, dtype=np.float64)
    t = np.asarray(trials, dtype=np.float64)
    if s.sum() == 0:
        return float(r.min()), math.inf
    if np.all(s == t):
        return float(r.max()), math.inf
    # in the form 1 / (1 + exp(-(a0 + a1 rho))), a1 < 0 for a falling curve
    a = np.array([0.0, 0.0])
    frac = (s + 0.5) / (t + 1.0)
    # start from a least-squares fit of the logits
    A = np.stack([np.ones_like(r), r], axis=1)
    a = np.linalg.lstsq(A, np.log(frac / (1.0 - frac)), rcond=None)[0]
    for _ in range(iters):
        z = np.clip(A @ a, -40, 40)
        p = 1.0 / (1.0 + np.exp(-z))
        g = A.T @ (s - t * p)
        H = -(A * (t * p * (1 - p))[:, None]).T @ A - 1e-9 * np.eye(2)
        step = np.linalg.solve(H, g)
        a = a - step
        if np.max(np.abs(step)) < 1e-12:
            break
    if a[1] >= 0:
        return float("nan"), float("nan")
    return float(-a[0] / a[1]), float(-a[1])


@dataclass
class LadderResult:
    n: int
    delta: float
    sigma: float
    variant: int
    rhos: list = field(default_factory=list)
    succ: list = field(default_factory=list)
    trials: list = field(default_factory=list)
    ms_mean: list = field(default_factory=list)    # mean decode time of the recovered ones
    rho50: float = float("nan")
    width: float = float("nan")                    # 1 / b of the fitted logistic
    rho_half: float = float("nan")                 # largest rho with >= 50% recovered

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k in ("n", "delta", "sigma", "variant", "rhos", "succ", "trials",
                                               "ms_mean", "rho50", "width", "rho_half")}


def ladder(run_trials, n: int, delta: float, sigma: float, variant: int = 0, trials: int = 10,
           rho0: float = 0.01, step: float = 0.01, rho_max: float = 0.6, seed: int = 0) -> LadderResult:
    """The paper's ladder.  run_trials(n, m, k, sigma, variant, trials, seed) returns a
    list of (recovered, ms) per trial."""
    m = max(2, int(round(delta * n)))
    res = LadderResult(n=n, delta=delta, sigma=sigma, variant=variant)
    level = 0
    while True:
        rho = round(rho0 + level * step, 10)
        if rho > rho_max:
            break
        k = max(1, min(m - 1, int(round(rho * m))))
        out = run_trials(n, m, k, sigma, variant, trials, seed + 1000 * level)
        ok = [o for o in out if o[0]]
        res.rhos.append(rho)
        res.succ.append(len(ok))
        res.trials.append(len(out))
        res.ms_mean.append(float(np.mean([o[1] for o in ok])) if ok else float("nan"))
        if not ok:
            break
        level += 1
    res.rho50, b = logistic_fit(res.rhos, res.succ, res.trials)
    res.width = 1.0 / b if b and math.isfinite(b) else 0.0
    half = [r for r, s, t in zip(res.rhos, res.succ, res.trials) if 2 * s >= t]
    res.rho_half = max(half) if half else float("nan")
    return res


def gpu_trials(n: int, m: int, k: int, sigma: float, variant: int, trials: int, seed: int, d: int = 7,
               batched: bool | None = None):
    """run_trials for ladder(): `trials` instances drawn on the device and decoded by librl0
    (one batched launch for small instances, else one rl0_decode each); returns
    [(recovered, decode ms)]."""
    import torch
    from . import rl0 as R

    if batched is None:
        batched = n <= 2 ** 18 and m <= R.RL0_BATCH_MAX_M
    sig = float(np.float32(sigma))
    probs, xs = [], []
    for i in range(trials):
        A, x, eta = I.draw_instance_device(n, m, k, d, sig, seed * 7919 + i)
        y = R.sketch(A, x, m) + eta
        probs.append({"A": A, "y": y.contiguous(), "sigma": sig, "k": k, "variant": variant})
        xs.append(x)
    out = []
    if batched:
        stats = R.decode_batched(probs)
        for p, x, st in zip(probs, xs, stats):
            out.append((success(x.cpu().numpy(), p["out"].cpu().numpy(), m, sig), st["ms_total"]))
    else:
        xh = torch.empty(n, dtype=torch.float32, device="cuda")
        for p, x in zip(probs, xs):
            _, st = R.decode(p["A"], p["y"], sigma=sig, k=k, variant=variant, out=xh)
            out.append((success(x.cpu().numpy(), xh.cpu().numpy(), m, sig), st["ms_total"]))
    return out
