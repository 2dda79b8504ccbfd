"""Training the learned column decision on the decoder's own trajectories.

Every numerical step runs in librl0 on the GPU: the decodes that produce the
trajectories (rl0_step), the features and labels (rl0_mlp_features, rl0_mlp_labels)
and the training (rl0_mlp_train: fp32 forward, backward and Adam kernels).  This module
only draws the synthetic instances, picks which samples to keep, and shuffles them.

Samples: the analytic decoder is run on instances of GM(n, m, k, d, N(0,1), N(0, s^2))
with the SNR drawn uniformly; at every iteration it >= 1 (iteration 0 cannot update) the
state before the sweep gives one sample per column: the features of the column on the
residual r_hat and the labels from the true signal and x_hat.  All positives are kept and
`neg_per_pos` negatives per positive are drawn at random.
"""
from __future__ import annotations

import numpy as np

from . import instances as I
from . import rl0 as R


def _torch():
    import torch
    return torch


def trajectories(count: int, seed: int, n: int = 1024, m: int = 256, k: int = 25, d: int = 7,
                 snr_db=(20.0, 60.0), neg_per_pos: int = 4, device: str = "cuda"):
    """(features [N][d+1], labels [N][2]) device tensors from `count` analytic decodes."""
    torch = _torch()
    rng = np.random.Generator(np.random.PCG64(seed))
    feats, labs = [], []
    for i in range(count):
        snr = float(rng.uniform(*snr_db))
        sig = float(np.float32(I.sigma_for_snr(snr, n, m, k, d)))
        inst = I.draw_instance(n, m, k, d, sig, seed * 1000003 + i)
        A = torch.from_numpy(inst.A_cols).to(device)
        x = torch.from_numpy(inst.x_dense()).to(device)
        y = R.sketch(A, x, m) + torch.from_numpy(inst.eta).to(device)
        params = R.params_default(n, m, d, k, sig)
        C = R.compute_constants(params, n, m, d)
        x_hat = torch.zeros(n, dtype=torch.float32, device=device)
        r_hat = torch.empty(m, dtype=torch.float32, device=device)
        st = R.step(A, y, params, 0, x_hat, r_hat, 0, debug=False)   # iteration 0: r_hat of x_hat = 0
        L = st["L_hat"]
        tol = C.tol * 2.0 ** 30
        for it in range(1, C.n_iters):
            if L <= tol:
                break
            f = R.mlp_features(A, r_hat, sig)
            lab = R.mlp_labels(x, x_hat, d, sig)
            pos = torch.nonzero(lab[:, 0] > 0.5).flatten()
            neg = torch.nonzero(lab[:, 0] <= 0.5).flatten()
            take = min(neg.numel(), neg_per_pos * max(int(pos.numel()), 1))
            pick = torch.from_numpy(rng.choice(neg.numel(), take, replace=False)).to(device)
            idx = torch.cat([pos, neg[pick]])
            feats.append(f[idx])
            labs.append(lab[idx])
            st = R.step(A, y, params, it, x_hat, r_hat, L, debug=False)
            L = st["L_hat"]
    F = torch.cat(feats)
    Y = torch.cat(labs)
    perm = torch.from_numpy(rng.permutation(F.shape[0])).to(device)
    return F[perm].contiguous(), Y[perm].contiguous()


def train(F, Y, d: int = 7, epochs: int = 4, batch: int = 4096, lr: float = 1e-3, seed: int = 0, w=None):
    """Adam on (F, Y) for `epochs` passes; returns (weights, loss of the last steps)."""
    torch = _torch()
    if w is None:
        w = R.mlp_init(d, seed, device=F.device)
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    batch = min(batch, F.shape[0])
    steps = max(1, epochs * (F.shape[0] // batch))
    loss = R.mlp_train(F, Y, w, m, v, steps, 0, lr=lr, batch=batch)
    return w, loss


def compare(w, n: int, m: int, k: int, snr_db: float, seeds, d: int = 7, device: str = "cuda") -> list[dict]:
    """Decode each seeded instance of GM(n, m, k, d) at the given SNR with the analytic
    decision and with the learned one (w); per instance: relative l2 errors, iterations
    executed and accepted, and the wall time of each decode (inputs already on the GPU)."""
    import time

    torch = _torch()
    out = []
    for seed in seeds:
        sig = float(np.float32(I.sigma_for_snr(snr_db, n, m, k, d)))
        inst = I.draw_instance(n, m, k, d, sig, seed)
        A = torch.from_numpy(inst.A_cols).to(device)
        x = torch.from_numpy(inst.x_dense()).to(device)
        y = R.sketch(A, x, m) + torch.from_numpy(inst.eta).to(device)
        row = {"seed": seed, "sigma": sig}
        for tag, kw in (("analytic", {}), ("learned", {"mlp": w})):
            R.decode(A, y, sigma=sig, k=k, **kw)       # warm (constants, graphs)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xh, st = R.decode(A, y, sigma=sig, k=k, **kw)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0)
            row[tag] = {"rel_err": float(torch.linalg.norm(xh - x) / torch.linalg.norm(x)),
                        "iterations": st["iterations"], "accepted": st["accepted"],
                        "converged": st["converged"], "ms": ms}
        out.append(row)
    return out
