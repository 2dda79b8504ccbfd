"""Seeded synthetic problem instances for the generating model GM(n, m, k, d, mu, nu).

The generating model (Definition "Generating model", Sec. 1 of the paper, and its
Figure 1) draws
  * each column support of A uniformly from the d-subsets of [m],
  * supp(x) uniformly from the k-subsets of [n],
  * x_j iid mu on the support, eta_i iid nu,
and measures y_hat = A x + eta.  Here mu = N(0, sigma_s^2) and nu = N(0, sigma_n^2)
as in the paper's experiments (Sec. 4, "Stopping conditions"), or Laplace laws of the
same standard deviations (scale b = s / sqrt(2)) for the general-distribution posteriors.

This module only draws random numbers.  It holds none of the decoder's arithmetic and
does not form the sketch A x: the oracle and the HIP library each form it themselves.
Both the CPU oracle and the GPU path consume the arrays it returns, so they see
identical bytes.

Layout of the returned expander: ``A_cols`` is int32 ``[n][d]``; row ``j`` lists the d
row indices of column j, distinct and ascending.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Instance",
    "draw_batch_shapes",
    "draw_batch",
    "sigma_for_snr",
    "draw_columns",
    "draw_signal",
    "draw_noise",
    "draw_instance",
    "draw_instance_device",
    "seed_for",
]


@dataclass
class Instance:
    n: int
    m: int
    k: int
    d: int
    sigma: float          # noise standard deviation sigma_n
    sigma_s: float        # signal standard deviation sigma_s
    A_cols: np.ndarray    # int32 [n][d], ascending distinct rows per column
    support: np.ndarray   # int64 [k], ascending
    values: np.ndarray    # float32 [k]
    eta: np.ndarray       # float32 [m]

    def x_dense(self) -> np.ndarray:
        x = np.zeros(self.n, dtype=np.float32)
        x[self.support] = self.values
        return x


def sigma_for_snr(snr_db: float, n: int, m: int, k: int, d: int, sigma_s: float = 1.0) -> float:
    """Noise std for a target SNR in dB.

    The paper parameterises noise by sigma directly.  A workload quoted as an SNR is
    mapped with the expected signal power per measurement, d*k/m * sigma_s^2 (each row
    of A x is a Poisson(d*rho) sum of N(0, sigma_s^2) entries, rho = k/m), divided by
    sigma_n^2.
    """
    return float(sigma_s * math.sqrt(d * k / m) * 10.0 ** (-snr_db / 20.0))


def seed_for(config: int, snr_idx: int, i: int) -> int:
    return 10000 * config + 100 * snr_idx + i


def draw_columns(rng: np.random.Generator, n: int, m: int, d: int) -> np.ndarray:
    """d distinct rows per column, uniform over the d-subsets of [m], sorted ascending.

    Each column draws d iid uniform rows; columns with a repeated row are redrawn whole,
    which leaves the accepted columns exactly uniform over the d-subsets.
    """
    if not (0 < d <= m):
        raise ValueError("need 0 < d <= m")
    cols = rng.integers(0, m, size=(n, d), dtype=np.int64)
    cols.sort(axis=1)
    bad = np.nonzero((np.diff(cols, axis=1) == 0).any(axis=1))[0] if d > 1 else np.zeros(0, np.int64)
    while bad.size:
        redraw = rng.integers(0, m, size=(bad.size, d), dtype=np.int64)
        redraw.sort(axis=1)
        cols[bad] = redraw
        still = (np.diff(redraw, axis=1) == 0).any(axis=1)
        bad = bad[still]
    return np.ascontiguousarray(cols.astype(np.int32))


def draw_signal(rng: np.random.Generator, n: int, k: int, sigma_s: float = 1.0,
                kind: str = "gaussian") -> tuple[np.ndarray, np.ndarray]:
    """Support uniform over the k-subsets of [n]; values iid N(0, sigma_s^2) in float32.

    ``kind="dyadic"`` draws instead nonzero integers in [-2^12, 2^12] times 2^-6 (exact in
    float32 and in any short float32 sum); such signals are dissociated with high
    probability and serve the noiseless exact-recovery checks.  ``kind="laplace"`` draws
    Laplace values of standard deviation sigma_s.
    """
    support = np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)
    if kind == "gaussian":
        values = rng.standard_normal(k, dtype=np.float32) * np.float32(sigma_s)
    elif kind == "laplace":
        values = rng.laplace(0.0, sigma_s / math.sqrt(2.0), size=k).astype(np.float32)
    elif kind == "dyadic":
        mag = rng.integers(1, 2 ** 12 + 1, size=k)
        sign = np.where(rng.integers(0, 2, size=k) == 1, 1, -1)
        values = (sign * mag).astype(np.float32) * np.float32(2.0 ** -6)
    else:
        raise ValueError(kind)
    return support, values.astype(np.float32)


def draw_noise(rng: np.random.Generator, m: int, sigma: float, kind: str = "gaussian") -> np.ndarray:
    """eta iid N(0, sigma^2), or Laplace of standard deviation sigma (kind="laplace")."""
    if sigma == 0.0:
        return np.zeros(m, dtype=np.float32)
    if kind == "laplace":
        return rng.laplace(0.0, sigma / math.sqrt(2.0), size=m).astype(np.float32)
    if kind != "gaussian":
        raise ValueError(kind)
    return (rng.standard_normal(m, dtype=np.float32) * np.float32(sigma)).astype(np.float32)


def draw_instance(n: int, m: int, k: int, d: int, sigma: float, seed: int,
                  sigma_s: float = 1.0, kind: str = "gaussian", noise_kind: str = "gaussian") -> Instance:
    """One seeded instance of GM(n, m, k, d, mu, nu): mu = N(0, sigma_s^2) (or the law of
    `kind`), nu = N(0, sigma^2) (or Laplace of standard deviation sigma)."""
    if not (0 < k < m):
        raise ValueError("need 0 < k < m")
    rng = np.random.Generator(np.random.PCG64(seed))
    A_cols = draw_columns(rng, n, m, d)
    support, values = draw_signal(rng, n, k, sigma_s, kind)
    eta = draw_noise(rng, m, sigma, noise_kind)
    return Instance(n=n, m=m, k=k, d=d, sigma=float(sigma), sigma_s=float(sigma_s),
                    A_cols=A_cols, support=support, values=values, eta=eta)


def draw_batch_shapes(count: int, seed: int, d: int = 7, log2_n=(12, 18), delta=(0.05, 0.5),
                      rho=(0.05, 0.3), snr_db=(20.0, 60.0)) -> list[tuple[int, int, int, float]]:
    """Shapes of a batch of uneven instances: n log-uniform in [2^a, 2^b], m = n * U(delta),
    k = m * U(rho) (at least 1), SNR uniform; returns (n, m, k, snr_db) per instance."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        n = int(round(2.0 ** rng.uniform(*log2_n)))
        m = max(d + 1, int(round(n * rng.uniform(*delta))))
        k = min(m - 1, max(1, int(round(m * rng.uniform(*rho)))))
        out.append((n, m, k, float(rng.uniform(*snr_db))))
    return out


def draw_batch(count: int, seed: int, d: int = 7, **shape_kw) -> list[Instance]:
    """A batch of instances with the shapes of draw_batch_shapes, each drawn from its own
    seed (seed * 100000 + i) with sigma_n from its SNR."""
    shapes = draw_batch_shapes(count, seed, d, **shape_kw)
    return [batch_member(shapes, seed, i, d) for i in range(count)]


def batch_member(shapes, seed: int, i: int, d: int = 7) -> Instance:
    """Instance i of the batch draw_batch(len(shapes), seed, d) makes from these shapes."""
    n, m, k, snr = shapes[i]
    sig = float(np.float32(sigma_for_snr(snr, n, m, k, d)))
    return draw_instance(n, m, k, d, sig, seed * 100000 + i)


def draw_instance_device(n: int, m: int, k: int, d: int, sigma: float, seed: int, device="cuda",
                         sigma_s: float = 1.0):
    """One instance of GM(n, m, k, d, N(0, sigma_s^2), N(0, sigma^2)) drawn on the device
    with torch's generator seeded by `seed` (for experiments of many large instances,
    where the host generator is the bottleneck; not the stream draw_instance gives).
    Returns (A_cols int32 [n][d], x float32 [n], eta float32 [m]) device tensors; the
    columns follow draw_columns' recipe: d iid rows, a column with a repeated row is
    redrawn whole, rows sorted ascending."""
    import torch

    if not (0 < k < m) or not (0 < d <= m):
        raise ValueError("need 0 < k < m and 0 < d <= m")
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    cols = torch.randint(0, m, (n, d), generator=g, device=device, dtype=torch.int64)
    cols, _ = torch.sort(cols, dim=1)
    while d > 1:
        bad = torch.nonzero((cols[:, 1:] == cols[:, :-1]).any(dim=1)).flatten()
        if bad.numel() == 0:
            break
        redraw = torch.randint(0, m, (bad.numel(), d), generator=g, device=device, dtype=torch.int64)
        cols[bad] = torch.sort(redraw, dim=1)[0]
    A = cols.to(torch.int32).contiguous()
    support = torch.randperm(n, generator=g, device=device)[:k]
    x = torch.zeros(n, dtype=torch.float32, device=device)
    x[support] = torch.randn(k, generator=g, device=device, dtype=torch.float32) * float(sigma_s)
    eta = torch.randn(m, generator=g, device=device, dtype=torch.float32) * float(sigma)
    return A, x, eta
