"""Robust-l0 (Alg. 1) and its noiseless reduction Parallel-l0 (Alg. 2), step by step.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Plain (continuous-score, non-adaptive) Robust-l0, Alg. 1:
    x_hat <- 0, r_hat <- y, t <- 1
    while not converged and t > 0:
        x' <- x_hat, r <- r_hat
        for every column j (all on the same snapshot r):
            for i in N(j) with 1 - p_breve_z(r_i) >= t:
                n_e   = sum_{l in N(j)} q_e(r_i - r_l)
                n_z   = sum_{l in N(j)} q_z(r_l)
                omega = sum_{l in N(j)} r_l q_e(r_i - r_l) / n_e
                candidate i passes if ||r - omega a_j||_1 <= ||r||_1 and n_e - n_z >= alpha
            x'_j <- x'_j + omega of the chosen passing candidate
        x' <- H_k(x')          (keep the k largest magnitudes)
        r  <- y - A x'
        t  <- t - c
        if ||r||_1 < ||r_hat||_1: x_hat <- x', r_hat <- r

Readings (listed with the rest in the design notes):
  * one update per column and iteration: among the passing candidates the one with the
    largest n_e wins (n_z is the same for all of them), ties to the smaller row index;
    this mirrors Parallel-l0's single assignment u_j <- r_i;
  * the l1 test compares the column's own rows: ||r - omega e_i||_1 is read as the
    change the update makes, omega times the column a_j, so the test is
    sum_{l in N(j)} |r_l - omega| <= sum_{l in N(j)} |r_l| (non-strict);
  * l = i is part of the sums, so n_e >= q_e(0) = 1;
  * "converged" is ||r_hat||_1 <= m sigma sqrt(2/pi), checked at the top of the loop;
  * the output is the best accepted iterate x_hat;
  * H_k keeps only nonzero entries; equal magnitudes go to the smaller column index.

Float32 contract (both this oracle and the GPU follow it, so their bits agree):
  * the sweep works in float32, every operation rounded in the order written below, no
    fused multiply-add; slot p runs over the column's rows in ascending row order;
      z_p  = Tz(|v_p|);  n_z = (((z_0 + z_1) + z_2) + ...);  S1 = sum_p |v_p| likewise
      candidate p iff fl32(1 - z_p) >= t
      w_pl = 1 if l == p else Te(|fl32(v_p - v_l)|)
      n_e  = sum_l w_pl,  s = sum_l fl32(v_l * w_pl)  (left folds from 0)
      omega = s / n_e (IEEE division),  L_p = sum_l |fl32(v_l - omega)|
      pass iff fl32(n_e - n_z) >= alpha and L_p <= S1
      x'_j = fl32(x_hat_j + omega_{p*})
  * residual in 64-bit fixed point with 40 fractional bits:
      S_i = rint(2^40 y_i) - sum_{j in supp x'} rint(2^40 x'_j) for i in N(j)
      r_i = fl32(fl64(S_i) * 2^-40)
    an exact integer sum, hence independent of summation order; it equals the exactly
    rounded y - A x' whenever every value is a multiple of 2^-40, which every float32 of
    magnitude >= 2^-17 is.  Smaller entries are rounded to the grid first (this also
    holds for r_hat <- y: rows with |y_i| < 2^-17 start at fl32(2^-40 rint(2^40 y_i)));
    fx_inexact counts them;
  * ||r||_1 is the integer L(r) = sum_i rint(2^30 |r_i|) (unit 2^-30), accepted on a
    strict decrease.

Quantised scores (Table "scores", middle column; Alg. 1's quantised flag): the weights
become indicators of the same tabulated scores, taken in float32,
      q_z(v) = 1{Tz(|v|) >= fl32(1 - t)},   q_e(a) = 1{Te(|a|) >= t}   (w_pp = 1 as before),
so n_e and n_z count rows and omega is the mean of the rows agreeing with row p; the
outer test is unchanged, and c = 0 selects eq:finetune_c_quant.  At t = 1 every row
counts as a zero (q_z = 1), so iteration 0 updates nothing.

adaptive_k (Alg. 1's adaptive_k branch; reading R17): after an accepted iteration the
posteriors are rebuilt for the sparsity still to be found,
      k_0 = max(k - sum_j (1 - p_breve_z(x_hat_j)), floor(m/100), 1),
each term taken on the current z-table in float32, fl32(1 - Tz(|x_hat_j|)), and summed
exactly as the integer sum_j rint(2^30 term) (x_hat_j = 0 adds 0), so k_0 is an exact
fp64 number; the tables are rebuilt with rho = k_0 / m.  H_k keeps the decoder's k, and the
schedule (c, the iterations) and the tolerance stay those of the start.

With sigma = 0 the scores are Parallel-l0's indicators and the same loop is Alg. 2
with its one-update-per-column rule (exact recovery check, Thm. "Convergence of
Algorithm 2").
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

from . import general as _general
from . import scores as _scores

__all__ = [
    "FX_SHIFT",
    "L1_SHIFT",
    "Constants",
    "make_constants",
    "adapted_sparsity",
    "adapt",
    "to_fixed",
    "from_fixed",
    "l1_fixed",
    "fx_inexact",
    "sketch",
    "measure",
    "sweep",
    "hard_threshold",
    "residual",
    "State",
    "init_state",
    "step",
    "decode",
    "DecodeResult",
]

FX_SHIFT = 40
L1_SHIFT = 30
_FX_LIMIT = 2.0 ** 62


@dataclass
class Constants:
    n: int
    m: int
    d: int
    k: int
    sigma: float
    sigma_s: float
    alpha: np.float32
    c: float
    n_iters: int
    tol: float
    Tz: _scores.Table
    Te: _scores.Table
    l1_test: int = 0
    variant: int = 0          # 0 continuous scores, 1 quantised (indicator) scores
    adaptive_k: int = 0       # rebuild the posteriors after each accepted iteration
    ell: int = 4
    k_post: float = 0.0       # the sparsity the current posteriors assume (k at the start)
    signal: str = "gaussian"  # the laws mu and nu (module general; gaussian: eq:pz_approx)
    noise: str = "gaussian"


def make_constants(n, m, d, k, sigma, sigma_s=1.0, alpha=2.0, c=0.0, ell=4,
                   max_iters=0, l1_test=0, variant=0, adaptive_k=0, signal="gaussian", noise="gaussian",
                   tables=None) -> Constants:
    """Alg. 1 prologue: p_breve_z, p_breve_e for GM(n, m, k, d, mu, nu), mu and nu of the
    given families with standard deviations sigma_s and sigma: N(0, ss^2), N(0, sn^2) by
    default (eq:pz_approx); otherwise the theorem's series (module general).  `tables` =
    (Tz, Te) replaces the score tables by given ones."""
    # Alg. 1 takes the consensus level alpha from (1, d]
    if not (1.0 < alpha <= d):
        raise ValueError("alpha must be in (1, d]")
    if variant not in (0, 1):
        raise ValueError("variant must be 0 (continuous) or 1 (quantised)")
    if signal not in _general.FAMILIES or noise not in _general.FAMILIES:
        raise ValueError(f"signal and noise laws must be among {_general.FAMILIES}")
    general = (signal, noise) != ("gaussian", "gaussian") or tables is not None
    if adaptive_k and general:
        raise ValueError("adaptive_k rebuilds the Gaussian posteriors of eq:pz_approx only")
    rho = k / m
    if c == 0.0:
        c = _scores.c_rule(m / n, rho, quantised=variant == 1)
    n_it = _scores.n_iters(c)
    if max_iters > 0:
        n_it = min(n_it, max_iters)
    if sigma == 0.0 or not general:
        Tz = _scores.build_table("z", d, rho, sigma, sigma_s, ell)
        Te = _scores.build_table("e", d, rho, sigma, sigma_s, ell)
    elif tables is not None:
        Tz, Te = tables
    else:
        Tz = _general.build_table("z", d, rho, (signal, sigma_s), (noise, sigma))
        Te = _general.build_table("e", d, rho, (signal, sigma_s), (noise, sigma))
    return Constants(n=n, m=m, d=d, k=k, sigma=float(sigma), sigma_s=float(sigma_s),
                     alpha=np.float32(alpha), c=float(c), n_iters=n_it,
                     tol=_general.noise_l1_mean(m, (noise, sigma)), Tz=Tz, Te=Te, l1_test=l1_test,
                     variant=variant, adaptive_k=adaptive_k, ell=ell, k_post=float(k), signal=signal, noise=noise)


def adapted_sparsity(C: Constants, x_hat: np.ndarray) -> float:
    """k_0 of the adaptive_k branch (module docstring, reading R17)."""
    x = np.asarray(x_hat, dtype=np.float32)
    nz = x[x != 0]
    z = _scores.lookup(C.Tz, np.abs(nz))
    term = (np.float32(1.0) - z).astype(np.float32)
    S = int(np.rint(term.astype(np.float64) * (2.0 ** L1_SHIFT)).astype(np.int64).sum(dtype=np.int64))
    k0 = float(C.k) - float(S) * (2.0 ** -L1_SHIFT)
    return max(k0, float(C.m // 100), 1.0)


def adapt(C: Constants, x_hat: np.ndarray) -> Constants:
    """The constants after an accepted iteration of the adaptive_k branch: the tables of
    p_breve_z and p_breve_e rebuilt with rho = k_0 / m; everything else kept."""
    k0 = adapted_sparsity(C, x_hat)
    rho = k0 / C.m
    Tz = _scores.build_table("z", C.d, rho, C.sigma, C.sigma_s, C.ell)
    Te = _scores.build_table("e", C.d, rho, C.sigma, C.sigma_s, C.ell)
    return replace(C, Tz=Tz, Te=Te, k_post=k0)


# ----------------------------------------------------------------------------- fixed point

def to_fixed(v) -> np.ndarray:
    """rint(2^40 v) as int64, for float32 v (round half to even)."""
    s = np.asarray(v, dtype=np.float32).astype(np.float64) * (2.0 ** FX_SHIFT)
    if s.size and not (np.abs(s) < _FX_LIMIT).all():
        raise OverflowError("value outside the fixed-point range")
    return np.rint(s).astype(np.int64)


def from_fixed(S: np.ndarray) -> np.ndarray:
    """fl32(fl64(S) * 2^-40)."""
    return (np.asarray(S, dtype=np.int64).astype(np.float64) * (2.0 ** -FX_SHIFT)).astype(np.float32)


def fx_inexact(v) -> int:
    """Entries of v (float32) that are not multiples of 2^-40, so that rint(2^40 v) rounds.
    Only such entries make the fixed-point residual differ from the exactly rounded
    y - A x; a float32 value is a multiple of 2^-40 whenever |v| >= 2^-17."""
    s = np.asarray(v, dtype=np.float32).astype(np.float64) * (2.0 ** FX_SHIFT)
    return int(np.count_nonzero(s != np.rint(s)))


def l1_fixed(r: np.ndarray) -> int:
    """L(r) = sum_i rint(2^30 |r_i|), an exact integer in units of 2^-30."""
    a = np.abs(np.asarray(r, dtype=np.float32)).astype(np.float64) * (2.0 ** L1_SHIFT)
    return int(np.rint(a).astype(np.int64).sum(dtype=np.int64))


# ----------------------------------------------------------------------------- sketch

def sketch(A_cols: np.ndarray, x: np.ndarray, m: int) -> np.ndarray:
    """y = A x (Sec. 1): y_i = fl32(2^-40 sum_{j: i in N(j)} rint(2^40 x_j))."""
    A_cols = np.asarray(A_cols)
    n, d = A_cols.shape
    fx = to_fixed(x)
    S = np.zeros(m, dtype=np.int64)
    for p in range(d):
        np.add.at(S, A_cols[:, p].astype(np.int64), fx)
    return from_fixed(S)


def measure(A_cols, x, eta, m) -> np.ndarray:
    """y_hat = y + eta with y = A x (Definition "Generating model"), in float32."""
    return (sketch(A_cols, x, m) + np.asarray(eta, dtype=np.float32)).astype(np.float32)


# ----------------------------------------------------------------------------- one sweep

@dataclass
class SweepOut:
    x_prime: np.ndarray      # float32 [n]: x_hat with the accepted column updates
    updated: np.ndarray      # bool [n]
    omega: np.ndarray        # float32 [n]: chosen omega (0 where not updated)
    n_e: np.ndarray          # float32 [n]: n_e of the chosen candidate (0 if none)
    n_z: np.ndarray          # float32 [n]
    p_star: np.ndarray       # int8 [n]: chosen slot, -1 if none


def sweep(A_cols, r_hat, x_hat, t, C: Constants) -> SweepOut:
    """The column loop of Alg. 1 on the snapshot r_hat (float32 contract above)."""
    A_cols = np.asarray(A_cols)
    n, d = A_cols.shape
    f32 = np.float32
    V = np.asarray(r_hat, dtype=np.float32)[A_cols]          # v_p = r_hat[row_p]
    absV = np.abs(V)
    t = f32(t)
    Z = np.stack([_scores.lookup(C.Tz, absV[:, p]) for p in range(d)], axis=1)
    quant = C.variant == 1 and not C.Tz.exact
    # the z-weights: the score itself, or its indicator at level 1 - t (quantised)
    Zw = (Z >= (f32(1.0) - t).astype(f32)).astype(f32) if quant else Z
    n_z = Zw[:, 0].copy()
    S1 = absV[:, 0].copy()
    for p in range(1, d):
        n_z = (n_z + Zw[:, p]).astype(f32)
        S1 = (S1 + absV[:, p]).astype(f32)
    has = np.zeros(n, dtype=bool)
    best_ne = np.zeros(n, dtype=f32)
    best_om = np.zeros(n, dtype=f32)
    p_star = np.full(n, -1, dtype=np.int8)
    for p in range(d):
        outer = (f32(1.0) - Z[:, p]).astype(f32) >= t
        n_e = np.zeros(n, dtype=f32)
        s = np.zeros(n, dtype=f32)
        for l in range(d):
            if l == p:
                w = np.ones(n, dtype=f32)
            else:
                w = _scores.lookup(C.Te, np.abs((V[:, p] - V[:, l]).astype(f32)))
                if quant:
                    w = (w >= t).astype(f32)
            n_e = (n_e + w).astype(f32)
            s = (s + (V[:, l] * w).astype(f32)).astype(f32)
        omega = (s / n_e).astype(f32)
        if C.l1_test == 0:
            Lp = np.abs((V[:, 0] - omega).astype(f32))
            for l in range(1, d):
                Lp = (Lp + np.abs((V[:, l] - omega).astype(f32))).astype(f32)
            l1_ok = Lp <= S1
        else:   # literal reading |r_i - omega| <= |r_i| (exploration only)
            l1_ok = np.abs((V[:, p] - omega).astype(f32)) <= absV[:, p]
        passed = outer & ((n_e - n_z).astype(f32) >= C.alpha) & l1_ok
        better = passed & (~has | (n_e > best_ne))
        best_ne = np.where(better, n_e, best_ne).astype(f32)
        best_om = np.where(better, omega, best_om).astype(f32)
        p_star = np.where(better, p, p_star).astype(np.int8)
        has |= passed
    x_prime = np.asarray(x_hat, dtype=f32).copy()
    x_prime[has] = (x_prime[has] + best_om[has]).astype(f32)
    return SweepOut(x_prime=x_prime, updated=has, omega=np.where(has, best_om, f32(0)).astype(f32),
                    n_e=np.where(has, best_ne, f32(0)).astype(f32), n_z=n_z, p_star=p_star)


# ----------------------------------------------------------------------------- H_k

def hk_keys(x: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """Order key of H_k: magnitude first, then the smaller column index."""
    mag = np.abs(x[idx].astype(np.float32)).view(np.uint32).astype(np.uint64)
    return (mag << np.uint64(32)) | (np.uint64(0xFFFFFFFF) - idx.astype(np.uint64))


def hard_threshold(x: np.ndarray, k: int) -> np.ndarray:
    """H_k: keep the k entries of largest magnitude (nonzero entries only)."""
    x = np.asarray(x, dtype=np.float32)
    nz = np.nonzero(x)[0]
    out = np.zeros_like(x)
    if nz.size <= k:
        out[nz] = x[nz]
        return out
    keys = hk_keys(x, nz)
    keep = nz[np.argsort(keys)[::-1][:k]]
    out[keep] = x[keep]
    return out


# ----------------------------------------------------------------------------- residual

def residual(A_cols, y_hat, x: np.ndarray, m: int) -> np.ndarray:
    """r = y_hat - A x in the fixed-point contract above."""
    A_cols = np.asarray(A_cols)
    S = to_fixed(y_hat)
    nz = np.nonzero(x)[0]
    fx = to_fixed(x[nz])
    for p in range(A_cols.shape[1]):
        np.subtract.at(S, A_cols[nz, p].astype(np.int64), fx)
    return from_fixed(S)


# ----------------------------------------------------------------------------- loop

@dataclass
class State:
    x_hat: np.ndarray
    r_hat: np.ndarray
    L_hat: int
    it: int
    accepted: int = 0


def init_state(y_hat: np.ndarray, n: int) -> State:
    """x_hat <- 0, r_hat <- y (as the residual of x = 0)."""
    y_hat = np.asarray(y_hat, dtype=np.float32)
    r0 = from_fixed(to_fixed(y_hat))
    return State(x_hat=np.zeros(n, np.float32), r_hat=r0, L_hat=l1_fixed(r0), it=0)


def converged(state: State, C: Constants) -> bool:
    return float(state.L_hat) * (2.0 ** -L1_SHIFT) <= C.tol


@dataclass
class StepOut:
    state: State
    accepted: bool
    L_trial: int
    x_trial: np.ndarray
    r_trial: np.ndarray
    sweep: SweepOut


def step(A_cols, y_hat, state: State, C: Constants) -> StepOut:
    """One pass of the while-loop body of Alg. 1 at t = 1 - it c."""
    t = _scores.t_of(state.it, C.c)
    sw = sweep(A_cols, state.r_hat, state.x_hat, t, C)
    x_trial = hard_threshold(sw.x_prime, C.k)
    r_trial = residual(A_cols, y_hat, x_trial, C.m)
    L_trial = l1_fixed(r_trial)
    acc = L_trial < state.L_hat
    if acc:
        new = State(x_hat=x_trial, r_hat=r_trial, L_hat=L_trial, it=state.it + 1,
                    accepted=state.accepted + 1)
    else:
        new = State(x_hat=state.x_hat, r_hat=state.r_hat, L_hat=state.L_hat,
                    it=state.it + 1, accepted=state.accepted)
    return StepOut(state=new, accepted=acc, L_trial=L_trial, x_trial=x_trial,
                   r_trial=r_trial, sweep=sw)


@dataclass
class DecodeResult:
    x_hat: np.ndarray
    r_hat: np.ndarray
    L_hat: int
    iterations: int
    accepted: int
    converged: bool
    updates_total: int
    fx_inexact_y: int = 0     # entries of y_hat whose fixed-point conversion rounds
    fx_inexact_x: int = 0     # nonzero x'_j of updated columns whose conversion rounds,
                              # summed over the executed iterations
    k_post: float = 0.0       # the sparsity the posteriors of the last executed iteration
                              # assumed (k unless adaptive_k)
    trace: list = field(default_factory=list)


def decode(A_cols, y_hat, C: Constants, keep_trace: bool = False) -> DecodeResult:
    """Alg. 1 from x_hat = 0 until converged or t <= 0."""
    A_cols = np.asarray(A_cols)
    st = init_state(y_hat, A_cols.shape[0])
    trace = []
    updates = 0
    inexact_x = 0
    k_last = C.k_post
    while st.it < C.n_iters and not converged(st, C):
        k_last = C.k_post
        out = step(A_cols, y_hat, st, C)
        n_upd = int(out.sweep.updated.sum())
        updates += n_upd
        xp = out.sweep.x_prime[out.sweep.updated]
        inexact_x += fx_inexact(xp[xp != 0])
        if C.adaptive_k and out.accepted and not C.Tz.exact:
            C = adapt(C, out.state.x_hat)
        if keep_trace:
            # (||r_hat||_1 before, ||r||_1 of the trial iterate, accepted, column updates)
            trace.append((st.L_hat, out.L_trial, out.accepted, n_upd))
        st = out.state
    return DecodeResult(x_hat=st.x_hat, r_hat=st.r_hat, L_hat=st.L_hat, iterations=st.it,
                        accepted=st.accepted, converged=converged(st, C),
                        updates_total=updates, fx_inexact_y=fx_inexact(y_hat), fx_inexact_x=inexact_x,
                        k_post=k_last, trace=trace)
