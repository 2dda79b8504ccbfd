"""Benchmark of the Robust-l0 hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--seeds S] [--no-cpu-baseline]

Workload: n = 2^20 columns, m = n/10 = 104857 rows, d = 7 ones per column at uniformly
random distinct rows, k = m/10 = 10485 nonzeros drawn N(0,1), Gaussian noise at 40 dB
SNR (sigma_n = 0.00836632), synthetic and seeded.  One step is one pass of the whole
hot path over one instance already resident in HBM: the sketch y = A x, y_hat = y + eta,
and the Robust-l0 decode of y_hat (initialisation, every loop iteration, the copy of
x_hat).  Step i decodes seed i mod S of S pre-generated seeds (S = 20 by default); the
time to solution T is the median over the timed steps.  The score tables, thresholds
and tolerance of a parameter set are computed on the host once and cached: every seed
shares them, so they are outside T.

Printed: one JSON line with the throughput in nnz(A)-updates/s (d * n * iterations
executed / wall time), T, the recovery error, the roofline and the CPU oracle's rate on
a bounded sample of the same workload.  Roofline bytes per loop iteration follow the
method's data movement: B_it = 4dn (column indices) + 4m (r_hat) + 24m (residual rebuild:
y read, 64-bit residual written and read, r written) + 16dk (64-bit scatter of the kept
columns) + 12(k + u) (candidates and update lists, u = updates of the iteration).  The
fractions of 8 TB/s reported: B_it over the sweep's average launch time (the dominant
kernel), over the sweep plus the row kernel (one iteration), and end to end,
(sum of B_it + 4dn of ingest) / T.  The timed steps replay each decode's captured launch
graph; the kernels' average launch times come from HIP events on the decode stream around
every launch, in a second pass over the same steps that launches eagerly (events cannot
sit inside the graph).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1704_09012_amd import instances as I  # noqa: E402

METRIC = "Robust-l0 nnz(A)-updates/s and time-to-solution, n=2^20 d=7, rel err<1e-2"
N, M, K, DD, SNR = 2 ** 20, 104857, 10485, 7, 40
HBM_PEAK_GBS = 8000.0

# HBM byte counters of the sweep (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE, mean KiB
# per dispatch at this workload) and the factors a 256 MiB plain copy gives each counter;
# valid only for the kernel source they were taken on.
SWEEP_COUNTERS = {
    "kernels_sha256": "d625cf34883c045351ef61fdbdd89553892360ab8bf95c04c7c638a16c450824",
    "fetch_kib": 13384.0, "write_kib": 221.0, "fetch_factor": 2.000, "write_factor": 1.000,
}


def sweep_traffic():
    """Bytes per sweep dispatch from the byte counters, or None once the kernels changed."""
    import hashlib

    src = os.path.join(ROOT, "paper_1704_09012_amd", "csrc", "kernels.hip")
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != SWEEP_COUNTERS["kernels_sha256"]:
            return None
    c = SWEEP_COUNTERS
    return 1024.0 * (c["fetch_kib"] * c["fetch_factor"] + c["write_kib"] * c["write_factor"])


def instance_record(workload, inst, seed, snr, sigma, st, x_hat, x_true, rel, b_it) -> dict:
    """One decoded instance as a record: the instance, its decode's statistics and device
    time, throughput and algorithmic bytes, and its recovery (relative l2 error, the l1
    success condition ||r_hat||_1 <= tol, and how much of the true support x_hat found)."""
    true_s = x_true != 0
    hat_s = x_hat != 0
    found = int((true_s & hat_s).sum())
    ms = float(st["ms_total"])
    nnz_upd = inst.d * inst.n * st["iterations"]
    return {"workload": workload, "seed": int(seed), "n": inst.n, "m": inst.m, "k": inst.k, "d": inst.d,
            "snr_db": snr, "sigma": sigma, "iterations": st["iterations"], "accepted": st["accepted"],
            "updates_total": st["updates_total"], "device_ms": ms,
            "nnz_updates_per_s": nnz_upd / (ms * 1e-3) if ms > 0 else None,
            "algorithmic_bytes": b_it * st["iterations"] + 4.0 * inst.d * inst.n,
            "rel_l2_err": rel, "l1_success": bool(st["converged"]),
            "support_found": found / max(int(true_s.sum()), 1), "support_size": int(hat_s.sum())}


def write_records(path: str, records) -> None:
    with open(path, "w") as f:
        for r in records:
            f.write(json.dumps(r) + "\n")
    print(f"{len(records)} instance records written to {path}", file=sys.stderr, flush=True)


def iteration_bytes(n: int, m: int, d: int, k: int, u: float) -> float:
    """Algorithmic bytes B_it of one loop iteration with u column updates (module
    docstring)."""
    return 4.0 * d * n + 4.0 * m + 24.0 * m + 16.0 * d * k + 12.0 * (k + u)


def _oracle_sample(args) -> tuple[int, float]:
    """One process of the CPU baseline: the oracle's first loop iterations of the seeded
    instance, as many as fit in budget_s seconds; returns (iterations, seconds)."""
    n, m, k, d, sigma, seed, budget_s, variant, adaptive, laws = args
    from oracle import decoder as D
    from oracle import scores as S
    inst = I.draw_instance(n, m, k, d, sigma, seed, kind=laws[0], noise_kind=laws[1])
    y_hat = D.measure(inst.A_cols[inst.support], inst.values, inst.eta, m)
    tables = None
    if laws != ("gaussian", "gaussian"):
        # the oracle's own tables of these laws, stored by tests/golden/make_tables.py
        g = np.load(general_tables_path(n, m, k, d, laws))
        tables = (S.Table(g["Tz"], np.float32(g["inv_h_z"]), float(g["R_z"])),
                  S.Table(g["Te"], np.float32(g["inv_h_e"]), float(g["R_e"])))
    C = D.make_constants(n, m, d, k, sigma, variant=variant, adaptive_k=adaptive, signal=laws[0], noise=laws[1],
                         tables=tables)
    st = D.init_state(y_hat, n)
    t0 = time.perf_counter()
    done = 0
    while time.perf_counter() - t0 < budget_s:
        if st.it >= C.n_iters or D.converged(st, C):
            break
        out = D.step(inst.A_cols, y_hat, st, C)
        if adaptive and out.accepted and not C.Tz.exact:
            C = D.adapt(C, out.state.x_hat)
        st = out.state
        done += 1
    return done, time.perf_counter() - t0


def general_tables_path(n, m, k, d, laws) -> str:
    return os.path.join(ROOT, "tests", "golden", f"tables_n{n}_m{m}_k{k}_d{d}_snr{SNR}_{laws[0]}_{laws[1]}.npz")


def cpu_baseline(n, m, k, d, sigma, seeds, budget_s: float = 12.0, procs: int = 8, variant: int = 0,
                 adaptive: int = 0, laws=("gaussian", "gaussian")) -> dict:
    """The oracle (test infrastructure) timed on the host: single-threaded numpy, first on
    one core, then `procs` processes at once on different seeds (the aggregate rate)."""
    import multiprocessing as mp

    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    done1, dt1 = _oracle_sample((n, m, k, d, sigma, seeds[0], budget_s, variant, adaptive, laws))
    rate1 = d * n * done1 / dt1
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    procs = max(1, min(procs, avail))
    ctx = mp.get_context("spawn")
    with ctx.Pool(procs) as pool:
        res = pool.map(_oracle_sample,
                       [(n, m, k, d, sigma, seeds[i % len(seeds)], budget_s, variant, adaptive, laws)
                        for i in range(procs)])
    agg = sum(d * n * it / t for it, t in res)
    its = [it for it, _ in res]
    return {"value": agg, "unit": "nnz(A)-updates/s", "cores": procs, "kind": "oracle",
            "value_1core": rate1,
            "sample": f"the first loop iterations of decodes of the same n={n} workload, about {budget_s:.0f} s "
                      f"each, numpy float32 contract, 1 thread per process: {procs} processes at once on "
                      f"{procs} seeds ({min(its)}-{max(its)} iterations each; value = the sum of their rates); "
                      f"alone on one core: {done1} iterations in {dt1:.1f} s (value_1core)"}


def copy_calibration() -> int:
    """Plain copies of known size: each reads and writes 256 MiB per launch, so the
    FETCH_SIZE and WRITE_SIZE counters a profiler reports for them give their scale."""
    import torch

    nbytes = 256 << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)                 # the runtime's copy kernel
    for _ in range(3):
        torch.neg(src, out=dst)        # an elementwise kernel: 16-byte loads and stores per lane
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read_per_launch": nbytes, "copy_bytes_written_per_launch": nbytes,
                      "launches": {"copyBuffer": 3, "neg (elementwise)": 3}}), flush=True)
    return 0


def bench_learned(args) -> int:
    """The learned decision against the analytic one at the headline size: the network
    is trained on the GPU on trajectories of the n = 1024 workload (2000 decodes, SNR in
    [20, 60] dB, 30 epochs), then `--seeds` instances per SNR (20, 40, 60 dB) are decoded
    both ways."""
    import torch
    from paper_1704_09012_amd import learned as Lrn

    t0 = time.perf_counter()
    F, Y = Lrn.trajectories(2000, 1)
    torch.cuda.synchronize()
    t_traj = time.perf_counter() - t0
    print(f"trajectories: {F.shape[0]} samples in {t_traj:.1f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    w, loss = Lrn.train(F, Y, epochs=30)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    print(f"trained in {t_train:.1f} s, loss {loss:.4f}", file=sys.stderr, flush=True)
    per_snr = {}
    for snr in (20, 40, 60):
        print(f"comparing at {snr} dB", file=sys.stderr, flush=True)
        rows = Lrn.compare(w, N, M, K, snr, [I.seed_for(5, i, j) for i, j in [(snr // 20, j) for j in range(args.seeds)]])
        agg = {}
        for tag in ("analytic", "learned"):
            agg[tag] = {
                "rel_err_median": float(np.median([r[tag]["rel_err"] for r in rows])),
                "frac_rel_err_below_1e-2": float(np.mean([r[tag]["rel_err"] < 1e-2 for r in rows])),
                "converged_frac": float(np.mean([r[tag]["converged"] for r in rows])),
                "iterations_mean": float(np.mean([r[tag]["iterations"] for r in rows])),
                "ms_median": float(np.median([r[tag]["ms"] for r in rows])),
                "ms_each": [round(r[tag]["ms"], 3) for r in rows],
            }
        per_snr[str(snr)] = agg
    kernels = _learned_kernel_costs(w)
    out = {
        "metric": "learned vs analytic column decision, n=2^20 d=7",
        "value": per_snr["40"]["learned"]["ms_median"],
        "unit": "ms per decode (learned, 40 dB)",
        "n_gpus": 1,
        "higher_is_better": False,
        "dtype": "bf16 inference (fp32 accumulate), fp32 training",
        "data": "synthetic",
        "config": {"workload": "train on n=1024 m=256 k=25 trajectories (2000 decodes, SNR U[20,60]); "
                               "evaluate n=2^20 m=104857 k=10485 at SNR 20/40/60 dB",
                   "seeds_per_snr": args.seeds},
        "training": {"samples": int(F.shape[0]), "positives": int(Y[:, 0].sum()), "loss": loss,
                     "trajectory_s": t_traj, "train_s": t_train},
        "per_snr": per_snr,
        "kernels": kernels,
    }
    print(json.dumps(out), flush=True)
    return 0


# VALU model of the learned column decision (bf16 network on the matrix cores): per column
# 128 GELUs (two hidden layers of 64), each 12 full-rate VALU instructions and 2
# transcendental ones (reciprocal, base-2 exponential), which issue at a quarter of the
# rate, so 12 + 2 * 4 = 20 issue slots per GELU.  Packed fp32 instructions are not used, so
# the peak is 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 3.93e13 lane-slots/s.
LEARNED_SLOTS_PER_COLUMN = 128 * (12 + 2 * 4)
VALU_LANE_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9
# fp32 training arithmetic per sample: forward 2 (64 F + 64 * 64 + 2 * 64) flops, backward
# twice that (input gradients and weight gradients), F = d + 1 = 8
TRAIN_FLOPS_PER_SAMPLE = 3 * 2 * (64 * 8 + 64 * 64 + 2 * 64)


def _learned_kernel_costs(w, reps: int = 10, train_steps: int = 200, batch: int = 4096) -> dict:
    """Live costs of the learned path's kernels with HIP events on the stream they run on:
    one learned iteration (rl0_step with the network's decisions, which evaluates the
    network on every column: n = 2^20, d = 7, 40 dB, from x_hat = 0 at t-step 10) against
    the same analytic iteration, and training steps of `batch` samples (gradient + Adam)."""
    import torch
    from paper_1704_09012_amd import rl0 as R

    sigma = float(np.float32(I.sigma_for_snr(SNR, N, M, K, DD)))
    A, x, eta = I.draw_instance_device(N, M, K, DD, sigma, 777)
    y = R.sketch(A, x, M) + eta
    x0 = torch.zeros(N, dtype=torch.float32, device="cuda")
    L0 = int(torch.round(torch.abs(y).double() * 2.0 ** 30).sum().item())

    def time_steps(params) -> float:
        xs, rs = x0.clone(), y.clone()
        R.step(A, y, params, 10, xs, rs, L0, debug=False)            # warm
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms = []
        for _ in range(reps):
            xs.copy_(x0)
            rs.copy_(y)
            ev0.record()
            R.step(A, y, params, 10, xs, rs, L0, debug=False)
            ev1.record()
            torch.cuda.synchronize()
            ms.append(ev0.elapsed_time(ev1))
        return float(np.median(ms))

    step_learned = time_steps(R.params_default(N, M, DD, K, sigma, mlp=w))
    step_analytic = time_steps(R.params_default(N, M, DD, K, sigma))
    # the learned decision's own kernel, timed by the library with HIP events around it
    R.profile_enable(True)
    time_steps(R.params_default(N, M, DD, K, sigma, mlp=w))
    lc_ms, lc_launches = R.profile_read_learned()
    R.profile_enable(False)
    lc_us = 1e3 * lc_ms / max(lc_launches, 1)
    bound_us = 1e6 * N * LEARNED_SLOTS_PER_COLUMN / VALU_LANE_SLOTS_PER_S

    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    F = torch.randn(batch * 8, DD + 1, device="cuda", generator=g)
    Y = torch.stack([(torch.rand(batch * 8, device="cuda", generator=g) < 0.1).float(),
                     torch.randn(batch * 8, device="cuda", generator=g)], dim=1).contiguous()
    wt = w.clone()
    mm, vv = torch.zeros_like(wt), torch.zeros_like(wt)
    R.mlp_train(F, Y, wt, mm, vv, 8, batch=batch)                     # warm
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    R.mlp_train(F, Y, wt, mm, vv, train_steps, t0=8, batch=batch)
    ev1.record()
    torch.cuda.synchronize()
    train_us = 1e3 * ev0.elapsed_time(ev1) / train_steps
    return {
        "learned_step_ms": step_learned,
        "analytic_step_ms": step_analytic,
        "learned_cols_full_us": lc_us,
        "learned_cols_launches": lc_launches,
        "learned_cols_valu_bound_us": bound_us,
        "learned_cols_frac_of_bound": bound_us / lc_us,
        "learned_cols_model": "every column of n = 2^20 through the network; bound = 128 GELUs per column x "
                              "(12 + 2 x 4) issue slots / (256 CU x 64 lanes x 2.4 GHz)",
        "train_step_us": train_us,
        "train_batch": batch,
        "train_tflops": TRAIN_FLOPS_PER_SAMPLE * batch / (train_us * 1e-6) / 1e12,
    }


def bench_phase(args) -> int:
    """Phase transitions for extreme subsampling (Sec. 4): the ladder of
    paper_1704_09012_amd.phase for (delta, sigma) in {0.001, 0.01} x {0.001, 0.01} at n =
    --phase-n, Robust-l0 and Robust-l0-quantised, 10 instances per rho drawn on the device;
    reports the 50% point of the logistic fit and the largest rho with half recovered.
    The paper states, for Robust-l0 at n = 2^22 -> 2^24: rho* ~ 0.08 -> 0.1 at delta =
    sigma = 0.001, ~0.17 at delta = 0.01, sigma = 0.001 and ~0.12 at delta = sigma = 0.01."""
    from paper_1704_09012_amd import phase as PH

    t0 = time.perf_counter()
    rows = []
    for variant in (0, 1):
        for delta in (0.001, 0.01):
            for sigma in (0.001, 0.01):
                res = PH.ladder(PH.gpu_trials, n=args.phase_n, delta=delta, sigma=sigma, variant=variant,
                                trials=10, seed=int(1e6 * delta + 1e3 * sigma))
                rows.append(res.as_dict())
                print(json.dumps({"ladder": rows[-1]}), flush=True)
    paper = {"(0.001, 0.001)": "0.08 (n=2^22) -> 0.1 (n=2^24)", "(0.01, 0.001)": "0.17",
             "(0.01, 0.01)": "0.12"}
    out = {
        "metric": "Robust-l0 phase transition rho* (50% point of the logistic fit), extreme subsampling",
        "value": next(r["rho50"] for r in rows if r["variant"] == 0 and r["delta"] == 0.01 and r["sigma"] == 0.001),
        "unit": "rho* at delta=0.01, sigma=0.001",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"ladders rho = 0.01, 0.02, ... with 10 GM instances each (N(0,1) signal, "
                               f"N(0, sigma^2) noise, d=7), n={args.phase_n}; success = eq:success_condition_clip, "
                               "C1 = 1", "n": args.phase_n},
        "paper_rho_star_robust_l0": paper,
        "ladders": rows,
        "seconds": time.perf_counter() - t0,
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_batched(args) -> int:
    """Batched decoding: `--batch` instances with n log-uniform in [2^12, 2^18], m/n in
    [0.05, 0.5], k/m in [0.05, 0.3], d = 7, SNR in [20, 60] dB.  The schedule is tuned
    once on the batch; then `--steps` timed batched decodes (graph replays), and one
    timed pass of single decodes over the same instances for comparison."""
    import torch
    from paper_1704_09012_amd import rl0 as R

    insts = I.draw_batch(args.batch, 0, DD)
    probs = []
    for inst in insts:
        A = torch.from_numpy(inst.A_cols).cuda()
        x = torch.from_numpy(inst.x_dense()).cuda()
        y = R.sketch(A, x, inst.m) + torch.from_numpy(inst.eta).cuda()
        probs.append({"A": A, "y": y, "sigma": inst.sigma, "k": inst.k, "x": x})
    batch = [{k: v for k, v in p.items() if k != "x"} for p in probs]
    best, tuned_ms = R.autotune_batched(batch, reps=2)
    # the problem array is marshalled once, as a C caller holds its rl0_problem array;
    # the library still plans, uploads and decodes the whole batch in every call
    prepared = R.PreparedBatch(batch)
    for _ in range(args.warmup):
        R.decode_batched(prepared, stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        R.decode_batched(prepared, stats=False)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.steps
    stats = [prepared.stats[i].as_dict() for i in range(len(prepared))]
    t_start, t_end, groups = R.batch_timeline(len(batch))
    busy = float(np.sum((t_end - t_start) * groups))          # workgroup-milliseconds
    W = 256 * best["per_cu"]
    upd = sum(DD * inst.n * st["iterations"] for inst, st in zip(insts, stats))
    # algorithmic HBM bytes of every executed iteration: indices and one residual read
    algo = sum((4.0 * DD * inst.n + 8.0 * inst.m) * st["iterations"] for inst, st in zip(insts, stats))
    rel = [float(torch.linalg.norm(b["out"] - p["x"]) / torch.linalg.norm(p["x"])) for b, p in zip(batch, probs)]
    # the same instances one decode at a time (second pass: graphs already captured)
    outs = [torch.empty(inst.n, dtype=torch.float32, device="cuda") for inst in insts]
    for rep in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b, o in zip(batch, outs):
            R.decode(b["A"], b["y"], sigma=b["sigma"], k=b["k"], out=o)
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t0
    same = all(bool(torch.equal(b["out"], o)) for b, o in zip(batch, outs))
    achieved = algo / t_batch / 1e9
    out = {
        "metric": "batched Robust-l0 decode, nnz(A)-updates/s",
        "value": upd / t_batch,
        "unit": "nnz(A)-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_batch,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.batch} uneven instances: n log-uniform [2^12, 2^18], m/n U[0.05, 0.5], "
                               "k/m U[0.05, 0.3], d=7, SNR U[20, 60] dB; step = one batched decode",
                   "instances": args.batch, "sum_n": int(sum(i.n for i in insts)), "d": DD},
        "schedule": best,
        "timeline": {"span_ms": float(t_end.max() - t_start.min()), "mean_workgroup_busy_ms": busy / W,
                     "span_over_mean_busy": float(t_end.max() - t_start.min()) / (busy / W),
                     "instances_split": int(np.sum(groups > 1)), "largest_group": int(groups.max()),
                     "note": "device clock of the last timed call; busy = sum of decode durations times "
                             "group size over the resident workgroups"},
        "sequential_single_decodes_ms": 1e3 * t_seq,
        "speedup_vs_sequential": t_seq / t_batch,
        "identical_to_single_decodes": same,
        "rel_l2_err_median": float(np.median(rel)),
        "frac_rel_err_below_1e-2": float(np.mean(np.array(rel) < 1e-2)),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_decode_batched<7>",
                     "bytes": "4dn + 8m per executed iteration, summed; over the whole batched call"},
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_decode(args, N: int, M: int, K: int, DD: int, config: int, seeds: int, workload: str,
                 cpu: bool, variant: int = 0, adaptive: int = 0, laws=("gaussian", "gaussian")) -> int:
    """Single decodes of `seeds` seeded instances of GM(N, M, K, DD) at SNR 40 dB, step i on
    seed i mod seeds (sketch + decode, graph replay), then the same steps again with HIP
    events on every loop kernel for the roofline."""
    import torch
    from paper_1704_09012_amd import rl0 as R

    dev = torch.device("cuda:0")
    sigma = float(np.float32(I.sigma_for_snr(SNR, N, M, K, DD)))
    seed_ids = [I.seed_for(config, 1, i) for i in range(seeds)]
    insts = []
    for sd in seed_ids:
        inst = I.draw_instance(N, M, K, DD, sigma, sd, kind=laws[0], noise_kind=laws[1])
        insts.append({
            "inst": inst,
            "A": torch.from_numpy(inst.A_cols).to(dev),
            "x": torch.from_numpy(inst.x_dense()).to(dev),
            "eta": torch.from_numpy(inst.eta).to(dev),
        })
        del inst
    params = R.params_default(N, M, DD, K, sigma, variant=variant, adaptive_k=adaptive, signal_law=laws[0],
                              noise_law=laws[1])
    y = torch.empty(M, dtype=torch.float32, device=dev)
    y_hat = torch.empty(M, dtype=torch.float32, device=dev)
    x_hat = torch.empty(N, dtype=torch.float32, device=dev)

    def one_step(i):
        b = insts[i % len(insts)]
        R.sketch(b["A"], b["x"], M, out=y)
        torch.add(y, b["eta"], out=y_hat)
        _, st = R.decode(b["A"], y_hat, params=params, out=x_hat)
        return st

    # setup, untimed: one decode of each instance captures its graph (a serving loop
    # captures once per problem); then the warm-up steps
    for i in range(len(insts)):
        one_step(i)
    for i in range(args.warmup):
        one_step(i)
    torch.cuda.synchronize()
    iters = updates = 0
    per_step, dev_ms, rel = [], [], []
    t_start = time.perf_counter()
    for i in range(args.steps):
        t0 = time.perf_counter()
        st = one_step(i)          # returns after the decode's stream synchronised
        per_step.append(time.perf_counter() - t0)
        dev_ms.append(st["ms_total"])
        iters += st["iterations"]
        updates += st["updates_total"]
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    # recovery error of every timed step's instance (outside the timed region)
    records = []
    for i in range(min(args.steps, len(insts))):
        st_i = one_step(i)
        b = insts[i]
        rel.append(float(torch.linalg.norm(x_hat - b["x"]) / torch.linalg.norm(b["x"])))
        if args.records:
            records.append(instance_record(workload, b["inst"], seed_ids[i], SNR, sigma, st_i, x_hat, b["x"], rel[-1],
                                           iteration_bytes(N, M, DD, K, st_i["updates_total"] / max(st_i["iterations"], 1))))
    if args.records:
        write_records(args.records, records)

    # Kernel durations: the same K steps again, with HIP events on the decode stream
    # around every sweep, select and row launch (a decode with events launches eagerly
    # instead of replaying its captured graph, so this pass is not the timed one).
    R.profile_enable(True)
    t_prof = time.perf_counter()
    for i in range(args.steps):
        one_step(i)
    torch.cuda.synchronize()
    t_prof = time.perf_counter() - t_prof
    kern = R.profile_read_kernels()
    R.profile_enable(False)
    # the roofline's launches: the iterations that ran (those after the stopping
    # condition exit early and are reported apart)
    n_exec = max(kern["executed_launches"], 1)
    sweep_avg_s = kern["executed"]["sweep"] / 1e3 / n_exec
    iter_avg_s = (kern["executed"]["sweep"] + kern["executed"]["hk_rows"]) / 1e3 / n_exec

    T = float(np.median(per_step))
    it_mean = iters / args.steps
    u_mean = updates / max(iters, 1)                      # updates per executed iteration
    B_it = iteration_bytes(N, M, DD, K, u_mean)
    B_total = it_mean * B_it + 4.0 * DD * N              # per decode, with the ingest read
    value = DD * N * iters / t_total
    achieved = B_it / sweep_avg_s / 1e9
    large = (M + 31) // 32 > 12288
    packed = DD <= 4 or M <= 2 ** (128 // DD)
    metric = METRIC if (N, DD) == (2 ** 20, 7) else f"Robust-l0 nnz(A)-updates/s and time-to-solution, n={N} d={DD}"
    if variant == 1:
        metric = metric.replace("Robust-l0", "Robust-l0-quantised", 1)
    if adaptive:
        metric = metric.replace("Robust-l0", "Robust-l0 (adaptive_k)", 1)
    if laws != ("gaussian", "gaussian"):
        metric = metric.replace("Robust-l0", f"Robust-l0 ({laws[0]} signal, {laws[1]} noise)", 1)
    out = {
        "metric": metric,
        "value": value,
        "unit": "nnz(A)-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_total / args.steps,
        "time_to_solution_ms_median": 1e3 * T,
        "decode_device_ms_median": float(np.median(dev_ms)),
        "iterations_per_step": it_mean,
        "rel_l2_err_median": float(np.median(rel)),
        "rel_l2_err_max": float(np.max(rel)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "n": N, "m": M, "d": DD, "k": K, "snr_db": SNR, "seeds": seeds,
                   "scores": "quantised" if variant == 1 else "continuous", "adaptive_k": adaptive,
                   "laws": {"signal": laws[0], "noise": laws[1]},
                   "setup": ("one untimed decode per instance captures its graph before the warm-up; "
                             "y_hat and x_hat are fixed device buffers; the host constants of the "
                             "parameter set (score tables, thresholds) are computed once and cached")
                            if not adaptive else
                            ("eager launches; after every iteration the host reads back the decision and "
                             "k_0 and, after an accepted one, recomputes the score tables and thresholds "
                             "(inside the timed region)")},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": sweep_traffic() if (N, M, DD) == (2 ** 20, 104857, 7) else None,
                     "kernel": f"k_sweep<{DD}, {'true' if large else 'false'}, {'true' if packed else 'false'}, false>",
                     "bytes_per_launch": B_it,
                     "bytes_model": "B_it = 4dn + 28m + 16dk + 12(k + u) per loop iteration, u = mean updates "
                                    f"per executed iteration ({u_mean:.1f}); one sweep launch per iteration",
                     "avg_launch_us": sweep_avg_s * 1e6,
                     "launches": kern["executed_launches"],
                     "frac_iteration": B_it / iter_avg_s / 1e9 / HBM_PEAK_GBS,
                     "iteration_us": iter_avg_s * 1e6,
                     "frac_end_to_end": B_total / T / 1e9 / HBM_PEAK_GBS,
                     "bytes_per_decode": B_total},
        "kernels_us_per_iteration": {k: 1e3 * v / n_exec for k, v in kern["executed"].items()},
        "kernels_us_per_launch_all": {k: 1e3 * v / max(kern["all_launches"], 1) for k, v in kern["all"].items()},
        "launches_all": kern["all_launches"],
        "ms_per_step_eager_profiled": 1e3 * t_prof / args.steps,
    }
    if cpu:
        del insts
        out["cpu_baseline"] = cpu_baseline(N, M, K, DD, sigma, seed_ids[:8], variant=variant, adaptive=adaptive,
                                           laws=laws)
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seeds", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--phase-n", type=int, default=2 ** 22, help="n of the phase-transition ladders")
    ap.add_argument("--workload", choices=["headline", "batched", "learned", "large", "quantised", "phase",
                                           "adaptive", "laplace"],
                    default="headline",
                    help="batched: 512 uneven instances in one persistent launch, against "
                         "sequential single decodes of the same instances")
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--records", default="",
                    help="single-decode workloads: write one JSON line per decoded instance (seed, sizes, SNR, "
                         "iterations, device time, throughput, bytes, relative error, l1 success, support found) "
                         "to this file")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy (3 times), the "
                         "reference kernel that scales HBM byte counters")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the decoder has no multi-GPU path",
                          "n_gpus": args.gpus}))
        return 2

    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "phase":
        return bench_phase(args)
    if args.workload == "learned":
        return bench_learned(args)

    if args.workload == "large":
        return bench_decode(args, 2 ** 24, 2 ** 21, 2 ** 18, 8, 3, min(args.seeds, 3),
                            "Robust-l0 decode of y_hat = A x + eta, n=2^24, m=2^21, d=8, k=2^18 N(0,1) "
                            "nonzeros, SNR 40 dB; step = sketch + decode", cpu=False)
    if args.workload == "quantised":
        return bench_decode(args, N, M, K, DD, 6, args.seeds,
                            "Robust-l0-quantised decode of y_hat = A x + eta, n=2^20, m=104857, d=7, "
                            "k=10485 N(0,1) nonzeros, SNR 40 dB; step = sketch + decode",
                            cpu=not args.no_cpu_baseline, variant=1)
    if args.workload == "laplace":
        return bench_decode(args, N, M, K, DD, 2, args.seeds,
                            "Robust-l0 decode of y_hat = A x + eta with Laplace signal (std 1) and Laplace noise, "
                            "n=2^20, m=104857, d=7, k=10485, SNR 40 dB; posteriors of the general-distribution "
                            "theorem tabulated by the library; step = sketch + decode",
                            cpu=not args.no_cpu_baseline, laws=("laplace", "laplace"))
    if args.workload == "adaptive":
        return bench_decode(args, N, M, K, DD, 2, args.seeds,
                            "Robust-l0 decode with adaptive_k of y_hat = A x + eta, n=2^20, m=104857, d=7, "
                            "k=10485 N(0,1) nonzeros, SNR 40 dB; step = sketch + decode (eager launches, "
                            "one host round trip per iteration)",
                            cpu=not args.no_cpu_baseline, adaptive=1)
    return bench_decode(args, N, M, K, DD, 2, args.seeds,
                        "Robust-l0 decode of y_hat = A x + eta, n=2^20, m=104857, d=7, "
                        "k=10485 N(0,1) nonzeros, SNR 40 dB; step = sketch + decode",
                        cpu=not args.no_cpu_baseline)


if __name__ == "__main__":
    sys.exit(main())
