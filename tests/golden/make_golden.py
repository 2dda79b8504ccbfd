"""Write the oracle's full-size decodes used by the GPU parity tests.

    python tests/golden/make_golden.py [--jobs 6]

Only the CPU oracle (oracle/) and the seeded instance generator are called.  Each file
holds, for one seeded instance of the n = 2^20, m = n/10, k = m/10, d = 7 workload
(Gaussian N(0,1) signal, Gaussian noise at the stated SNR), the oracle's recovered
x_hat (support and values) and its loop statistics.
"""
from __future__ import annotations

import argparse
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import decoder as D  # noqa: E402
from paper_1704_09012_amd import instances as I  # noqa: E402

N = 2 ** 20
M = N // 10
K = M // 10
DD = 7
SNRS = (20, 40, 60)
SEEDS_PER_SNR = 2


def case_name(snr: int, i: int) -> str:
    return f"decode_n1048576_d7_snr{snr}_i{i}.npz"


def one(args):
    snr_idx, snr, i = args
    seed = I.seed_for(2, snr_idx, i)
    sig = float(np.float32(I.sigma_for_snr(snr, N, M, K, DD)))
    inst = I.draw_instance(N, M, K, DD, sig, seed)
    x = inst.x_dense()
    y = D.measure(inst.A_cols, x, inst.eta, M)
    C = D.make_constants(N, M, DD, K, sig)
    res = D.decode(inst.A_cols, y, C)
    supp = np.nonzero(res.x_hat)[0].astype(np.int32)
    path = os.path.join(HERE, case_name(snr, i))
    np.savez_compressed(path, n=N, m=M, k=K, d=DD, snr=snr, seed=seed, sigma=np.float32(sig),
                        support=supp, values=res.x_hat[supp].astype(np.float32),
                        iterations=res.iterations, accepted=res.accepted, L_hat=np.int64(res.L_hat),
                        converged=int(res.converged), updates_total=res.updates_total)
    err = float(np.linalg.norm(res.x_hat - x) / np.linalg.norm(x))
    return path, res.iterations, res.accepted, err


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=6)
    a = ap.parse_args()
    work = [(si, snr, i) for si, snr in enumerate(SNRS) for i in range(SEEDS_PER_SNR)]
    with ProcessPoolExecutor(a.jobs) as ex:
        for path, it, acc, err in ex.map(one, work):
            print(os.path.basename(path), "iterations", it, "accepted", acc, "rel_l2_vs_truth", f"{err:.3e}", flush=True)


if __name__ == "__main__":
    main()
