"""Write the oracle's score tables for non-Gaussian laws used by the GPU tests.

    python tests/golden/make_tables.py [--jobs 6] [--only NAME_PREFIX]

Only the CPU oracle (oracle/general.py) is called.  Each file (tables_*.npz) holds, for
one problem shape and pair of laws (Thm "Probabilities for general signal and noise
distributions", tabulated by oracle.general.build_table), the tables T_z and T_e, their
inv_h and ranges, and the parameters they were built for: d, rho = k / m, the signal and
noise laws with their standard deviations (sigma_n is the float32 value the library is
given, so that both sides build from the same number).  The GPU tests pass these tables
to the library (rl0_params.tables) and to the oracle decode alike.
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

from oracle import general as G  # noqa: E402
from paper_1704_09012_amd import instances as I  # noqa: E402

# (file name, n, m, k, d, snr, signal law, noise law)
CASES = [
    ("tables_n1024_m256_k25_d7_snr40_laplace_laplace.npz", 1024, 256, 25, 7, 40, "laplace", "laplace"),
    ("tables_n65536_m6553_k655_d7_snr30_laplace_laplace.npz", 65536, 6553, 655, 7, 30, "laplace", "laplace"),
    ("tables_n65536_m6553_k655_d7_snr40_gaussian_laplace.npz", 65536, 6553, 655, 7, 40, "gaussian", "laplace"),
    ("tables_n65536_m6553_k655_d7_snr40_laplace_gaussian.npz", 65536, 6553, 655, 7, 40, "laplace", "gaussian"),
    # the headline shape with Laplace laws (bench.py --workload laplace, and its stored decode)
    ("tables_n1048576_m104857_k10485_d7_snr40_laplace_laplace.npz", 2 ** 20, 104857, 10485, 7, 40, "laplace",
     "laplace"),
]


def sigma_of(n, m, k, d, snr) -> float:
    return float(np.float32(I.sigma_for_snr(snr, n, m, k, d)))


def one(case):
    name, n, m, k, d, snr, sl, nl = case
    sig = sigma_of(n, m, k, d, snr)
    rho = k / m
    Tz = G.build_table("z", d, rho, (sl, 1.0), (nl, sig))
    Te = G.build_table("e", d, rho, (sl, 1.0), (nl, sig))
    path = os.path.join(HERE, name)
    np.savez_compressed(path, n=n, m=m, k=k, d=d, snr=snr, sigma=np.float32(sig), signal=sl, noise=nl,
                        Tz=Tz.T, Te=Te.T, inv_h_z=Tz.inv_h, inv_h_e=Te.inv_h, R_z=Tz.R, R_e=Te.R)
    return path


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=6)
    ap.add_argument("--only", default="", help="write only the files whose name starts with this")
    a = ap.parse_args()
    work = [c for c in CASES if c[0].startswith(a.only)]
    with ProcessPoolExecutor(a.jobs) as ex:
        for path in ex.map(one, work):
            print(os.path.basename(path), flush=True)


if __name__ == "__main__":
    main()
