"""Write the oracle's full-size decodes used by the GPU parity tests.

    python tests/golden/make_golden.py [--jobs 6] [--only NAME_PREFIX]

Only the CPU oracle (oracle/) and the seeded instance generator are called.  Each file
holds, for one seeded instance (Gaussian N(0,1) signal, Gaussian noise at the stated
SNR), the oracle's recovered x_hat (support and values) and its loop statistics.  The
workloads:
  * n = 2^20, m = n/10, k = m/10, d = 7 at 20, 40 and 60 dB, five seeds each;
  * n = 2^20, m = n/2, k = m/8, d = 8 at 40 dB: the large workload's d and k/m at 1/16 of
    its n, with m above 393216 rows (the decoder's large-m paths);
  * n = 2^21, m = n/2, a signal of m/8 nonzeros decoded with k = m/16, d = 8 at 40 dB:
    every iteration then has more candidates than k, so H_k selects on the large-m
    path, with boundary buckets of about 2 100 and 5 000 entries;
  * the large workload itself: n = 2^24, m = 2^21, k = 2^18, d = 8 at 40 dB (sigma_n =
    0.01), seed 30100.  Its oracle decode takes about half an hour on one core;
  * the quantised variant (files decodeq_*) at n = 2^20, m = n/10, k = m/10, d = 7 at 20,
    40 and 60 dB, one seed each (c from eq:finetune_c_quant: 0.05, 20 iterations);
  * Laplace signal and noise laws (decodel_*): n = 2^20, m = n/10, k = m/10, d = 7 at 40 dB,
    decoded with the oracle's tables of those laws (make_tables.py writes them first);
  * Alg. 1's adaptive_k branch (files decodea_*): n = 2^20, m = n/10, k = m/10, d = 7 at
    20, 40 and 60 dB, the quantised variant at 40 dB (decodeaq_*), and n = 2^20, m = n/2,
    k = m/8, d = 8 at 40 dB (m above 393216); these also store the last k_0;
  * the batched workload (batch512_seed0.npz): the 512 uneven instances of
    instances.draw_batch(512, 0, 7) (n log-uniform in [2^12, 2^18], m/n in [0.05, 0.5],
    k/m in [0.05, 0.3], 20 to 60 dB), every one decoded by the oracle.  Per instance the
    loop statistics and the SHA-256 of x_hat's support (int32, ascending) followed by its
    values (float32), both little-endian: a bitwise comparison without storing 10^6
    nonzeros; batch512q_seed0.npz holds the same batch decoded with the quantised scores;
  * the headline workload's twenty seeds per SNR (c2digests_n1048576_d7_20seeds.npz):
    n = 2^20, m = n/10, k = m/10, d = 7 at 20, 40 and 60 dB, seeds seed_for(2, snr index,
    i) for i < 20 (the first five are also stored whole above); per instance the loop
    statistics and the same SHA-256 of x_hat;
  * the same for the quantised variant (c2qdigests_*: twenty seeds per SNR, seeds
    seed_for(6, snr index, i)), for Laplace signal and noise laws at 40 dB with the
    oracle's tables of those laws (c2ldigests_*: ten seeds, seed_for(9, 1, i)), for the
    adaptive_k branch (c2adigests_*: ten seeds per SNR, seed_for(7, snr index, i)) and for
    the large-m shape n = 2^20, m = n/2, k = n/16, d = 8 at 40 dB (lmdigests_*: eight
    seeds, seed_for(3, 1, 10 + i)).
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
from oracle import scores as S  # noqa: E402
from paper_1704_09012_amd import instances as I  # noqa: E402

N = 2 ** 20
M = N // 10
K = M // 10
DD = 7
SNRS = (20, 40, 60)
SEEDS_PER_SNR = 5


def case_name(snr: int, i: int) -> str:
    return f"decode_n1048576_d7_snr{snr}_i{i}.npz"


# (file name, n, m, k of the signal, d, snr, seed, k of the decoder[, variant[, adaptive_k[, laws]]]);
# laws = (signal law, noise law), decoded with the oracle's tables of those laws stored by
# make_tables.py
CASES = [(case_name(snr, i), N, M, K, DD, snr, I.seed_for(2, si, i), K)
         for si, snr in enumerate(SNRS) for i in range(SEEDS_PER_SNR)]
CASES += [(f"decodeq_n1048576_d7_snr{snr}_i0.npz", N, M, K, DD, snr, I.seed_for(6, si, 0), K, 1)
          for si, snr in enumerate(SNRS)]
CASES.append(("decode_n1048576_m524288_d8_snr40_i0.npz", N, N // 2, N // 16, 8, 40, I.seed_for(3, 1, 10), N // 16))
CASES.append(("decode_n2097152_m1048576_d8_snr40_kdec65536_i0.npz", 2 * N, N, N // 8, 8, 40, I.seed_for(3, 1, 10),
              N // 16))
CASES += [(f"decodea_n1048576_d7_snr{snr}_i0.npz", N, M, K, DD, snr, I.seed_for(7, si, 0), K, 0, 1)
          for si, snr in enumerate(SNRS)]
CASES.append(("decodeaq_n1048576_d7_snr40_i0.npz", N, M, K, DD, 40, I.seed_for(8, 1, 0), K, 1, 1))
CASES.append(("decodea_n1048576_m524288_d8_snr40_i0.npz", N, N // 2, N // 16, 8, 40, I.seed_for(7, 1, 10), N // 16,
              0, 1))
CASES.append(("decodel_n1048576_d7_snr40_laplace_laplace_i0.npz", N, M, K, DD, 40, I.seed_for(9, 1, 0), K, 0, 0,
              ("laplace", "laplace")))
CASES.append(("decode_n16777216_m2097152_d8_snr40_i0.npz", 2 ** 24, 2 ** 21, 2 ** 18, 8, 40, I.seed_for(3, 1, 0),
              2 ** 18))


def one(case):
    name, n, m, k, d, snr, seed, k_dec = case[:8]
    variant = case[8] if len(case) > 8 else 0
    adaptive = case[9] if len(case) > 9 else 0
    laws = case[10] if len(case) > 10 else ("gaussian", "gaussian")
    sig = float(np.float32(I.sigma_for_snr(snr, n, m, k, d)))
    inst = I.draw_instance(n, m, k, d, sig, seed, kind=laws[0], noise_kind=laws[1])
    x = inst.x_dense()
    # only the support's columns contribute to A x
    y = D.measure(inst.A_cols[inst.support], inst.values, inst.eta, m)
    tables = None
    if laws != ("gaussian", "gaussian"):
        g = np.load(os.path.join(HERE, f"tables_n{n}_m{m}_k{k_dec}_d{d}_snr{snr}_{laws[0]}_{laws[1]}.npz"))
        tables = (S.Table(g["Tz"], np.float32(g["inv_h_z"]), float(g["R_z"])),
                  S.Table(g["Te"], np.float32(g["inv_h_e"]), float(g["R_e"])))
    C = D.make_constants(n, m, d, k_dec, sig, variant=variant, adaptive_k=adaptive, signal=laws[0], noise=laws[1],
                         tables=tables)
    res = D.decode(inst.A_cols, y, C)
    supp = np.nonzero(res.x_hat)[0].astype(np.int32)
    path = os.path.join(HERE, name)
    np.savez_compressed(path, n=n, m=m, k=k, k_decode=k_dec, d=d, snr=snr, seed=seed, sigma=np.float32(sig),
                        variant=variant, adaptive_k=adaptive, k_post=np.float64(res.k_post),
                        signal=laws[0], noise=laws[1],
                        fx_inexact_y=res.fx_inexact_y, fx_inexact_x=res.fx_inexact_x,
                        support=supp, values=res.x_hat[supp].astype(np.float32),
                        iterations=res.iterations, accepted=res.accepted, L_hat=np.int64(res.L_hat),
                        converged=int(res.converged), updates_total=res.updates_total)
    err = float(np.linalg.norm(res.x_hat - x) / np.linalg.norm(x))
    return path, res.iterations, res.accepted, err


BATCH = (512, 0, 7)   # count, seed, d of the batched workload
BATCH_FILE = "batch512_seed0.npz"
BATCH_FILES = {BATCH_FILE: 0, "batch512q_seed0.npz": 1}   # file -> variant (1: quantised scores)


def batch_one(job):
    i, variant = job
    count, seed, d = BATCH
    inst = I.batch_member(I.draw_batch_shapes(count, seed, d), seed, i, d)
    y = D.measure(inst.A_cols[inst.support], inst.values, inst.eta, inst.m)
    res = D.decode(inst.A_cols, y, D.make_constants(inst.n, inst.m, d, inst.k, inst.sigma, variant=variant))
    supp = np.nonzero(res.x_hat)[0].astype(np.int32)
    stats = (res.iterations, res.accepted, res.L_hat, int(res.converged), res.updates_total, res.fx_inexact_x)
    return i, supp, res.x_hat[supp].astype(np.float32), stats


def write_batch(jobs: int, name: str = BATCH_FILE) -> None:
    variant = BATCH_FILES[name]
    count = BATCH[0]
    parts = [None] * count
    # the largest instances first, so that none of them starts last
    shapes = I.draw_batch_shapes(*BATCH)
    order = sorted(range(count), key=lambda i: -shapes[i][0] * shapes[i][2] / shapes[i][1])
    with ProcessPoolExecutor(jobs) as ex:
        for i, supp, vals, stats in ex.map(batch_one, [(i, variant) for i in order]):
            parts[i] = (x_hat_digest(supp, vals), len(supp), stats)
    st = np.array([p[2] for p in parts], np.int64)
    extra = {"variant": variant} if variant else {}
    np.savez_compressed(os.path.join(HERE, name), count=count, seed=BATCH[1], d=BATCH[2], **extra,
                        digest=np.array([p[0] for p in parts]), nnz=np.array([p[1] for p in parts], np.int64),
                        iterations=st[:, 0], accepted=st[:, 1], L_hat=st[:, 2], converged=st[:, 3],
                        updates_total=st[:, 4], fx_inexact_x=st[:, 5])
    print(name, "instances", count, "nonzeros", int(sum(p[1] for p in parts)), "converged",
          int(st[:, 3].sum()), flush=True)


def x_hat_digest(support, values) -> str:
    """SHA-256 of the support (int32) then the values (float32), little-endian."""
    import hashlib

    h = hashlib.sha256(np.ascontiguousarray(support, dtype="<i4").tobytes())
    h.update(np.ascontiguousarray(values, dtype="<f4").tobytes())
    return h.hexdigest()


C2_FILE = "c2digests_n1048576_d7_20seeds.npz"
GAUSS = ("gaussian", "gaussian")
# digest sets: file -> (shape (n, m, k, d), SNRs, seeds per SNR, variant, adaptive_k, laws,
# seed_for's config, first seed index)
DIGEST_SETS = {
    C2_FILE: ((N, M, K, DD), SNRS, 20, 0, 0, GAUSS, 2, 0),
    "c2qdigests_n1048576_d7_20seeds.npz": ((N, M, K, DD), SNRS, 20, 1, 0, GAUSS, 6, 0),
    "c2ldigests_n1048576_d7_snr40_10seeds.npz": ((N, M, K, DD), (40,), 10, 0, 0, ("laplace", "laplace"), 9, 0),
    "c2adigests_n1048576_d7_10seeds.npz": ((N, M, K, DD), SNRS, 10, 0, 1, GAUSS, 7, 0),
    "lmdigests_n1048576_m524288_d8_snr40_8seeds.npz": ((N, N // 2, N // 16, 8), (40,), 8, 0, 0, GAUSS, 3, 10),
}


def digest_one(job):
    name, snr, i = job
    (n, m, k, d), _, _, variant, adaptive, laws, cfg, i0 = DIGEST_SETS[name]
    si = SNRS.index(snr)
    sig = float(np.float32(I.sigma_for_snr(snr, n, m, k, d)))
    inst = I.draw_instance(n, m, k, d, sig, I.seed_for(cfg, si, i0 + i), kind=laws[0], noise_kind=laws[1])
    y = D.measure(inst.A_cols[inst.support], inst.values, inst.eta, m)
    tables = None
    if laws != GAUSS:
        g = np.load(os.path.join(HERE, f"tables_n{n}_m{m}_k{k}_d{d}_snr{snr}_{laws[0]}_{laws[1]}.npz"))
        tables = (S.Table(g["Tz"], np.float32(g["inv_h_z"]), float(g["R_z"])),
                  S.Table(g["Te"], np.float32(g["inv_h_e"]), float(g["R_e"])))
    C = D.make_constants(n, m, d, k, sig, variant=variant, adaptive_k=adaptive, signal=laws[0], noise=laws[1],
                         tables=tables)
    res = D.decode(inst.A_cols, y, C)
    supp = np.nonzero(res.x_hat)[0].astype(np.int32)
    stats = (res.iterations, res.accepted, res.L_hat, int(res.converged), res.updates_total, res.fx_inexact_x)
    return name, snr, i, x_hat_digest(supp, res.x_hat[supp].astype(np.float32)), stats


def write_digest_sets(names, jobs: int) -> None:
    work = [(nm, snr, i) for nm in names for snr in DIGEST_SETS[nm][1] for i in range(DIGEST_SETS[nm][2])]
    # the slowest instances first (the adaptive branch rebuilds its tables, the large-m shape)
    work.sort(key=lambda w: -(DIGEST_SETS[w[0]][4] * 4 + (DIGEST_SETS[w[0]][0][1] > M)))
    out = {nm: ({}, {}) for nm in names}
    with ProcessPoolExecutor(jobs) as ex:
        for nm, snr, i, dg, stats in ex.map(digest_one, work):
            out[nm][0][(snr, i)] = dg
            out[nm][1][(snr, i)] = stats
    for nm in names:
        (n, m, k, d), snrs, seeds, variant, adaptive, laws, cfg, i0 = DIGEST_SETS[nm]
        digest = np.array([[out[nm][0][(snr, i)] for i in range(seeds)] for snr in snrs], dtype="U64")
        st = np.array([[out[nm][1][(snr, i)] for i in range(seeds)] for snr in snrs], np.int64)
        extra = {} if nm == C2_FILE else {"variant": variant, "adaptive_k": adaptive, "signal": laws[0],
                                          "noise": laws[1], "config": cfg, "first_seed": i0,
                                          "snr_index": np.array([SNRS.index(x) for x in snrs])}
        np.savez_compressed(os.path.join(HERE, nm), n=n, m=m, k=k, d=d, snrs=np.array(snrs), seeds=seeds,
                            digest=digest, iterations=st[..., 0], accepted=st[..., 1], L_hat=st[..., 2],
                            converged=st[..., 3], updates_total=st[..., 4], fx_inexact_x=st[..., 5], **extra)
        print(nm, "instances", digest.size, "converged", int(st[..., 3].sum()), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=6)
    ap.add_argument("--only", default="", help="write only the files whose name starts with this")
    ap.add_argument("--missing", action="store_true", help="write only the files that do not exist yet")
    a = ap.parse_args()
    for name in BATCH_FILES:
        if name.startswith(a.only) and not (a.missing and os.path.exists(os.path.join(HERE, name))):
            write_batch(a.jobs, name)
    sets = [nm for nm in DIGEST_SETS if nm.startswith(a.only)
            and not (a.missing and os.path.exists(os.path.join(HERE, nm)))]
    if sets:
        write_digest_sets(sets, a.jobs)
    work = [c for c in CASES if c[0].startswith(a.only)]
    if a.missing:
        work = [c for c in work if not os.path.exists(os.path.join(HERE, c[0]))]
    # the largest first, so that it does not start last
    work.sort(key=lambda c: -c[1] * c[4])
    with ProcessPoolExecutor(a.jobs) as ex:
        for path, it, acc, err in ex.map(one, work):
            print(os.path.basename(path), "iterations", it, "accepted", acc, "rel_l2_vs_truth", f"{err:.3e}", flush=True)


if __name__ == "__main__":
    main()
