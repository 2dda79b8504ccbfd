"""Decoding under non-Gaussian signal and noise laws on the GPU against the oracle, through
the C-ABI.

The oracle's score tables for Laplace and Gaussian laws (Thm "Probabilities for general
signal and noise distributions"; stored by tests/golden/make_tables.py from
oracle.general) are handed to the library (rl0_params.tables) and to the oracle decode
alike, so the bar is bitwise: x_hat and the loop statistics, continuous and quantised
scores, single and batched decodes.  The library's own tables for the same laws (another
numerical route, whose float32 tables equal the oracle's entry by entry:
test_capi_general.py) then give the oracle's decodes too."""
import os

import numpy as np
import pytest

from oracle import decoder as D
from oracle import scores as S
from paper_1704_09012_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_1704_09012_amd.rl0")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
SMALL = "tables_n1024_m256_k25_d7_snr40_laplace_laplace.npz"
MID = sorted(f for f in os.listdir(GOLDEN) if f.startswith("tables_n65536")) if os.path.isdir(GOLDEN) else []


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def load(name):
    g = np.load(os.path.join(GOLDEN, name))
    packed = R.pack_tables(g["Tz"], g["Te"], g["inv_h_z"], g["inv_h_e"])
    tables = (S.Table(g["Tz"], np.float32(g["inv_h_z"]), float(g["R_z"])),
              S.Table(g["Te"], np.float32(g["inv_h_e"]), float(g["R_e"])))
    return g, packed, tables


def instance(g, seed):
    n, m, k, d = int(g["n"]), int(g["m"]), int(g["k"]), int(g["d"])
    sig = float(g["sigma"])
    sl, nl = str(g["signal"]), str(g["noise"])
    inst = I.draw_instance(n, m, k, d, sig, seed, kind=sl, noise_kind=nl)
    y = D.measure(inst.A_cols[inst.support], inst.values, inst.eta, m)
    return inst, y, sig, sl, nl


def assert_same_decode(xg, stg, res):
    assert np.array_equal(xg, res.x_hat)
    assert stg["iterations"] == res.iterations
    assert stg["accepted"] == res.accepted
    assert stg["l1_final_fx"] == res.L_hat
    assert stg["converged"] == int(res.converged)
    assert stg["updates_total"] == res.updates_total
    assert stg["fx_inexact_x"] == res.fx_inexact_x


def decode_both(g, packed, tables, seed, variant):
    inst, y, sig, sl, nl = instance(g, seed)
    n, m, k, d = inst.n, inst.m, inst.k, inst.d
    xg, stg = R.decode(dev(inst.A_cols), dev(y), sigma=sig, k=k, variant=variant, signal_law=sl, noise_law=nl,
                       tables=packed)
    C = D.make_constants(n, m, d, k, sig, variant=variant, signal=sl, noise=nl, tables=tables)
    return inst, y, host(xg), stg, D.decode(inst.A_cols, y, C)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("seed", range(5))
def test_given_tables_small_bitwise(seed, variant):
    g, packed, tables = load(SMALL)
    print(f"laplace laws n=1024 seed={seed} variant={variant}", flush=True)
    _, _, xg, stg, res = decode_both(g, packed, tables, 500 + seed, variant)
    assert_same_decode(xg, stg, res)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("name", MID)
def test_given_tables_mid_size_bitwise(name, variant):
    g, packed, tables = load(name)
    print(f"{name} variant={variant}", flush=True)
    inst, _, xg, stg, res = decode_both(g, packed, tables, 61, variant)
    assert_same_decode(xg, stg, res)
    x = inst.x_dense()
    print("  rel err", float(np.linalg.norm(xg - x) / np.linalg.norm(x)), "iterations", res.iterations, flush=True)


def test_given_tables_in_a_batch():
    g, packed, tables = load(MID[0])
    probs, refs = [], []
    for seed in (71, 72, 73):
        inst, y, sig, sl, nl = instance(g, seed)
        A, yt = dev(inst.A_cols), dev(y)
        x = torch.empty(inst.n, dtype=torch.float32, device="cuda")
        p = R.params_default(inst.n, inst.m, inst.d, inst.k, sig, signal_law=sl, noise_law=nl, tables=packed)
        probs.append({"A": A, "y": yt, "out": x, "params": p})
        C = D.make_constants(inst.n, inst.m, inst.d, inst.k, sig, signal=sl, noise=nl, tables=tables)
        refs.append(D.decode(inst.A_cols, y, C))
    stats = R.decode_batched(probs)
    for pr, st, res in zip(probs, stats, refs):
        assert np.array_equal(host(pr["out"]), res.x_hat)
        assert st["l1_final_fx"] == res.L_hat and st["iterations"] == res.iterations


@pytest.mark.parametrize("name", MID)
def test_library_tables_decode_like_the_oracle(name):
    """The library's own tables for the laws (no given tables): they equal the oracle's
    entry by entry (checked here again through rl0_compute_constants), so the decode is
    bitwise the oracle's; it is also repeatable and keeps at most k nonzeros."""
    g, packed, tables = load(name)
    inst, y, sig, sl, nl = instance(g, 61)
    p = R.params_default(inst.n, inst.m, inst.d, inst.k, sig, signal_law=sl, noise_law=nl)
    c = R.compute_constants(p, inst.n, inst.m, inst.d)
    assert np.array_equal(c.table_z, g["Tz"]) and np.array_equal(c.table_e, g["Te"])
    A, yt = dev(inst.A_cols), dev(y)
    x1, st1 = R.decode(A, yt, params=p)
    x2, st2 = R.decode(A, yt, params=p)
    a = host(x1)
    assert np.array_equal(a, host(x2)) and R.stats_subset(st1) == R.stats_subset(st2)
    assert np.count_nonzero(a) <= inst.k
    C = D.make_constants(inst.n, inst.m, inst.d, inst.k, sig, signal=sl, noise=nl, tables=tables)
    assert_same_decode(a, st1, D.decode(inst.A_cols, y, C))


def _golden_l():
    if not os.path.isdir(GOLDEN):
        return []
    return sorted(f for f in os.listdir(GOLDEN) if f.startswith("decodel_") and f.endswith(".npz"))


@pytest.mark.parametrize("fname", _golden_l())
def test_laplace_laws_full_size_against_stored_oracle(fname):
    """n = 2^20, m = n/10, k = m/10, d = 7, Laplace signal and noise at 40 dB: the oracle's
    decode with its tables of those laws (tests/golden/make_golden.py), against the
    library's decode with the same given tables and with its own tables, bitwise."""
    g = np.load(os.path.join(GOLDEN, fname))
    n, m, k, d = int(g["n"]), int(g["m"]), int(g["k"]), int(g["d"])
    sig = float(g["sigma"])
    sl, nl = str(g["signal"]), str(g["noise"])
    tab = np.load(os.path.join(GOLDEN, f"tables_n{n}_m{m}_k{k}_d{d}_snr{int(g['snr'])}_{sl}_{nl}.npz"))
    packed = R.pack_tables(tab["Tz"], tab["Te"], tab["inv_h_z"], tab["inv_h_e"])
    print(f"golden {fname}", flush=True)
    inst = I.draw_instance(n, m, k, d, sig, int(g["seed"]), kind=sl, noise_kind=nl)
    y = D.measure(inst.A_cols[inst.support], inst.values, inst.eta, m)
    A, yt = dev(inst.A_cols), dev(y)
    ref = np.zeros(n, np.float32)
    ref[g["support"]] = g["values"]
    for kw in (dict(tables=packed), {}):
        xg, stg = R.decode(A, yt, sigma=sig, k=k, signal_law=sl, noise_law=nl, **kw)
        assert np.array_equal(host(xg), ref)
        assert stg["iterations"] == int(g["iterations"]) and stg["accepted"] == int(g["accepted"])
        assert stg["l1_final_fx"] == int(g["L_hat"]) and stg["updates_total"] == int(g["updates_total"])
