"""The library's posteriors for non-Gaussian laws (rl0_params.signal_law / noise_law) and
given score tables (rl0_params.tables), on the host: the tables against the oracle's
(oracle.general, which sums the theorem's series in direct space; the library inverts
characteristic functions) at spot nodes and, for the stored full oracle tables, entry by
entry; the stopping tolerance; the checks on given tables."""
import math

import numpy as np
import pytest

from oracle import general as G

R = pytest.importorskip("paper_1704_09012_amd.rl0")

NODES = list(range(0, 4097, 256)) + [1, 2, 4095]


@pytest.mark.parametrize("sl,nl,d,k,m,sig,ss", [
    ("laplace", "laplace", 7, 80, 1024, 0.01, 1.0),
    ("gaussian", "laplace", 12, 20, 1000, 0.001, 1.0),
    ("laplace", "gaussian", 7, 80, 1024, 0.01, 1.0),
    ("laplace", "laplace", 3, 300, 1000, 0.1, 2.0),
])
def test_general_tables_match_the_oracle(sl, nl, d, k, m, sig, ss):
    sig = float(np.float32(sig))
    p = R.params_default(4096, m, d, k, sig, signal_law=sl, noise_law=nl, sigma_signal=ss)
    c = R.compute_constants(p, 4096, m, d)
    rho = k / m
    for kind, T, inv_h, rng in (("z", c.table_z, c.inv_h_z, c.range_z), ("e", c.table_e, c.inv_h_e, c.range_e)):
        ref = G.build_table(kind, d, rho, (sl, ss), (nl, sig), nodes=NODES)
        assert abs(rng - ref.R) <= 1e-12 * ref.R                  # the same q in R = q h0
        assert inv_h == ref.inv_h
        # the two routes agree to about 1e-9; after rounding to float32 at most one unit
        assert np.max(np.abs(T[NODES].astype(np.float64) - ref.T[NODES])) <= 2.0 ** -24
        assert np.all(np.diff(T) <= 0) and T[0] == 1.0
    assert c.tol == G.noise_l1_mean(m, (nl, sig))


def _golden_tables():
    import os
    g = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    return sorted(os.path.join(g, f) for f in os.listdir(g) if f.startswith("tables_")) if os.path.isdir(g) else []


@pytest.mark.parametrize("path", _golden_tables(), ids=lambda p: p.split("/")[-1])
def test_general_tables_equal_the_stored_oracle_tables(path):
    """Every entry of the library's tables against the oracle's full tables (written by
    tests/golden/make_tables.py): the two numerical routes agree to about 1e-12, so even
    their float32 roundings coincide."""
    g = np.load(path)
    n, m, k, d = int(g["n"]), int(g["m"]), int(g["k"]), int(g["d"])
    p = R.params_default(n, m, d, k, float(g["sigma"]), signal_law=str(g["signal"]), noise_law=str(g["noise"]))
    c = R.compute_constants(p, n, m, d)
    assert np.array_equal(c.table_z, g["Tz"]) and np.array_equal(c.table_e, g["Te"])
    assert c.inv_h_z == g["inv_h_z"] and c.inv_h_e == g["inv_h_e"]
    assert c.range_z == float(g["R_z"]) and c.range_e == float(g["R_e"])


@pytest.mark.parametrize("sl,nl", [("laplace", "laplace"), ("gaussian", "laplace"), ("laplace", "gaussian")])
def test_general_tables_shape(sl, nl):
    sig = float(np.float32(0.02))
    c = R.compute_constants(R.params_default(8192, 2048, 9, 150, sig, signal_law=sl, noise_law=nl), 8192, 2048, 9)
    for T, inv_h, rng, v0 in ((c.table_z, c.inv_h_z, c.range_z, sig * sig), (c.table_e, c.inv_h_e, c.range_e, 2 * sig * sig)):
        q = rng / (math.sqrt(v0) / 8)
        assert abs(q - round(q)) < 1e-9 and round(q) >= 8
        assert inv_h == np.float32(4096 / rng)
        assert T[0] == 1.0 and np.all(np.diff(T) <= 0) and 0.0 <= T[-1] < 2.0 ** -27 and T[4096 // 8] > 0


def test_gaussian_laws_keep_the_paper_tables():
    # both laws Gaussian: eq:pz_approx, exactly as without the fields
    a = R.compute_constants(R.params_default(4096, 1024, 7, 80, 0.01), 4096, 1024, 7)
    b = R.compute_constants(R.params_default(4096, 1024, 7, 80, 0.01, signal_law="gaussian", noise_law="gaussian"),
                            4096, 1024, 7)
    assert np.array_equal(a.table_z, b.table_z) and np.array_equal(a.table_e, b.table_e) and a.tol == b.tol


def _tables():
    Tz = np.linspace(1.0, 0.0, 4097).astype(np.float32)
    Te = (np.linspace(1.0, 0.0, 4097) ** 2).astype(np.float32)
    return R.pack_tables(Tz, Te, 4096 / 0.07, 4096 / 0.1)


def test_given_tables_are_used_as_they_are():
    T = _tables()
    p = R.params_default(4096, 1024, 7, 80, 0.01, tables=T, noise_law="laplace")
    c = R.compute_constants(p, 4096, 1024, 7)
    assert np.array_equal(c.table_z, T[:4097]) and np.array_equal(c.table_e, T[4097:8194])
    assert c.inv_h_z == T[-2] and c.inv_h_e == T[-1]
    assert c.tol == 1024 * np.float32(0.01) / math.sqrt(2.0)
    # the outer-test thresholds follow the given z-table: |r| >= tau  <=>  1 - Tz(|r|) >= t
    one = np.float32(1.0)
    for t, tau in zip(c.t[:5], c.tau[:5]):
        assert np.float32(one - R_lookup(c.table_z, c.inv_h_z, tau)) >= t
        if tau > 0:
            lo = np.nextafter(np.float32(tau), np.float32(0))
            assert np.float32(one - R_lookup(c.table_z, c.inv_h_z, lo)) < t


def R_lookup(T, inv_h, a):
    u = np.float32(np.float32(a) * inv_h)
    if not u < 4096:
        return np.float32(0)
    i = int(u)
    f = np.float32(u - np.float32(i))
    return np.float32(T[i] + np.float32(f * np.float32(T[i + 1] - T[i])))


@pytest.mark.parametrize("spoil", ["start", "above_one", "increasing", "nan", "inv_h_zero", "inv_h_inf"])
def test_bad_given_tables_are_rejected(spoil):
    T = _tables()
    if spoil == "start":
        T[0] = np.float32(0.99)
    elif spoil == "above_one":
        T[4097 + 3] = np.float32(1.5)
    elif spoil == "increasing":
        T[100] = T[99] + np.float32(1e-3)
    elif spoil == "nan":
        T[2000] = np.nan
    elif spoil == "inv_h_zero":
        T[-2] = 0.0
    else:
        T[-1] = np.inf
    with pytest.raises(R.Rl0Error) as e:
        R.compute_constants(R.params_default(4096, 1024, 7, 80, 0.01, tables=T), 4096, 1024, 7)
    assert e.value.code == -1 and "tables" in str(e.value)


def test_laws_are_checked():
    with pytest.raises(R.Rl0Error):
        R.compute_constants(R.params_default(4096, 1024, 7, 80, 0.01, noise_law=2), 4096, 1024, 7)
    with pytest.raises(R.Rl0Error) as e:
        R.compute_constants(R.params_default(4096, 1024, 7, 80, 0.01, noise_law="laplace", adaptive_k=1),
                            4096, 1024, 7)
    assert "adaptive_k" in str(e.value)
    with pytest.raises(R.Rl0Error):
        R.compute_constants(R.params_default(4096, 1024, 7, 80, 0.01, tables=_tables(), adaptive_k=1), 4096, 1024, 7)
