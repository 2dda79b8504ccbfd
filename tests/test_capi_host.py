"""The C-ABI library on the CPU: it loads, exports every declared symbol, rejects bad
arguments before touching a device, and computes its host constants (score tables,
t-sweep, outer-test thresholds) exactly as the oracle does.  No device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import decoder as D
from oracle import scores as S
from paper_1704_09012_amd import instances as I
from paper_1704_09012_amd import rl0 as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    syms = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            syms += re.findall(r"^\s*(?:int|void|const char\*|size_t)\s+(rl0_\w+)\s*\(", text, re.M)
    return sorted(set(syms))


def test_library_exports_every_declared_symbol():
    L = R.lib()
    syms = _declared_symbols()
    assert "rl0_decode" in syms and "rl0_sketch" in syms and "rl0_step" in syms
    for s in syms:
        assert hasattr(L, s), s


def test_params_default_follow_the_paper():
    p = R.params_default(1024, 256, 7, 25, 0.01)
    assert p.k == 25 and p.alpha == 2.0 and p.series_terms == 4 and p.validate == 1 and p.c == 0.0
    assert R.compute_constants(p, 1024, 256, 7).c == 0.025      # delta = 0.25 > 0.05 (eq:finetune_c_cont)
    p = R.params_default(100000, 1000, 7, 25, 0.01)
    assert R.compute_constants(p, 100000, 1000, 7).c == 0.01    # delta = 0.01 <= 0.05


@pytest.mark.parametrize("field,value", [
    ("k", 0), ("k", 256), ("alpha", 1.0), ("alpha", 7.5), ("c", 1.0), ("c", -0.1),
    ("sigma", -1.0), ("sigma", float("nan")), ("sigma_signal", 0.0), ("series_terms", 0),
    ("max_iters", -1), ("l1_test", 2), ("posterior", 3), ("variant", 2), ("variant", -1), ("adaptive_k", 2),
    ("adaptive_k", -1), ("log", 2), ("signal_law", 5), ("wg_order", 2), ("wg_order", -1),
])
def test_bad_params_are_rejected_on_the_host(field, value):
    p = R.params_default(1024, 256, 7, 25, 0.01)
    setattr(p, field, value)
    with pytest.raises(R.Rl0Error) as e:
        R.compute_constants(p, 1024, 256, 7)
    assert e.value.code == -1


def test_unknown_parameter_names_are_rejected():
    # a misspelt override must not be set on the structure and then ignored by the library
    import torch
    with pytest.raises(KeyError):
        R.params_default(1024, 256, 7, 25, 0.01, alpah=3.0)
    A = torch.zeros((1024, 7), dtype=torch.int32)
    y = torch.zeros(256, dtype=torch.float32)
    with pytest.raises(KeyError):
        R.decode(A, y, params=R.params_default(1024, 256, 7, 25, 0.01), alpah=3.0)


def test_single_row_columns_are_rejected():
    # with d = 1 no alpha lies in (1, d], so the library refuses the problem
    p = R.params_default(3000, 900, 1, 60, 0.01)
    with pytest.raises(R.Rl0Error) as e:
        R.compute_constants(p, 3000, 900, 1)
    assert e.value.code == -1 and "alpha" in str(e.value)


def test_learned_posterior_without_weights():
    p = R.params_default(1024, 256, 7, 25, 0.01)
    p.posterior = 1
    with pytest.raises(R.Rl0Error) as e:
        R.compute_constants(p, 1024, 256, 7)
    assert e.value.code == -5


@pytest.mark.parametrize("n,m,d", [(0, 10, 2), (10, 0, 2), (10, 10, 0), (10, 10, 17), (10, 5, 6)])
def test_bad_dims_are_rejected(n, m, d):
    with pytest.raises(R.Rl0Error) as e:
        R.params_default(n, m, d, 1, 0.01)
    assert e.value.code == -1


CONFIGS = [
    (1024, 256, 7, 25, 40),
    (2 ** 20, 104857, 7, 10485, 20),
    (2 ** 20, 104857, 7, 10485, 40),
    (2 ** 20, 104857, 7, 10485, 60),
    (2 ** 24, 2 ** 21, 8, 2 ** 18, None),   # sigma = 0.01
    (4096, 150, 7, 20, 30),                 # delta <= 0.05: c = 0.01
]


@pytest.mark.parametrize("n,m,d,k,snr", CONFIGS)
def test_host_constants_equal_the_oracle(n, m, d, k, snr):
    sig = 0.01 if snr is None else I.sigma_for_snr(snr, n, m, k, d)
    sig = float(np.float32(sig))
    p = R.params_default(n, m, d, k, sig)
    hc = R.compute_constants(p, n, m, d)
    C = D.make_constants(n, m, d, k, sig)
    assert hc.n_iters == C.n_iters
    assert np.array_equal(hc.table_z, C.Tz.T) and np.array_equal(hc.table_e, C.Te.T)
    assert hc.inv_h_z == C.Tz.inv_h and hc.inv_h_e == C.Te.inv_h
    assert hc.tol == pytest.approx(C.tol, rel=1e-15)
    ts = np.array([S.t_of(i, C.c) for i in range(C.n_iters)], np.float32)
    assert np.array_equal(hc.t, ts)


@pytest.mark.parametrize("n,m,k,want", [(1024, 256, 25, 0.05), (1024, 256, 40, 0.075), (1024, 256, 60, 0.1),
                                        (10000, 400, 60, 0.01)])
def test_quantised_c_rule_on_the_host(n, m, k, want):
    """eq:finetune_c_quant through rl0_compute_constants, as the oracle takes it."""
    sig = float(np.float32(0.01))     # sigma crosses the C-ABI as float32
    p = R.params_default(n, m, 7, k, sig, variant=1)
    hc = R.compute_constants(p, n, m, 7)
    C = D.make_constants(n, m, 7, k, sig, variant=1)
    assert hc.c == want == C.c and hc.n_iters == C.n_iters
    assert np.array_equal(hc.table_z, C.Tz.T) and np.array_equal(hc.table_e, C.Te.T)


@pytest.mark.parametrize("n,m,d,k,snr", CONFIGS[:4])
def test_outer_threshold_equals_the_outer_test(n, m, d, k, snr):
    """|r| >= tau_t  <=>  fl32(1 - p_breve_z(r)) >= t, on every float near tau and at random."""
    sig = float(np.float32(I.sigma_for_snr(snr, n, m, k, d)))
    p = R.params_default(n, m, d, k, sig)
    hc = R.compute_constants(p, n, m, d)
    C = D.make_constants(n, m, d, k, sig)
    rng = np.random.Generator(np.random.PCG64(0))
    for it in range(C.n_iters):
        t = hc.t[it]
        tau = hc.tau[it]
        tb = np.float32(tau).view(np.uint32)
        near = (np.arange(-300, 300, dtype=np.int64) + int(tb)).clip(0, 0x7F800000).astype(np.uint32).view(np.float32)
        rnd = (rng.random(20000) * 10 * sig).astype(np.float32)
        a = np.concatenate([near, rnd])
        formula = (np.float32(1.0) - S.lookup(C.Tz, a)).astype(np.float32) >= t
        assert np.array_equal(a >= tau, formula), it


def test_exact_mode_constants():
    p = R.params_default(1024, 256, 7, 25, 0.0)
    hc = R.compute_constants(p, 1024, 256, 7)
    assert hc.exact and hc.tol == 0.0
    assert np.all(hc.tau == np.float32(1e-45))


# ---------------------------------------------------------------- batched: host checks

def _fake_problem(n=1000, m=200, d=7, k=10, sigma=0.01, align=0):
    p = R.Problem()
    p.A_cols = 4096 + align
    p.n, p.m, p.d = n, m, d
    p.y = 8192
    p.x_out = 16384
    R.lib().rl0_params_default(ctypes.byref(p.params), n, m, d, k, ctypes.c_float(sigma))
    return p


def test_batched_rejects_bad_instances_before_device_work():
    L = R.lib()
    arr = (R.Problem * 3)(_fake_problem(), _fake_problem(), _fake_problem())
    assert L.rl0_decode_batched(arr, -1, None, None) == -1
    assert L.rl0_decode_batched(arr, 0, None, None) == 0
    arr[1].params.alpha = 9.0
    assert L.rl0_decode_batched(arr, 3, None, None) == -1
    assert b"instance 1" in L.rl0_last_error()
    arr[1] = _fake_problem(align=4)
    assert L.rl0_decode_batched(arr, 3, None, None) == -1
    assert b"aligned" in L.rl0_last_error()
    arr[1] = _fake_problem(m=R.RL0_BATCH_MAX_M + 1, n=R.RL0_BATCH_MAX_M * 2)
    assert L.rl0_decode_batched(arr, 3, None, None) == -1
    assert b"RL0_BATCH_MAX_M" in L.rl0_last_error()
    arr[2].y = 0
    arr[1] = _fake_problem()
    assert L.rl0_decode_batched(arr, 3, None, None) == -1
    assert b"instance 2" in L.rl0_last_error()


def test_adaptive_k_is_refused_where_it_does_not_apply():
    # the branch needs the analytic posteriors and a whole decode: a learned decode, one
    # step from a caller's state and the batched kernel refuse it before any device work
    L = R.lib()
    p = R.params_default(1024, 256, 7, 25, 0.01)
    p.adaptive_k = 1
    R.compute_constants(p, 1024, 256, 7)          # accepted on its own
    p.posterior, p.mlp = 1, 4096
    with pytest.raises(R.Rl0Error) as e:
        R.compute_constants(p, 1024, 256, 7)
    assert e.value.code == -1 and "analytic" in str(e.value)
    p.posterior, p.mlp = 0, None
    Lh = ctypes.c_int64(0)
    rc = L.rl0_step(ctypes.c_void_p(4096), 1024, 256, 7, ctypes.c_void_p(8192), ctypes.byref(p), 0,
                    ctypes.c_void_p(16384), ctypes.c_void_p(32768), ctypes.byref(Lh), None, None, None,
                    None, None, None)
    assert rc == -1 and b"whole decodes" in L.rl0_last_error()
    arr = (R.Problem * 2)(_fake_problem(), _fake_problem())
    arr[1].params.adaptive_k = 1
    assert L.rl0_decode_batched(arr, 2, None, None) == -1
    assert b"instance 1" in L.rl0_last_error() and b"adaptive_k" in L.rl0_last_error()


def test_batched_refuses_the_learned_posterior():
    # the batched kernel has only the analytic decision: a learned request is an error,
    # before any device work, rather than an analytic decode
    L = R.lib()
    arr = (R.Problem * 3)(_fake_problem(), _fake_problem(), _fake_problem())
    arr[2].params.posterior, arr[2].params.mlp = 1, 4096
    assert L.rl0_decode_batched(arr, 3, None, None) == -1
    assert b"instance 2" in L.rl0_last_error() and b"posterior" in L.rl0_last_error()


def test_batch_schedule_rejects_bad_fields():
    L = R.lib()
    for bad in ({"block": 128, "per_cu": 1, "cols": [4] * 12}, {"block": 256, "per_cu": 0, "cols": [4] * 12},
                {"block": 256, "per_cu": 9, "cols": [4] * 12}, {"block": 256, "per_cu": 1, "cols": [3] * 12},
                {"block": 256, "per_cu": 1, "cols": [4] * 12, "group": [3] * 12},
                {"block": 256, "per_cu": 1, "cols": [4] * 12, "group": [32] * 12},
                {"block": 256, "per_cu": 1, "cols": [4] * 12, "group": [0] * 12}):
        s = R.BatchSchedule.from_dict(bad)
        assert L.rl0_batch_schedule_set(ctypes.byref(s)) == -1


# ------------------------------------------------------------------ host utilities

def test_validate_host_accepts_good_and_rejects_malformed_columns():
    rng = np.random.Generator(np.random.PCG64(11))
    A = I.draw_columns(rng, 300, 50, 5)
    R.validate_host(A, 50)
    for mut in ("range", "negative", "order", "repeat"):
        bad = A.copy()
        if mut == "range":
            bad[17, 4] = 50
        elif mut == "negative":
            bad[17, 0] = -1
        elif mut == "order":
            bad[17, [1, 2]] = bad[17, [2, 1]]
        else:
            bad[17, 2] = bad[17, 1]
        with pytest.raises(R.Rl0Error) as e:
            R.validate_host(bad, 50)
        assert e.value.code == -2
    with pytest.raises(R.Rl0Error) as e:
        R.validate_host(A, 4)            # d > m
    assert e.value.code == -1


def test_workspace_bytes_grow_with_the_problem_and_reject_bad_sizes():
    small = R.workspace_bytes(1024, 256, 7, 25)
    mid = R.workspace_bytes(2 ** 20, 104857, 7, 10485)
    big = R.workspace_bytes(2 ** 24, 2 ** 21, 8, 2 ** 18)
    assert 0 < small < mid < big
    # at least the residual state (int64 S twice, D, and y) and the packed indices
    assert mid >= 4 * 8 * 104857 + 16 * 2 ** 20
    for args in [(1024, 256, 17, 25), (1024, 256, 7, 256), (1024, 256, 7, 0), (1024, 6, 7, 2), (0, 256, 7, 25)]:
        assert R.workspace_bytes(*args) == 0


def _bf16_rne(x: float) -> int:
    """bf16 bits of a float32 value by the definition: the nearer of the two neighbours
    that keep the top 16 bits, ties to the even one (NaN to a quiet NaN)."""
    import math
    import struct
    u = struct.unpack("<I", struct.pack("<f", x))[0]
    if math.isnan(x):
        return (u >> 16) | 0x40
    lo = u >> 16
    hi = lo + 1
    f = lambda b: struct.unpack("<f", struct.pack("<I", (b << 16) & 0xFFFFFFFF))[0]
    xv = struct.unpack("<f", struct.pack("<I", u))[0]
    dlo, dhi = abs(xv - f(lo)), abs(f(hi) - xv) if hi & 0x7F80 != 0x7F80 or (hi & 0x7F) == 0 else math.inf
    if (hi & 0x7F80) == 0x7F80 and (hi & 0x7F) == 0:
        # the upper neighbour is infinity: halfway is the value 2^128 (1 - 2^-9) in magnitude
        half = 2.0 ** 128 * (1 - 2.0 ** -9)
        return hi if abs(xv) >= half and (abs(xv) > half or (lo & 1)) else lo
    if dlo < dhi:
        return lo
    if dhi < dlo:
        return hi
    return lo if lo % 2 == 0 else hi


def test_mlp_pack_bf16_rounds_to_nearest_even():
    d = 3
    P = R.mlp_num_params(d)
    vals = [1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -8 + 2.0 ** -20, -2.0, 0.0, -0.0,
            float("inf"), float("-inf"), 3.4028234663852886e38, 1e-40, 0.1, -0.333, 65504.0]
    rng = np.random.Generator(np.random.PCG64(3))
    w = np.concatenate([np.array(vals, np.float32), rng.standard_normal(P - len(vals)).astype(np.float32)])
    got = R.mlp_pack_bf16(w, d)
    want = np.array([_bf16_rne(float(v)) for v in w], np.uint16)
    assert np.array_equal(got, want)
    assert got[0] == 0x3F80 and got[1] == 0x3F80 and got[2] == 0x3F82 and got[3] == 0x3F81
    assert got[7] == 0x7F80 and got[9] == 0x7F80      # max float rounds up to infinity
    nan = R.mlp_pack_bf16(np.full(P, np.nan, np.float32), d)
    assert np.all((nan & 0x7F80) == 0x7F80) and np.all((nan & 0x7F) != 0)


def test_mlp_pack_bf16_matches_torch_bfloat16_conversion():
    torch = pytest.importorskip("torch")
    d = 7
    P = R.mlp_num_params(d)
    rng = np.random.Generator(np.random.PCG64(4))
    w = (rng.standard_normal(P) * np.exp(rng.uniform(-20, 20, P))).astype(np.float32)
    got = R.mlp_pack_bf16(w, d)
    ref = torch.from_numpy(w).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(got, ref)


def test_device_checks_only_in_the_checked_library():
    """The normal library has no device index checks (rl0_device_check reports -1 without
    touching the GPU); the checked copy exports the same entry points."""
    import ctypes
    import os
    import subprocess

    line = ctypes.c_int32(7)
    assert R.lib().rl0_device_check(ctypes.byref(line), None) == 0 and line.value == -1
    checked = os.path.join(os.path.dirname(R.LIB_PATH), "librl0_checked.so")
    if not os.path.exists(checked) or os.path.basename(R.LIB_PATH) != "librl0.so":
        pytest.skip("librl0_checked.so is not built")

    def exports(path):
        out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True).stdout
        return {ln.split()[-1] for ln in out.splitlines() if " T rl0_" in ln}

    names = exports(R.LIB_PATH)
    assert "rl0_device_check" in names and exports(checked) == names
