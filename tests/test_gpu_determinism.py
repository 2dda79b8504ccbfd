"""Determinism of the decoder on the GPU, standing in for a race detector.

Each decode runs three times through the C-ABI: twice with the workgroups of the loop
kernels in launch order and once with rl0_params.wg_order = 1, where every workgroup of
the sweep, of H_k's classification kernel and of the row kernel takes the tile of its
mirror in the grid (column chunks, candidate segment, row range, partial-sum slot).  That
changes which CU and which XCD handles which tile and the order in which tiles start and
finish; any result that depended on it (an unordered float reduction, a read that races a
write, a lost update) would show.  The bar is bitwise: x_hat, the loop statistics and the
per-iteration log (all but its wall-clock stamps), on the paths the decoder has: the
continuous and quantised scores, the bitmask in LDS and the large-m path (8-row summary,
dense mode, H_k's classification kernel), adaptive k, Laplace laws, the learned decision,
and single teacher-forced steps with their per-column outputs."""
import numpy as np
import pytest

from oracle import decoder as D
from paper_1704_09012_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_1704_09012_amd.rl0")

LOG_FIELDS = ("l1_trial_fx", "l1_hat_fx", "accepted", "updates", "t", "it")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def instance(n, m, k, d, snr, seed, kind="gaussian"):
    sig = float(np.float32(I.sigma_for_snr(snr, n, m, k, d)))
    inst = I.draw_instance(n, m, k, d, sig, seed, kind=kind, noise_kind=kind)
    y = D.measure(inst.A_cols[inst.support], inst.values, inst.eta, m)
    return dev(inst.A_cols), dev(y), sig


def run(A, y, sig, k, order, **kw):
    x, st = R.decode(A, y, sigma=sig, k=k, log=1, wg_order=order, **kw)
    log = R.last_log()
    torch.cuda.synchronize()
    return x.cpu(), R.stats_subset(st), {f: log[f].copy() for f in LOG_FIELDS}


def assert_same(a, b):
    xa, sa, la = a
    xb, sb, lb = b
    assert torch.equal(xa, xb)
    assert sa == sb
    for f in LOG_FIELDS:
        assert np.array_equal(la[f], lb[f]), f


@pytest.mark.parametrize("n,m,k,d,snr,seed,kw", [
    (1024, 256, 25, 7, 40, 1, {}),
    (50003, 2999, 400, 8, 30, 2, {}),
    (1048576, 104857, 10485, 7, 40, 3, {}),
    (1048576, 104857, 10485, 7, 20, 4, {"variant": 1}),
    (200000, 400003, 40000, 6, 40, 5, {}),
    (65536, 6553, 655, 7, 40, 6, {"adaptive_k": 1}),
    (65536, 6553, 655, 7, 40, 7, {"signal_law": "laplace", "noise_law": "laplace"}),
], ids=["small", "ragged", "headline", "quantised_20db", "large_m", "adaptive", "laplace"])
def test_reversed_workgroup_order_gives_the_same_bits(n, m, k, d, snr, seed, kw):
    kind = "laplace" if kw.get("signal_law") == "laplace" else "gaussian"
    print(f"determinism n={n} m={m} {kw}", flush=True)
    A, y, sig = instance(n, m, k, d, snr, seed, kind)
    first = run(A, y, sig, k, 0, **kw)
    assert len(first[2]["it"]) == first[1]["iterations"] > 0
    assert_same(first, run(A, y, sig, k, 0, **kw))
    assert_same(first, run(A, y, sig, k, 1, **kw))


def test_reversed_order_in_the_learned_decode():
    n, m, d, k = 8192, 2048, 7, 160
    A, y, sig = instance(n, m, k, d, 40, 11)
    w = R.mlp_init(d, 3)
    first = run(A, y, sig, k, 0, mlp=w)
    assert_same(first, run(A, y, sig, k, 1, mlp=w))


@pytest.mark.parametrize("n,m,k,d", [(1048576, 104857, 10485, 7), (200000, 400003, 40000, 6)])
def test_reversed_order_in_teacher_forced_steps(n, m, k, d):
    """Four rl0_step iterations from x_hat = 0 in each order: the per-column outputs
    (updated, omega, x_trial), r_trial, the state after each step and ||r||_1 agree."""
    A, y, sig = instance(n, m, k, d, 40, 21)
    out = []
    for order in (0, 1):
        p = R.params_default(n, m, d, k, sig, wg_order=order)
        x = torch.zeros(n, dtype=torch.float32, device="cuda")
        r = torch.empty(m, dtype=torch.float32, device="cuda")
        L = R.step(A, y, p, 0, x, r, 0, debug=False)["L_hat"]
        trace = []
        for it in range(1, 5):
            g = R.step(A, y, p, it, x, r, L)
            L = g["L_hat"]
            trace.append({key: (v.cpu() if torch.is_tensor(v) else v) for key, v in g.items()})
            trace[-1]["x"] = x.cpu()
            trace[-1]["r"] = r.cpu()
        out.append(trace)
    for a, b in zip(*out):
        assert a.keys() == b.keys()
        for key in a:
            if torch.is_tensor(a[key]):
                assert torch.equal(a[key], b[key]), key
            else:
                assert a[key] == b[key], key


def test_wg_order_is_checked():
    with pytest.raises(R.Rl0Error):
        A, y, sig = instance(1024, 256, 25, 7, 40, 1)
        R.decode(A, y, sigma=sig, k=25, wg_order=2)
