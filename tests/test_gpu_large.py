"""The large workload: n = 2^24, m = 2^21, d = 8, k = 2^18, 40 dB (sigma_n = 0.01).

Here the column indices are not packed (8 x 16 bits cannot hold a row of m = 2^21) and the
outer-test bitmask does not fit in LDS: the sweep's other paths run.  The oracle cannot
decode this size in a test's time, so the bar is
  * bitwise equality of the per-column decisions and omegas of the first two iterations
    (teacher-forced from x_hat = 0) on a sample of 300 000 columns, the oracle's sweep
    being evaluated column by column on that sample, and
  * for a full decode, properties that hold at any size: at most k nonzeros; the l1 norm
    of the oracle's fixed-point residual of the returned x_hat equals the reported one;
    recovery within 1e-2; a second decode is identical.
"""
import numpy as np
import pytest

from oracle import decoder as D
from oracle import scores as S
from paper_1704_09012_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_1704_09012_amd.rl0")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def large():
    n, m, d, k = 2 ** 24, 2 ** 21, 8, 2 ** 18
    sig = float(np.float32(I.sigma_for_snr(40, n, m, k, d)))
    print("drawing n=2^24 instance", flush=True)
    inst = I.draw_instance(n, m, k, d, sig, I.seed_for(3, 1, 0))
    supp = inst.support
    # y = A x + eta; only the support contributes to A x
    y = D.measure(inst.A_cols[supp], inst.values, inst.eta, m)
    C = D.make_constants(n, m, d, k, sig)
    return inst, y, C, sig


def test_large_first_iterations_on_sampled_columns(large):
    inst, y, C, sig = large
    n, m, d, k = inst.n, inst.m, inst.d, inst.k
    st0 = D.init_state(y, n)
    rng = np.random.default_rng(5)
    sample = np.unique(np.concatenate([rng.choice(n, 250000, replace=False), inst.support[:50000]]))
    A_t, y_t = dev(inst.A_cols), dev(y)
    params = R.params_default(n, m, d, k, sig)
    for it in (0, 1):
        print("teacher-forced iteration", it, flush=True)
        x_t = torch.zeros(n, dtype=torch.float32, device="cuda")
        r_t = torch.empty(m, dtype=torch.float32, device="cuda")
        out = R.step(A_t, y_t, params, it, x_t, r_t, st0.L_hat)
        ref = D.sweep(inst.A_cols[sample], st0.r_hat, st0.x_hat[sample], S.t_of(it, C.c), C)
        gu = host(out["updated"])[sample].astype(bool)
        go = host(out["omega"])[sample]
        assert np.array_equal(gu, ref.updated)
        assert np.array_equal(go, ref.omega)
        print(f"  sampled updates: {int(ref.updated.sum())}", flush=True)


def test_large_decode_properties(large):
    inst, y, C, sig = large
    n, m, d, k = inst.n, inst.m, inst.d, inst.k
    A_t, y_t = dev(inst.A_cols), dev(y)
    params = R.params_default(n, m, d, k, sig)
    x1, st1 = R.decode(A_t, y_t, params=params)
    x2, st2 = R.decode(A_t, y_t, params=params)
    a, b = host(x1), host(x2)
    print("decode stats", st1, flush=True)
    assert np.array_equal(a, b) and R.stats_subset(st1) == R.stats_subset(st2)
    assert np.count_nonzero(a) <= k
    r = D.residual(inst.A_cols, y, a, m)
    assert D.l1_fixed(r) == st1["l1_final_fx"]
    x = inst.x_dense()
    rel = float(np.linalg.norm(a - x) / np.linalg.norm(x))
    print("rel err", rel, flush=True)
    assert rel < 1e-2
