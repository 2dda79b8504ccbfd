"""The stored oracle results agree with one another (no GPU): the digests of the headline
workload's seeds (c2digests_*; the quantised, Laplace-law and adaptive_k sets c2qdigests_*,
c2ldigests_*, c2adigests_*; the large-m set lmdigests_*) against the whole decodes of the
same instances stored beside them, all written by tests/golden/make_golden.py from the
oracle."""
import hashlib
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
C2 = os.path.join(GOLDEN, "c2digests_n1048576_d7_20seeds.npz")


def digest(support, values) -> str:
    h = hashlib.sha256(np.ascontiguousarray(support, dtype="<i4").tobytes())
    h.update(np.ascontiguousarray(values, dtype="<f4").tobytes())
    return h.hexdigest()


@pytest.mark.skipif(not os.path.exists(C2), reason="digest file not stored")
def test_twenty_seed_digests_match_the_whole_decodes():
    c = np.load(C2)
    assert c["digest"].shape == (3, 20) and list(c["snrs"]) == [20, 40, 60]
    checked = 0
    for si, snr in enumerate(c["snrs"]):
        for i in range(20):
            path = os.path.join(GOLDEN, f"decode_n1048576_d7_snr{int(snr)}_i{i}.npz")
            if not os.path.exists(path):
                continue
            g = np.load(path)
            assert digest(g["support"], g["values"]) == str(c["digest"][si, i]), (snr, i)
            assert int(g["iterations"]) == c["iterations"][si, i] and int(g["accepted"]) == c["accepted"][si, i]
            assert int(g["L_hat"]) == c["L_hat"][si, i] and int(g["updates_total"]) == c["updates_total"][si, i]
            checked += 1
    assert checked == 15
    # the twenty decodes per SNR are distinct instances
    for si in range(3):
        assert len(set(str(x) for x in c["digest"][si])) == 20


@pytest.mark.parametrize("digests,whole", [
    ("c2qdigests_n1048576_d7_20seeds.npz", "decodeq_n1048576_d7_snr{snr}_i0.npz"),
    ("c2ldigests_n1048576_d7_snr40_10seeds.npz", "decodel_n1048576_d7_snr{snr}_laplace_laplace_i0.npz"),
    ("c2adigests_n1048576_d7_10seeds.npz", "decodea_n1048576_d7_snr{snr}_i0.npz"),
    ("lmdigests_n1048576_m524288_d8_snr40_8seeds.npz", "decode_n1048576_m524288_d8_snr{snr}_i0.npz"),
])
def test_variant_digests_match_the_whole_decodes(digests, whole):
    path = os.path.join(GOLDEN, digests)
    if not os.path.exists(path):
        pytest.skip("digest file not stored")
    c = np.load(path)
    checked = 0
    for row, snr in enumerate(c["snrs"]):
        w = os.path.join(GOLDEN, whole.format(snr=int(snr)))
        if not os.path.exists(w):
            continue
        g = np.load(w)
        first = int(c["first_seed"]) if "first_seed" in c else 0
        assert int(g["seed"]) == 10000 * int(c["config"]) + 100 * int(c["snr_index"][row]) + first   # seed i = 0
        assert digest(g["support"], g["values"]) == str(c["digest"][row, 0])
        assert int(g["iterations"]) == c["iterations"][row, 0] and int(g["L_hat"]) == c["L_hat"][row, 0]
        checked += 1
    assert checked == len(c["snrs"])
    assert all(len(set(str(x) for x in c["digest"][r])) == int(c["seeds"]) for r in range(len(c["snrs"])))
