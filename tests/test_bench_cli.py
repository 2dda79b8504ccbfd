"""bench.py's command line on the host: the one-GPU limit is refused before any device work."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_instance_records(tmp_path):
    """The per-instance records (--records): support found, l1 success and throughput from
    a decode's statistics, one JSON object a line."""
    import importlib.util
    import types

    import numpy as np

    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    inst = types.SimpleNamespace(n=8, m=4, k=3, d=2)
    x_true = np.array([0, 1.5, 0, 0, -2.0, 0, 0.5, 0], np.float32)
    x_hat = np.array([0, 1.5, 0, 0.25, -2.0, 0, 0, 0], np.float32)
    st = {"iterations": 5, "accepted": 4, "updates_total": 9, "ms_total": 0.5, "converged": 1}
    r = bench.instance_record("headline", inst, 17, 40, 0.01, st, x_hat, x_true, 0.1, 1000.0)
    assert r["support_found"] == 2 / 3 and r["support_size"] == 3 and r["l1_success"] is True
    assert r["nnz_updates_per_s"] == 2 * 8 * 5 / 0.5e-3 and r["algorithmic_bytes"] == 5 * 1000.0 + 4 * 2 * 8
    path = str(tmp_path / "rec.jsonl")
    bench.write_records(path, [r, dict(r, seed=18)])
    lines = open(path).read().splitlines()
    assert len(lines) == 2 and json.loads(lines[1])["seed"] == 18
