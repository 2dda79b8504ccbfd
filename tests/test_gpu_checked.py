"""The parity, determinism, log, general-law, quantised, adaptive, batched and learned GPU
tests once more, against librl0_checked.so: the library whose loop kernels, batched kernel
and network kernel test every data-dependent index (rows from A_cols and its packed form,
candidate-segment sizes and positions, the sweeps' and the network's queues, H_k's
boundary bucket, change- and key-list slots, columns read back from lists or decoded from
keys, the copy-out) against its range.
They run in a child process that loads the checked library (RL0_LIBRARY) with
RL0_EXPECT_DEVICE_CHECKS=1, under which tests/conftest.py requires rl0_device_check to
report no failed check after each test; the results must also still match the oracle,
since a failed check would have replaced an index.  Skipped where the checked library was
not built."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHECKED = os.path.join(ROOT, "paper_1704_09012_amd", "librl0_checked.so")
FILES = ["test_gpu_parity.py", "test_gpu_determinism.py", "test_gpu_log.py", "test_gpu_general.py",
         "test_gpu_quantised.py", "test_gpu_adaptive.py", "test_gpu_batched.py", "test_gpu_mlp.py"]


@pytest.mark.timeout(900)
def test_gpu_suite_under_device_index_checks():
    if not os.path.exists(CHECKED):
        pytest.skip("librl0_checked.so is not built")
    env = dict(os.environ, RL0_LIBRARY=CHECKED, RL0_EXPECT_DEVICE_CHECKS="1")
    cmd = [sys.executable, "-u", "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "gpu",
           "--timeout", "300", "--timeout-method", "thread", *[os.path.join(ROOT, "tests", f) for f in FILES]]
    print("checked library:", " ".join(cmd), flush=True)
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=880)
    tail = r.stdout[-4000:] + r.stderr[-3000:]
    print(tail, flush=True)
    assert r.returncode == 0, tail
    assert " passed" in r.stdout and "failed" not in r.stdout.splitlines()[-1], tail
