import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(autouse=True)
def _device_index_checks(request):
    """Under RL0_EXPECT_DEVICE_CHECKS=1 (tests/test_gpu_checked.py runs GPU tests that way,
    against librl0_checked.so), every GPU test must end with no failed index check in the
    library's kernels."""
    if os.environ.get("RL0_EXPECT_DEVICE_CHECKS") != "1" or request.node.get_closest_marker("gpu") is None:
        yield
        return
    from paper_1704_09012_amd import rl0 as R

    assert R.device_check() == 0, "a failed device index check before this test"
    yield
    line = R.device_check()
    where = (f"mlp.hip line {line - 200000}" if line >= 200000 else
             f"batched.hip line {line - 100000}" if line >= 100000 else f"kernels.hip line {line}")
    assert line == 0, f"device index check failed at {where}"
