"""The C ABI used from C++ without Python or torch (tests/c_abi_driver.cpp):
forward, adjoint, both in one pass and an unfused step against the oracle, and
argument errors."""
import os
import subprocess

import pytest

from gpu_util import need_gpu

pytestmark = pytest.mark.gpu

DRIVER = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_build", "c_abi_driver")


def test_c_driver():
    need_gpu()
    if not os.path.exists(DRIVER):
        pytest.fail("tests/_build/c_abi_driver is missing: run __graft_entry__.build() first")
    import build_c_driver
    stamp = open(build_c_driver.STAMP).read() if os.path.exists(build_c_driver.STAMP) else ""
    if stamp != build_c_driver.sources_digest():
        pytest.fail("tests/_build/c_abi_driver was built from other sources: run "
                    "__graft_entry__.build() again")
    r = subprocess.run([DRIVER], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "c_abi_driver: ok" in r.stdout
