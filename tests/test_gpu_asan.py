"""Host AddressSanitizer over the C ABI: tests/asan_driver.cpp, linked with the
library's sources whose host code is instrumented, walks every entry point (all
flag combinations, graphs, growing buffers, multi-context runs, the learned start
and the error paths) on the GPU and must finish with no ASan report and every call
returning the code its header documents."""

import os
import subprocess

import pytest

from paper_2504_10118_amd.build import ASAN_DRIVER

pytestmark = pytest.mark.gpu


def test_c_abi_under_host_address_sanitizer():
    if not os.path.exists(ASAN_DRIVER):
        pytest.skip("AddressSanitizer driver not built (build(asan_driver=True))")
    env = dict(os.environ)
    # the HIP runtime keeps allocations for the process lifetime; leak checks would
    # report those, so only memory errors are checked
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    res = subprocess.run([ASAN_DRIVER], capture_output=True, text=True, timeout=110, env=env)
    print(res.stdout[-2000:], res.stderr[-4000:], flush=True)
    assert "AddressSanitizer" not in res.stderr
    assert res.returncode == 0
    assert "0 unexpected return codes" in res.stdout
